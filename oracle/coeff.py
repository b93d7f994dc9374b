"""Truncated affine coefficient (Assumption A1, eq. coeff; truncation eq. coeff_s).

    a^s(x, y) = a0 + sum_{j=1}^{s} y_j a_j(x),   a_j(x) = c_j sin(pi k1_j x1) sin(pi k2_j x2)

evaluated at the element centroids: the stiffness matrix needs the
coefficient "at the quadrature points for each element" (cost analysis,
section 4.2); the one-point centroid rule is the reading taken here.  The
truncation is the length of ``y``: components past it are zero.

Problem 2 of the numerical section (family kind "islands") adds a reaction
coefficient b(x, y) of the same affine form, and lets a0, b0 and every term
depend on the region (inside or outside the four islands).  Meshes with h a
multiple of 1/8 align with the islands, so the region of an element is the
region of its centroid.
"""

from __future__ import annotations

import math

import numpy as np

from . import mesh


def basis_at(n: int, fam, s: int) -> np.ndarray:
    """a_j at the centroids of mesh 1/n for j = 1..s, float64[s, 2n^2]."""
    xc, yc = mesh.centroids(n)
    out = np.empty((s, xc.size), dtype=np.float64)
    for j in range(s):
        out[j] = (fam["c"][j] * np.sin(math.pi * fam["k1"][j] * xc)
                  * np.sin(math.pi * fam["k2"][j] * yc))
    return out


def coefficient(n: int, y, fam) -> np.ndarray:
    """a^s at the element centroids of mesh 1/n with s = len(y), float64[2n^2]."""
    y = np.asarray(y, dtype=np.float64)
    s = y.size
    if s > len(fam["c"]):
        raise ValueError("truncation exceeds the family length")
    a = np.full(2 * n * n, float(fam["a0"]), dtype=np.float64)
    if s:
        phi = basis_at(n, fam, s)
        for j in range(s):
            a += y[j] * phi[j]
    return a


def bounds(fam, s: int) -> tuple[float, float]:
    """a_min, a_max over |y_j| <= 1/2 (Assumption A1.3 with |sin| <= 1)."""
    half = 0.5 * float(np.sum(np.abs(np.asarray(fam["c"][:s], dtype=np.float64))))
    return float(fam["a0"]) - half, float(fam["a0"]) + half


def in_islands(x, y) -> np.ndarray:
    """True where (x, y) lies in one of the four islands [1/8, 3/8] or
    [5/8, 7/8] in each coordinate (closed squares)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)

    def in_band(t):
        return ((t >= 0.125) & (t <= 0.375)) | ((t >= 0.625) & (t <= 0.875))

    return in_band(x) & in_band(y)


def islands_coefficients(n: int, y, fam) -> tuple[np.ndarray, np.ndarray]:
    """(a, b) of Problem 2 at the element centroids of mesh 1/n, s = len(y)."""
    y = np.asarray(y, dtype=np.float64)
    s = y.size
    if s > len(fam["ca"]):
        raise ValueError("truncation exceeds the family length")
    xc, yc = mesh.centroids(n)
    inside = in_islands(xc, yc)
    a = np.where(inside, fam["a0_in"], fam["a0_out"]).astype(np.float64)
    b = np.where(inside, fam["b0_in"], fam["b0_out"]).astype(np.float64)
    for j in range(s):
        shape = np.sin(math.pi * fam["k1"][j] * xc) * np.sin(math.pi * fam["k2"][j] * yc)
        mask = inside if fam["region"][j] == 1 else ~inside
        a += y[j] * fam["ca"][j] * shape * mask
        b += y[j] * fam["cb"][j] * shape * mask
    return a, b

