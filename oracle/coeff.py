"""Truncated affine coefficient (Assumption A1, eq. coeff; truncation eq. coeff_s).

    a^s(x, y) = a0 + sum_{j=1}^{s} y_j a_j(x),   a_j(x) = c_j sin(pi k1_j x1) sin(pi k2_j x2)

evaluated at the element centroids: the stiffness matrix needs the
coefficient "at the quadrature points for each element" (cost analysis,
section 4.2); the one-point centroid rule is the reading taken here.  The
truncation is the length of ``y``: components past it are zero.
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
