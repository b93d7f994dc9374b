"""P1 finite element matrices (section 2.3, eq. fe-evp; c = 1).

    A_ab = sum_K a_K |K| grad(phi_a) . grad(phi_b)      (stiffness, y-dependent)
    R_ab = sum_K b_K |K|/12 (1 + delta_ab)              (reaction, Problem 2)
    M_ab = sum_K |K|/12 (1 + delta_ab)                  (mass, exact for c = 1)

The reaction term uses the element value of b (centroid rule) with the exact
P1 element mass matrix; for Problem 1 (b = 0) the operator is A alone.

assembled element by element into CSR; the homogeneous Dirichlet condition
removes the boundary nodes.  ``full=True`` keeps every node (used by tests
that integrate functions which do not vanish on the boundary).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import mesh


def _element_geometry(n: int):
    x, y = mesh.node_coords(n)
    el = mesh.elements(n)
    xv, yv = x[el], y[el]                      # [E, 3]
    # signed twice-area and barycentric gradients grad(lambda_a) = (dy, dx) / (2|K|)
    det = ((xv[:, 1] - xv[:, 0]) * (yv[:, 2] - yv[:, 0])
           - (xv[:, 2] - xv[:, 0]) * (yv[:, 1] - yv[:, 0]))
    gx = np.empty_like(xv)
    gy = np.empty_like(yv)
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        gx[:, a] = (yv[:, b] - yv[:, c]) / det
        gy[:, a] = (xv[:, c] - xv[:, b]) / det
    area = 0.5 * np.abs(det)
    return el, area, gx, gy


def _restrict(mat: sp.spmatrix, n: int, full: bool) -> sp.csr_matrix:
    mat = mat.tocsr()
    if full:
        return mat
    keep = np.flatnonzero(mesh.interior_map(n) >= 0)
    return mat[keep][:, keep].tocsr()


def stiffness(n: int, aK, full: bool = False) -> sp.csr_matrix:
    """A(a) on mesh 1/n for per-element coefficient values aK[2n^2]."""
    aK = np.asarray(aK, dtype=np.float64)
    el, area, gx, gy = _element_geometry(n)
    if aK.shape != (el.shape[0],):
        raise ValueError("aK must have one value per element")
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(el[:, a])
            cols.append(el[:, b])
            vals.append(aK * area * (gx[:, a] * gx[:, b] + gy[:, a] * gy[:, b]))
    N = (n + 1) * (n + 1)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return _restrict(A, n, full)


def mass(n: int, full: bool = False) -> sp.csr_matrix:
    """Consistent P1 mass matrix M on mesh 1/n (y-independent, built once per level)."""
    el, area, _, _ = _element_geometry(n)
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(el[:, a])
            cols.append(el[:, b])
            vals.append(area / 12.0 * (2.0 if a == b else 1.0))
    N = (n + 1) * (n + 1)
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return _restrict(M, n, full)


def reaction(n: int, bK, full: bool = False) -> sp.csr_matrix:
    """R(b) on mesh 1/n for per-element reaction values bK[2n^2]."""
    bK = np.asarray(bK, dtype=np.float64)
    el, area, _, _ = _element_geometry(n)
    if bK.shape != (el.shape[0],):
        raise ValueError("bK must have one value per element")
    rows, cols, vals = [], [], []
    for a in range(3):
        for b in range(3):
            rows.append(el[:, a])
            cols.append(el[:, b])
            vals.append(bK * area / 12.0 * (2.0 if a == b else 1.0))
    N = (n + 1) * (n + 1)
    R = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return _restrict(R, n, full)

