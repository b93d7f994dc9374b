"""Two-grid-truncation method (Algorithm 1; level form eq. 2grid_src_ell and
eq. 2grid_update_ell).

Given y, a coarse mesh H with truncation S and a fine mesh h with truncation s:

1. (lambda_{H,S}, u_{H,S}): smallest eigenpair on the coarse mesh with y_{1:S};
2. solve  (A_h(y_{1:s}) - lambda_{H,S} M_h) w = M_h u_{H,S}  on the fine mesh,
   where u_{H,S} enters as its P1 interpolant at the fine nodes (section 3:
   linear interpolation suffices for piecewise linear elements);
3./4. lambda^h = w^T A_h w / w^T M_h w  (the Rayleigh quotient; the
   normalisation of step 3 does not change it).

The paper's level form writes the truncation of the coarse pair as s_l; it
is read as S_l, as in Algorithm 1.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import coeff, eig, fem


def prolong(u_H: np.ndarray, nH: int, nh: int) -> np.ndarray:
    """Values at the interior fine nodes of the coarse P1 function with
    interior nodal values u_H (zero on the boundary).  nh must be a multiple of nH."""
    if nh % nH:
        raise ValueError("fine mesh must refine the coarse mesh")
    U = np.zeros((nH + 1, nH + 1))                      # U[J, I]
    U[1:nH, 1:nH] = np.asarray(u_H, dtype=np.float64).reshape(nH - 1, nH - 1)
    out = np.empty((nh - 1) * (nh - 1))
    r = nh // nH
    for j in range(1, nh):
        for i in range(1, nh):
            I, J = i // r, j // r                       # coarse square
            xi, eta = (i - I * r) / r, (j - J * r) / r  # local coordinates in [0,1)
            I1, J1 = min(I + 1, nH), min(J + 1, nH)
            u00, u10, u11, u01 = U[J, I], U[J, I1], U[J1, I1], U[J1, I]
            if eta <= xi:   # lower triangle (I,J),(I+1,J),(I+1,J+1)
                v = u00 + xi * (u10 - u00) + eta * (u11 - u10)
            else:           # upper triangle (I,J),(I+1,J+1),(I,J+1)
                v = u00 + eta * (u01 - u00) + xi * (u11 - u01)
            out[(j - 1) * (nh - 1) + (i - 1)] = v
    return out


def operator(n: int, s: int, y, fam):
    """The y-dependent operator on mesh 1/n with y_{1:s}: the stiffness matrix,
    plus the reaction matrix for Problem 2 families."""
    yy = np.asarray(y)[:s]
    if fam.get("kind") == "islands":
        aK, bK = coeff.islands_coefficients(n, yy, fam)
        return fem.stiffness(n, aK) + fem.reaction(n, bK)
    return fem.stiffness(n, coeff.coefficient(n, yy, fam))


def coarse_pair(nH: int, S: int, y, fam):
    """Step 1: (lambda_{H,S}(y), u_{H,S}(y)) on mesh 1/nH with y_{1:S}."""
    A = operator(nH, S, y, fam)
    M = fem.mass(nH)
    return eig.smallest_eigenpair(A, M)


def two_grid_update(nh: int, s: int, y, fam, lam_H: float, u_H: np.ndarray, nH: int):
    """Steps 2-4 on mesh 1/nh with y_{1:s}, from a coarse pair on mesh 1/nH.
    Returns (lambda^h, w)."""
    A = operator(nh, s, y, fam)
    M = fem.mass(nh)
    v = prolong(u_H, nH, nh)
    lu = spla.splu((A - lam_H * M).tocsc())
    w = lu.solve(M @ v)
    lam = float(w @ (A @ w)) / float(w @ (M @ w))
    return lam, w


def two_grid(nh: int, s: int, nH: int, S: int, y, fam):
    """Algorithm 1 for one parameter value: returns (lambda^h, lambda_H, u_H)."""
    lam_H, u_H = coarse_pair(nH, S, y, fam)
    lam, _ = two_grid_update(nh, s, y, fam, lam_H, u_H, nH)
    return lam, lam_H, u_H


def direct(nh: int, s: int, y, fam):
    """lambda_{h,s}(y): the FE eigenvalue by a direct eigensolve (section 2.4)."""
    A = operator(nh, s, y, fam)
    M = fem.mass(nh)
    return eig.smallest_eigenpair(A, M)
