"""Smallest eigenpair of the generalised matrix EVP  A u = lambda M u  (section 2.4).

All eigenvalues are strictly positive (section 2.2), so the smallest one is
the eigenvalue nearest 0: ARPACK's shift-invert Lanczos with sigma = 0 (a
library routine over SuperLU) returns it to round-off.  The eigenvector is
normalised to ||u||_M = 1 (eq. fe-evp) and its sign fixed by sum(M u) > 0
(the introduction asks for a consistent sign; the first eigenfunction has one
sign, so its integral is nonzero).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _normalise(u: np.ndarray, M) -> np.ndarray:
    Mu = M @ u
    u = u / np.sqrt(u @ Mu)
    if np.sum(M @ u) < 0:
        u = -u
    return u


def smallest_eigenpair(A: sp.spmatrix, M: sp.spmatrix) -> tuple[float, np.ndarray]:
    """(lambda_1, u_1) with ||u_1||_M = 1 and sum(M u_1) > 0."""
    nd = A.shape[0]
    if nd < 3:
        w, V = sla.eigh(A.toarray(), M.toarray())
        lam, u = float(w[0]), V[:, 0].copy()
    else:
        w, V = spla.eigsh(A.tocsc(), k=1, M=M.tocsc(), sigma=0.0, which="LM", tol=0.0)
        lam, u = float(w[0]), V[:, 0].copy()
    u = _normalise(u, M)
    # report the Rayleigh quotient of the returned vector (equal to lam to round-off)
    lam = float(u @ (A @ u)) / float(u @ (M @ u))
    return lam, u


def dense_spectrum(A: sp.spmatrix, M: sp.spmatrix) -> np.ndarray:
    """All generalised eigenvalues by dense LAPACK (brute force, tiny meshes only)."""
    return sla.eigh(A.toarray(), M.toarray(), eigvals_only=True)
