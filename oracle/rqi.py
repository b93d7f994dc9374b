"""Rayleigh-quotient iteration for the smallest eigenpair, with its iteration
count (the RQ algorithm of section 4.3 and of the numerical section's set-up).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The paper solves each coarse eigenproblem by RQ iteration started either from
a fixed vector or from the eigenvector of a nearby QMC point (section 4.3:
v_0 = u(t'), sigma_0 = the Rayleigh quotient of v_0 for the current point),
and stops at an absolute tolerance of 5e-8 (section 5).  One iteration, with
exact (SuperLU) solves:

    x = (A - sigma_k M)^{-1} M v_k,   v_{k+1} = x / ||x||_M,
    sigma_{k+1} = v_{k+1}^T A v_{k+1},

stopping when |sigma_{k+1} - sigma_k| <= tol.  The fixed start is the nodal
interpolant of sin(pi x1) sin(pi x2), the first eigenfunction for a constant
coefficient.  The count is what the paper reports (3 iterations from the
fixed start in almost all cases, 2 from the previous point's eigenvector, for
Problem 1); the converged eigenvalue is the oracle's eig.smallest_eigenpair's.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from . import fem, twogrid


def sine_start(n: int) -> np.ndarray:
    """sin(pi x1) sin(pi x2) at the interior nodes of mesh 1/n (x fastest)."""
    t = np.sin(math.pi * np.arange(1, n) / n)
    return np.outer(t, t).ravel()


def rq_iteration(A, M, v0, tol: float, max_iter: int = 50):
    """RQ iteration from v0 with the absolute stopping tolerance tol.  Returns
    (sigma, v, iterations, [sigma_0, sigma_1, ...]); v is M-normalised."""
    v = np.asarray(v0, dtype=np.float64)
    v = v / math.sqrt(float(v @ (M @ v)))
    sigma = float(v @ (A @ v))
    hist = [sigma]
    for it in range(1, max_iter + 1):
        try:
            x = spla.splu((A - sigma * M).tocsc()).solve(M @ v)
        except RuntimeError:
            # an exactly singular shift: sigma is an eigenvalue to working
            # precision and v its eigenvector; the iteration has nothing left
            # to change (|sigma_{k+1} - sigma_k| = 0)
            return sigma, v, it, hist + [sigma]
        v = x / math.sqrt(float(x @ (M @ x)))
        new = float(v @ (A @ v))
        hist.append(new)
        done = abs(new - sigma) <= tol
        sigma = new
        if done:
            return sigma, v, it, hist
    return sigma, v, max_iter, hist


def chain_counts(n: int, S: int, points, fam, tol: float = 5e-8):
    """For consecutive points y_0, y_1, ... (rows of `points`, first S
    coordinates used) on mesh 1/n: the RQ iterations from the fixed start
    (cold) and from the previous point's converged eigenvector (nearby; the
    first point starts cold), and the converged eigenvalues of both runs."""
    M = fem.mass(n)
    cold, warm, lam_c, lam_w = [], [], [], []
    prev = None
    for y in points:
        A = twogrid.operator(n, S, y, fam)
        sc, _, ic, _ = rq_iteration(A, M, sine_start(n), tol)
        sw, vw, iw, _ = rq_iteration(A, M, sine_start(n) if prev is None else prev, tol)
        prev = vw
        cold.append(ic)
        warm.append(iw)
        lam_c.append(sc)
        lam_w.append(sw)
    return np.array(cold), np.array(warm), np.array(lam_c), np.array(lam_w)
