"""A linear functional of the eigenfunction (introduction: E_y[G(u)] by the
same telescoping sum; section 4's cost remark: G is applied to the u_l
computed with lambda_l).

G(u) = integral over D of u, applied to the FE eigenfunction approximation
normalised in L2 (u^T M u = 1) with its sign chosen consistently: the first
eigenfunction does not change sign, so the sign that makes the integral
positive is the consistent one.  For a P1 function the integral over one
triangle is its area times the mean of its three vertex values, summed here
element by element (boundary values are zero).

Test infrastructure: only tests and the measurement script's CPU baseline
use this module.
"""

from __future__ import annotations

import numpy as np

from . import mesh


def integral(n: int, u_int: np.ndarray) -> float:
    """Integral over D of the P1 function with interior values u_int."""
    imap = mesh.interior_map(n)
    full = np.zeros((n + 1) * (n + 1))
    full[imap >= 0] = np.asarray(u_int, dtype=np.float64)[imap[imap >= 0]]
    area = 0.5 / (n * n)
    total = 0.0
    for tri in mesh.elements(n):
        total += area * (full[tri[0]] + full[tri[1]] + full[tri[2]]) / 3.0
    return total


def G(n: int, w: np.ndarray, M) -> float:
    """G(u) for u = +-w / ||w||_M, the sign making the integral positive."""
    w = np.asarray(w, dtype=np.float64)
    return abs(integral(n, w)) / float(np.sqrt(w @ (M @ w)))
