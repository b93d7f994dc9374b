"""Coefficient families  a(x, y) = a0 + sum_j y_j c_j sin(pi k1_j x1) sin(pi k2_j x2).

The affine form is Assumption A1 (eq. coeff) truncated as in the section on
stochastic dimension truncation.  A family is handed to both implementations
as a table ``(a0, c[s], k1[s], k2[s])``; each evaluates the sines itself.

* ``coeff_family``: the benchmark family, c_j = j^-decay with (k1, k2) the
  j-th pair of positive integers ordered by k1^2 + k2^2, ties by k1.
* ``problem1_family``: Problem 1 of the numerical section, c_j = j^-p,
  k1 = j, k2 = j + 1, with a0 = 1 for p >= 2 and pi/sqrt(2) otherwise.
"""

from __future__ import annotations

import math

import numpy as np


def pair_ordering(s: int) -> tuple[np.ndarray, np.ndarray]:
    """First ``s`` pairs (k1, k2), k1, k2 >= 1, sorted by (k1^2 + k2^2, k1)."""
    if s < 0:
        raise ValueError("s must be >= 0")
    kmax = 1
    while kmax * kmax < 2 * s + 4:
        kmax += 1
    while True:
        pairs = [(k1 * k1 + k2 * k2, k1, k2)
                 for k1 in range(1, kmax + 1) for k2 in range(1, kmax + 1)]
        pairs.sort()
        # every pair with norm^2 <= kmax^2 is present once kmax bounds both legs
        complete = [p for p in pairs if p[0] <= kmax * kmax]
        if len(complete) >= s:
            sel = complete[:s]
            return (np.array([p[1] for p in sel], dtype=np.int32),
                    np.array([p[2] for p in sel], dtype=np.int32))
        kmax *= 2


def coeff_family(s: int, decay: float = 2.5, a0: float = 1.0):
    """Benchmark family: returns dict(a0, c, k1, k2) of length ``s``."""
    k1, k2 = pair_ordering(s)
    j = np.arange(1, s + 1, dtype=np.float64)
    return {"a0": float(a0), "c": j ** (-float(decay)), "k1": k1, "k2": k2}


def problem1_family(s: int, p: float):
    """Problem 1 of the numerical section: a_j = j^-p sin(j pi x1) sin((j+1) pi x2)."""
    j = np.arange(1, s + 1, dtype=np.int32)
    a0 = 1.0 if p >= 2.0 else math.pi / math.sqrt(2.0)
    return {"a0": a0, "c": j.astype(np.float64) ** (-float(p)),
            "k1": j.copy(), "k2": (j + 1).astype(np.int32)}
