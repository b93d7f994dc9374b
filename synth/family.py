"""Coefficient families  a(x, y) = a0 + sum_j y_j c_j sin(pi k1_j x1) sin(pi k2_j x2).

The affine form is Assumption A1 (eq. coeff) truncated as in the section on
stochastic dimension truncation.  A family is handed to both implementations
as a table ``(a0, c[s], k1[s], k2[s])``; each evaluates the sines itself.

* ``coeff_family``: the benchmark family, c_j = j^-decay with (k1, k2) the
  j-th pair of positive integers ordered by k1^2 + k2^2, ties by k1.
* ``problem1_family``: Problem 1 of the numerical section, c_j = j^-p,
  k1 = j, k2 = j + 1, with a0 = 1 for p >= 2 and pi/sqrt(2) otherwise.
* ``islands_family``: Problem 2 of the numerical section (four islands),
  which adds a reaction coefficient b(x, y) and makes every term live on
  one region only; see its docstring.
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


# Problem 2: the islands D_f = four squares [1/8, 3/8] or [5/8, 7/8] in each
# coordinate; the background values inside and outside them.
ISLAND_SQUARES = ((0.125, 0.375), (0.625, 0.875))
SIGMA_A_IN, SIGMA_A_OUT = 0.01, 0.011
SIGMA_B_IN, SIGMA_B_OUT = 2.0, 0.3


def islands_family(s: int, pa: float, pa_out: float, pb: float, pb_out: float):
    """Problem 2 of the numerical section as a table.

    a(x, y) = a0(x) + sum_j y_j a_j(x),  b(x, y) = b0(x) + sum_j y_j b_j(x),
    a0 / b0 piecewise constant (inside / outside the islands); term j (1-based)
    lives inside the islands for odd j (k = (j + 1) / 2, decays pa, pb) and
    outside them for even j (k = j / 2, decays pa_out, pb_out), with the shape
    sin(8 k pi x1) sin(8 (k + 1) pi x2) scaled by the region's background value
    times k^-decay.  A background value whose decay is below 2 is multiplied
    by pi / sqrt(2) (as for Problem 1).

    Keys: kind, a0_in, a0_out, b0_in, b0_out, ca[s], cb[s], k1[s], k2[s] (the
    sine frequencies 8k, 8(k + 1)), region[s] (1: islands, 2: outside)."""
    boost = math.pi / math.sqrt(2.0)
    a_in = SIGMA_A_IN * (boost if pa < 2.0 else 1.0)
    a_out = SIGMA_A_OUT * (boost if pa_out < 2.0 else 1.0)
    b_in = SIGMA_B_IN * (boost if pb < 2.0 else 1.0)
    b_out = SIGMA_B_OUT * (boost if pb_out < 2.0 else 1.0)
    ca = np.empty(s)
    cb = np.empty(s)
    k1 = np.empty(s, dtype=np.int32)
    k2 = np.empty(s, dtype=np.int32)
    region = np.empty(s, dtype=np.int32)
    for j in range(1, s + 1):
        if j % 2:
            k = (j + 1) // 2
            ca[j - 1] = SIGMA_A_IN * k ** (-pa)
            cb[j - 1] = SIGMA_B_IN * k ** (-pb)
            region[j - 1] = 1
        else:
            k = j // 2
            ca[j - 1] = SIGMA_A_OUT * k ** (-pa_out)
            cb[j - 1] = SIGMA_B_OUT * k ** (-pb_out)
            region[j - 1] = 2
        k1[j - 1] = 8 * k
        k2[j - 1] = 8 * (k + 1)
    return {"kind": "islands", "a0_in": a_in, "a0_out": a_out, "b0_in": b_in, "b0_out": b_out,
            "ca": ca, "cb": cb, "k1": k1, "k2": k2, "region": region}

