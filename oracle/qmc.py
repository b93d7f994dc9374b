"""Randomly shifted rank-1 lattice rules (section 2.5, eq. rqmc; level form eq. t_kl).

    t_k = {k z / N},   y_k = {t_k + Delta} - 1/2,   k = 0 .. N-1

The integer product k z_j is reduced mod N exactly (Python integers); with N
a power of two, (k z_j mod N) / N is exact in FP64, the shift is one rounded
FP64 add, the fractional part subtracts 1 when the sum reaches 1, and the
final subtraction of 1/2 is one rounded FP64 operation.

Embedded (nested) rules in base 2 (section 2.5 on embedded lattice rules;
section 5's point ordering): the points are enumerated in blocks of powers of
two, each block filling the gaps left by the earlier ones, so that the first
2^m points always form the rank-1 lattice with 2^m points.  Enumerating k by
the base-2 radical inverse does this:

    t_k = {phi_2(k) z},   phi_2(k) = sum_i b_i 2^{-i-1}  for k = sum_i b_i 2^i,

which for N = 2^m and k < N is {a z / N} with a = the m-bit reversal of k.

Shift average and sample variance over R independent shifts: eq. sample_var.
"""

from __future__ import annotations

import math

import numpy as np


def lattice_point(z, N: int, shift, k: int) -> np.ndarray:
    """y_k in [-1/2, 1/2)^s for one index k (0 <= k < N)."""
    if not 0 <= k < N:
        raise ValueError("k out of range")
    s = len(z)
    y = np.empty(s, dtype=np.float64)
    for j in range(s):
        t = float((k * int(z[j])) % N) / float(N)
        u = t + float(shift[j])
        if u >= 1.0:
            u = u - 1.0
        y[j] = u - 0.5
    return y


def lattice_points(z, N: int, shift, ks=None) -> np.ndarray:
    """Rows y_k for k in ``ks`` (default 0..N-1), float64[len(ks), s]."""
    if ks is None:
        ks = range(N)
    return np.array([lattice_point(z, N, shift, int(k)) for k in ks],
                    dtype=np.float64).reshape(-1, len(z))


def radical_inverse_numerator(k: int, m: int) -> int:
    """a with phi_2(k) = a / 2^m, for 0 <= k < 2^m: the binary digits of k
    read in reverse order."""
    if not 0 <= k < (1 << m):
        raise ValueError("k out of range")
    a = 0
    for i in range(m):
        if (k >> i) & 1:
            a += 1 << (m - 1 - i)
    return a


def embedded_point(z, N: int, shift, k: int) -> np.ndarray:
    """y_k of the base-2 embedded rule with N = 2^m points: the lattice point
    of index phi_2(k) N, shifted and centred as in lattice_point."""
    m = N.bit_length() - 1
    if N < 1 or (1 << m) != N:
        raise ValueError("N must be a power of two")
    return lattice_point(z, N, shift, radical_inverse_numerator(k, m))


def embedded_points(z, N: int, shift, count: int) -> np.ndarray:
    """The first ``count`` points of the embedded rule, float64[count, s]."""
    return np.array([embedded_point(z, N, shift, k) for k in range(count)],
                    dtype=np.float64).reshape(-1, len(z))


def qmc_mean(values) -> float:
    """Equal-weight rule (eq. qmc): (1/N) sum_k f(t_k), summed exactly rounded."""
    values = list(values)
    return math.fsum(values) / len(values)


def shift_average(Q_r) -> float:
    """Qhat = (1/R) sum_r Q^(r)."""
    Q_r = list(Q_r)
    return math.fsum(Q_r) / len(Q_r)


def sample_variance(Q_r) -> float:
    """eq. sample_var: sum_r (Qhat - Q^(r))^2 / (R (R - 1)); NaN for R = 1."""
    Q_r = list(Q_r)
    R = len(Q_r)
    if R < 2:
        return float("nan")
    qh = shift_average(Q_r)
    return math.fsum((qh - q) ** 2 for q in Q_r) / (R * (R - 1))
