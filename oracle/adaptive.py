"""Adaptive choice of the points per level N_l and of the number of levels L
for the nested estimator (shared shifts, one embedded rule; end of
section 4.3).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The paper chooses N_l and L with a greedy adaptive MLQMC algorithm that it
cites but does not state (section 4.2 and the numerical section's set-up).
This is the library's own rule, assembled from what the paper does state:

* the mean-square error of the estimator is its variance plus its squared
  bias; the rule asks for sum_l V_l <= eps^2 / 2 (V_l of eq. sample_var,
  eq. ml-var) and an estimated bias <= eps / sqrt(2);
* the cost of one sample on level l is C_l = s_l h_l^-2 + h_l^-gamma
  (section 4.2, d = 2);
* greedy step: while the variance is too large, double N_l on the level with
  the largest V_l / (N_l C_l) (first such level on ties): doubling costs
  N_l C_l and removes at least half of V_l for a rule converging at least
  like N^-1/2.  Nested rules need N_0 >= N_1 >= ..., so every coarser level
  is raised to at least the doubled N;
* bias: the level differences decay like h_l^alpha (alpha = 2 for the
  eigenvalue, section 2.3), and with h halving per level the remaining bias
  is about |Qhat_{L-1}| / (2^alpha - 1) for the finest level in use; while
  it exceeds eps / sqrt(2) a level is added with N_init points.

Sums are taken left to right in plain floating point (as the library's host
code does), so that both sides take the same decisions from the same values.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import mlqmc, qmc

DONE, DOUBLE, ADD, BUDGET, LEVELS = 0, 1, 2, 3, 4


def level_cost(n: int, s: int, gamma: float = 2.0) -> float:
    """C_l = s_l h_l^-2 + h_l^-gamma for h_l = 1/n (section 4.2, d = 2)."""
    return s * float(n) ** 2 + float(n) ** gamma


def decide(Qhat, V, N, cost, eps: float, alpha: float, n_levels: int, max_levels: int,
           N_max: int):
    """One decision of the rule: (DONE, -1), (DOUBLE, l), (ADD, n_levels),
    (BUDGET, l) if doubling level l would exceed N_max, or (LEVELS, n_levels - 1)
    if the bias needs a level beyond max_levels."""
    var = 0.0
    for l in range(n_levels):
        var += V[l]
    if var > eps * eps / 2.0:
        best, score = 0, -1.0
        for l in range(n_levels):
            sc = V[l] / (N[l] * cost[l])
            if sc > score:
                best, score = l, sc
        if 2 * N[best] > N_max:
            return BUDGET, best
        return DOUBLE, best
    if n_levels >= 2:
        bias = abs(Qhat[n_levels - 1]) / (2.0 ** alpha - 1.0)
        if bias > eps / math.sqrt(2.0):
            if n_levels >= max_levels:
                return LEVELS, n_levels - 1
            return ADD, n_levels
    return DONE, -1


def doubled(N, level: int):
    """N after doubling `level`, with every coarser level raised to at least
    its new value (nested rules: N non-increasing in l)."""
    out = list(N)
    out[level] *= 2
    for l in range(level - 1, -1, -1):
        out[l] = max(out[l], out[l + 1])
    return out


@dataclass
class Adaptive:
    n_levels: int
    N: list
    Q_lr: np.ndarray      # [n_levels, R]
    Qhat: np.ndarray
    V: np.ndarray
    Q_ml: float
    V_ml: float           # sum_l V_l
    converged: bool
    trace: list = field(default_factory=list)   # (action, level) per decision


def estimate_adaptive(levels, z, shifts, fam, eps: float, alpha: float = 2.0,
                      gamma: float = 2.0, N_init: int = 8, N_max: int = 1 << 20,
                      sums_fn=None) -> Adaptive:
    """The rule over the nested hierarchy `levels` (LevelSpec list, the most
    levels allowed; N fields unused), R = len(shifts) shifts and the embedded
    rule with vector z.  sums_fn(levels_in_use, N_done, N, r) returns the sums
    of Y_l over the points [N_done[l], N[l]) of shift r (default: the
    oracle's nested evaluation, oracle.mlqmc.nested_level_sums); the
    per-(level, shift) sums accumulate, and Q_l^(r) = sum / N_l."""
    shifts = np.asarray(shifts, dtype=np.float64)
    R = shifts.shape[0]
    max_levels = len(levels)
    if sums_fn is None:
        def sums_fn(lv, Nd, Nn, r):
            return mlqmc.nested_level_sums(lv, z, Nd, Nn, shifts[r], fam)
    cost = [level_cost(lv.n_fine, lv.s_fine, gamma) for lv in levels]
    L = min(2, max_levels)
    N = [N_init] * L
    N_done = [0] * L
    sums = np.zeros((max_levels, R))
    trace = []
    while True:
        for r in range(R):
            add = sums_fn(list(levels[:L]), N_done, N, r)
            for l in range(L):
                sums[l, r] += add[l]
        N_done = list(N)
        Q_lr = np.array([[sums[l, r] / N[l] for r in range(R)] for l in range(L)])
        Qhat = np.array([qmc.shift_average(Q_lr[l]) for l in range(L)])
        V = np.array([qmc.sample_variance(Q_lr[l]) for l in range(L)])
        act, lev = decide(Qhat, V, N, cost, eps, alpha, L, max_levels, N_max)
        trace.append((act, lev))
        if act == DOUBLE:
            N = doubled(N, lev)
        elif act == ADD:
            L += 1
            N = N + [N_init]
            N_done = N_done + [0]
        else:
            return Adaptive(L, N, Q_lr, Qhat, V, math.fsum(Qhat), math.fsum(V), act == DONE,
                            trace)
