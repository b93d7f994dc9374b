"""Pins for the oracle's adaptive choice of N_l and L (oracle/adaptive.py):
the decision function and the cascade on hand-made inputs, and a whole
adaptive run worked out by hand on a synthetic sampler with known level
means and variances; then the rule on the real nested evaluation, which must
end inside its own tolerance."""

import math

import numpy as np
import pytest

from oracle import adaptive as A
from synth import LevelSpec, lattice_vector, problem1_family, shifts_for

LEVELS = [LevelSpec(8, 8, 0, 0, 0, 0, 0), LevelSpec(16, 16, 8, 8, 8, 8, 0),
          LevelSpec(32, 32, 8, 8, 16, 16, 0), LevelSpec(64, 64, 8, 8, 32, 32, 0)]


def test_level_cost():
    # s h^-2 + h^-gamma
    assert A.level_cost(8, 8) == 8 * 64 + 64
    assert A.level_cost(16, 16, gamma=3.0) == 16 * 256 + 4096


def test_doubled_cascades_to_coarser_levels():
    assert A.doubled([64, 32, 16], 2) == [64, 32, 32]
    assert A.doubled([32, 32, 16], 1) == [64, 64, 16]
    assert A.doubled([16, 16, 16], 2) == [32, 32, 32]
    assert A.doubled([8, 4], 0) == [16, 4]


def test_decide_cases():
    cost = [1.0, 4.0, 16.0]
    N = [16, 8, 4]
    # variance too large: the largest V_l / (N_l C_l) is level 1 (0.5/32 > 1/16/... )
    V = [0.1, 0.5, 0.2]             # scores 0.1/16, 0.5/32, 0.2/64
    assert A.decide([1.0, 0.1, 0.01], V, N, cost, eps=0.1, alpha=2.0, n_levels=3, max_levels=3,
                    N_max=64) == (A.DOUBLE, 1)
    # a tie goes to the first level
    V = [0.16, 0.32, 0.0]           # scores 0.01 and 0.01
    assert A.decide([1.0, 0.1, 0.01], V, N, cost, 0.1, 2.0, 3, 3, 64) == (A.DOUBLE, 0)
    # doubling up to N_max is allowed, beyond it is the budget's end
    assert A.decide([1.0, 0.1, 0.01], V, N, cost, 0.1, 2.0, 3, 3, 32) == (A.DOUBLE, 0)
    assert A.decide([1.0, 0.1, 0.01], V, N, cost, 0.1, 2.0, 3, 3, 31) == (A.BUDGET, 0)
    # variance fine (sum 0.004 <= 0.005), bias |0.3|/3 = 0.1 > 0.1/sqrt(2): add a level
    V = [0.002, 0.001, 0.001]
    assert A.decide([1.0, 0.5, 0.3], V, N, cost, 0.1, 2.0, 3, 4, 64) == (A.ADD, 3)
    # ... unless no level is left
    assert A.decide([1.0, 0.5, 0.3], V, N, cost, 0.1, 2.0, 3, 3, 64) == (A.LEVELS, 2)
    # alpha = 1: bias |0.06| / 1 = 0.06 <= 0.0707: done
    assert A.decide([1.0, 0.5, 0.06], V, N, cost, 0.1, 1.0, 3, 4, 64) == (A.DONE, -1)
    # a single level has no bias estimate
    assert A.decide([1.0], [0.001], [16], [1.0], 0.1, 2.0, 1, 1, 64) == (A.DONE, -1)


def _synthetic(m, b):
    """Sums of Y_l over [N_done, N) for point values m_l, plus (-1)^r b_l at
    point 0: Q_l^(r) = m_l + (-1)^r b_l / N_l, so Qhat_l = m_l and (R = 2)
    V_l = (b_l / N_l)^2."""
    def fn(lv, Nd, N, r):
        out = []
        for l in range(len(lv)):
            s = (N[l] - Nd[l]) * m[l]
            if Nd[l] == 0 and N[l] > 0:
                s += (-1) ** r * b[l]
            out.append(s)
        return out
    return fn


def test_hand_worked_run():
    # costs C = 576, 4352, 33792, 266240; eps = 0.05: variance target 0.00125,
    # bias target 0.0354; V_l = b_l^2 / N_l^2 with b^2 = 64, 4, 0.25, 0.015625,
    # score_l = b_l^2 / (N_l^3 C_l).
    #  1 N=[8,8]      V=[1, .0625]           scores 2.2e-4, 1.8e-6      -> double 0
    #  2 N=[16,8]     V=[.25, .0625]         2.7e-5, 1.8e-6             -> double 0
    #  3 N=[32,8]     V=[.0625, .0625]       3.4e-6, 1.8e-6             -> double 0
    #  4 N=[64,8]     V=[.0156, .0625]       4.2e-7, 1.8e-6             -> double 1
    #  5 N=[64,16]    V=[.0156, .0156]       4.2e-7, 2.2e-7             -> double 0
    #  6 N=[128,16]   V=[.0039, .0156]       5.3e-8, 2.2e-7             -> double 1
    #  7 N=[128,32]   V=[.0039, .0039]       5.3e-8, 2.8e-8             -> double 0
    #  8 N=[256,32]   V=[.00098, .0039]      6.6e-9, 2.8e-8             -> double 1
    #  9 N=[256,64]   V=[.00098, .00098]     6.6e-9, 3.5e-9             -> double 0
    # 10 N=[512,64]   sum V = .00122 <= .00125; bias .4/3 = .133         -> add level 2
    # 11 N=[512,64,8] V2 = .0039, scores 8.3e-10, 3.5e-9, 1.4e-8         -> double 2
    # 12 N=[512,64,16] sum .0022; scores 8.3e-10, 3.5e-9, 1.8e-9         -> double 1
    # 13 N=[512,128,16] sum .00146; scores 8.3e-10, 4.4e-10, 1.8e-9      -> double 2
    # 14 N=[512,128,32] sum .00073; bias .1/3 = .0333 <= .0354           -> done
    m = [10.0, 0.4, 0.1, 0.025]
    b = [8.0, 2.0, 0.5, 0.125]
    res = A.estimate_adaptive(LEVELS, None, np.zeros((2, 1)), None, eps=0.05, N_init=8,
                              sums_fn=_synthetic(m, b))
    D, AD = A.DOUBLE, A.ADD
    assert res.trace == [(D, 0), (D, 0), (D, 0), (D, 1), (D, 0), (D, 1), (D, 0), (D, 1), (D, 0),
                         (AD, 2), (D, 2), (D, 1), (D, 2), (A.DONE, -1)]
    assert res.N == [512, 128, 32] and res.n_levels == 3 and res.converged
    assert res.Q_ml == 10.5
    assert res.V_ml == 64 / 512 ** 2 + 4 / 128 ** 2 + 0.25 / 32 ** 2
    # the same run with three levels at most stops unconverged only if the bias
    # needs a fourth: here it does not; with eps = 0.04 it does
    r3 = A.estimate_adaptive(LEVELS[:3], None, np.zeros((2, 1)), None, eps=0.04, N_init=8,
                             sums_fn=_synthetic(m, b))
    assert r3.trace[-1] == (A.LEVELS, 2) and not r3.converged
    rb = A.estimate_adaptive(LEVELS, None, np.zeros((2, 1)), None, eps=0.05, N_init=8,
                             N_max=128, sums_fn=_synthetic(m, b))
    assert rb.trace[-1] == (A.BUDGET, 0) and not rb.converged


def test_rule_on_the_nested_evaluation():
    # the real level values (Problem 1, p = 2; corrections fall by about 4 per
    # level, as h^2): the run ends with both its targets met
    fam = problem1_family(64, 2.0)
    z = lattice_vector(1 << 14, 64)
    sh = shifts_for(41, 0, 4, 64)
    levels = [LevelSpec(4, 4, 0, 0, 0, 0, 0), LevelSpec(8, 8, 4, 4, 4, 4, 0),
              LevelSpec(16, 16, 4, 4, 8, 8, 0), LevelSpec(32, 32, 4, 4, 16, 16, 0)]
    eps = 0.15
    res = A.estimate_adaptive(levels, z, sh, fam, eps=eps, N_init=4)
    assert res.converged and res.n_levels == 4
    assert res.trace == [(A.ADD, 2), (A.ADD, 3), (A.DONE, -1)]
    assert math.fsum(res.V) <= eps * eps / 2
    assert abs(res.Qhat[-1]) / 3.0 <= eps / math.sqrt(2.0) < abs(res.Qhat[-2]) / 3.0
    # a tighter target doubles the coarse levels first, then runs out of levels
    res = A.estimate_adaptive(levels, z, sh, fam, eps=0.003, N_init=4)
    assert not res.converged and res.trace[-1] == (A.LEVELS, 3)
    assert res.N[0] > res.N[-1] and all(res.N[l] >= res.N[l + 1] for l in range(3))
