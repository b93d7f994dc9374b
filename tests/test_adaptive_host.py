"""The library's adaptive decision (mlqmc_adaptive_decide: host arithmetic,
no device) against the oracle's rule (oracle/adaptive.py, pinned by hand in
test_oracle_adaptive.py), on the hand-worked cases and on random inputs."""

import numpy as np
import pytest

import paper_2103_03407_amd as m
from oracle import adaptive as A


def _both(Qhat, V, N, cost, eps, alpha, L, max_levels, N_max):
    lib = m.mlqmc_adaptive_decide(Qhat[:L], V[:L], N[:L], cost[:L], eps, alpha, max_levels, N_max)
    ora = A.decide(Qhat, V, N, cost, eps, alpha, L, max_levels, N_max)
    return lib, ora


def test_codes_match_the_oracle():
    assert (m.ADAPT_DONE, m.ADAPT_DOUBLE, m.ADAPT_ADD, m.ADAPT_BUDGET, m.ADAPT_LEVELS) == \
        (A.DONE, A.DOUBLE, A.ADD, A.BUDGET, A.LEVELS)


@pytest.mark.parametrize("case", [
    ([1.0, 0.1, 0.01], [0.1, 0.5, 0.2], [16, 8, 4], 0.1, 2.0, 3, 64),
    ([1.0, 0.1, 0.01], [0.16, 0.32, 0.0], [16, 8, 4], 0.1, 2.0, 3, 32),
    ([1.0, 0.1, 0.01], [0.16, 0.32, 0.0], [16, 8, 4], 0.1, 2.0, 3, 31),
    ([1.0, 0.5, 0.3], [0.002, 0.001, 0.001], [16, 8, 4], 0.1, 2.0, 4, 64),
    ([1.0, 0.5, 0.3], [0.002, 0.001, 0.001], [16, 8, 4], 0.1, 2.0, 3, 64),
    ([1.0, 0.5, 0.06], [0.002, 0.001, 0.001], [16, 8, 4], 0.1, 1.0, 4, 64),
])
def test_hand_cases(case):
    Qhat, V, N, eps, alpha, max_levels, N_max = case
    cost = [1.0, 4.0, 16.0]
    lib, ora = _both(Qhat, V, N, cost, eps, alpha, len(Qhat), max_levels, N_max)
    assert lib == ora


def test_random_inputs():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        L = int(rng.integers(1, 6))
        max_levels = L + int(rng.integers(0, 3))
        Qhat = rng.normal(0, 1, L) * 10.0 ** rng.uniform(-4, 1, L)
        V = 10.0 ** rng.uniform(-9, -1, L)
        N = np.sort(2 ** rng.integers(2, 12, L))[::-1].astype(np.int64)
        cost = np.array([(4 ** (l + 2)) * (2 ** l + 1) for l in range(L)], dtype=np.float64)
        eps = 10.0 ** rng.uniform(-4, -0.5)
        alpha = float(rng.choice([1.0, 2.0, 1.5]))
        N_max = int(2 ** rng.integers(8, 14))
        lib, ora = _both(Qhat, V, N, cost, eps, alpha, L, max_levels, N_max)
        assert lib == ora, (Qhat, V, N, eps, alpha, L, max_levels, N_max)


def test_invalid_arguments():
    with pytest.raises(m.MlqmcError):
        m.mlqmc_adaptive_decide([1.0], [0.1], [8], [1.0], -1.0, 2.0, 1, 64)
    with pytest.raises(m.MlqmcError):
        m.mlqmc_adaptive_decide([1.0, 2.0], [0.1, 0.1], [8, 8], [1.0, 1.0], 0.1, 2.0, 1, 64)
