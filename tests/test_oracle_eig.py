"""Pins for the oracle's direct eigensolve (sections 2.2-2.4).

* constant coefficient: lambda_h decreases to 2 pi^2 from above at O(h^2)
  (eq. fe_lam_u and the convergence-from-above statement of section 2.3);
* brute force: dense LAPACK on tiny meshes;
* linearity of A in a: homogeneity and the min-max bracket / monotonicity;
* the eigen-residual and normalisation (eq. fe-evp).
"""

import math

import numpy as np
import pytest

from oracle import coeff, eig, fem, twogrid
from synth import coeff_family, problem1_family

TWO_PI2 = 2.0 * math.pi ** 2


def _lam_const(n):
    return eig.smallest_eigenpair(fem.stiffness(n, np.ones(2 * n * n)), fem.mass(n))[0]


def test_constant_coefficient_converges_from_above_at_h2():
    lams = [_lam_const(n) for n in (8, 16, 32, 64)]
    errs = [l - TWO_PI2 for l in lams]
    assert all(e > 0 for e in errs)
    assert all(a > b for a, b in zip(lams, lams[1:]))
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    assert all(3.8 < r < 4.2 for r in ratios), ratios
    rich = (4 * lams[-1] - lams[-2]) / 3          # Richardson removes the h^2 term
    assert abs(rich - TWO_PI2) < 2e-5 * TWO_PI2


@pytest.mark.parametrize("n", [3, 4, 8, 16])
def test_matches_dense_brute_force(n):
    fam = problem1_family(12, 2.0)
    rng = np.random.default_rng(n)
    y = rng.random(12) - 0.5
    A = fem.stiffness(n, coeff.coefficient(n, y, fam))
    M = fem.mass(n)
    lam, u = eig.smallest_eigenpair(A, M)
    dense = eig.dense_spectrum(A, M)
    assert abs(lam - dense[0]) < 1e-12 * dense[0]
    assert dense[0] > 0


def test_eigenpair_residual_normalisation_sign():
    n = 32
    fam = coeff_family(16)
    y = np.random.default_rng(2).random(16) - 0.5
    A = fem.stiffness(n, coeff.coefficient(n, y, fam))
    M = fem.mass(n)
    lam, u = eig.smallest_eigenpair(A, M)
    r = A @ u - lam * (M @ u)
    assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(A @ u)
    assert abs(u @ (M @ u) - 1.0) < 1e-13
    assert np.sum(M @ u) > 0
    assert np.all(u > -1e-12)      # first eigenvector has one sign (Krein-Rutman)


def test_homogeneity_and_zero_parameter():
    n = 16
    fam = coeff_family(16)
    y = np.random.default_rng(3).random(16) - 0.5
    lam1 = twogrid.direct(n, 16, y, fam)[0]
    fam2 = dict(fam, a0=2 * fam["a0"], c=2 * fam["c"])
    lam2 = twogrid.direct(n, 16, y, fam2)[0]
    assert abs(lam2 - 2 * lam1) < 1e-12 * lam1
    lam0 = twogrid.direct(n, 16, np.zeros(16), fam)[0]
    assert abs(lam0 - fam["a0"] * _lam_const(n)) < 1e-12 * lam0


def test_min_max_bracket_and_monotonicity():
    n = 16
    fam = coeff_family(16)
    base = _lam_const(n)
    rng = np.random.default_rng(4)
    for _ in range(4):
        y = rng.random(16) - 0.5
        a = coeff.coefficient(n, y, fam)
        lam = eig.smallest_eigenpair(fem.stiffness(n, a), fem.mass(n))[0]
        assert a.min() * base <= lam * (1 + 1e-13)
        assert lam <= a.max() * base * (1 + 1e-13)
        bump = a + rng.random(a.size) * 0.1          # pointwise larger coefficient
        lam_b = eig.smallest_eigenpair(fem.stiffness(n, bump), fem.mass(n))[0]
        assert lam_b > lam


def test_truncation_monotone_in_s_is_small():
    # truncation error decays with s; lambda_{h,s} for s=16 vs s=64 differ
    # by a small amount relative to lambda
    fam = coeff_family(64)
    y = np.random.default_rng(6).random(64) - 0.5
    l16 = twogrid.direct(16, 16, y, fam)[0]
    l64 = twogrid.direct(16, 64, y, fam)[0]
    assert abs(l16 - l64) < 2e-2 * l64
