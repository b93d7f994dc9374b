"""Pins for the oracle's eigenfunction functional G(u) = integral of the
L2-normalised, sign-fixed eigenfunction (introduction: E[G(u)] by the same
telescoping sum).

* the element-by-element integral integrates every hat function to its
  exact value h^2 (so every P1 function exactly);
* for a = 1 the eigenfunction is 2 sin(pi x) sin(pi y), whose integral is
  8 / pi^2: the FE values converge to it, by about 2^4 per halving of h;
* G does not depend on the scale or sign of the vector, nor on a constant
  factor in the coefficient (the eigenfunction does not change);
* the two-grid G approaches the direct fine-mesh G as H is refined;
* over direct levels sharing a point, the level differences of G telescope
  to the finest level's G.
"""

import math

import numpy as np
import pytest

from oracle import coeff, eig, fem, functional, mlqmc, twogrid
from synth import LevelSpec, problem1_family


@pytest.mark.parametrize("n", [2, 4, 7])
def test_integral_of_each_hat_is_h_squared(n):
    m = (n - 1) ** 2
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        assert abs(functional.integral(n, e) - 1.0 / n ** 2) < 1e-15


def test_constant_coefficient_converges_to_8_over_pi2():
    exact = 8.0 / math.pi ** 2
    errs = []
    for n in (8, 16, 32, 64):
        A = fem.stiffness(n, np.ones(2 * n * n))
        M = fem.mass(n)
        _, u = eig.smallest_eigenpair(A, M)
        errs.append(abs(functional.G(n, u, M) - exact))
    for a, b in zip(errs, errs[1:]):
        assert 10.0 < a / b < 20.0
    assert errs[-1] < 2e-7


def test_scale_sign_and_coefficient_scaling():
    fam = problem1_family(6, 2.0)
    y = np.array([0.3, -0.2, 0.45, -0.4, 0.1, 0.0])
    n = 16
    aK = coeff.coefficient(n, y, fam)
    M = fem.mass(n)
    _, u = eig.smallest_eigenpair(fem.stiffness(n, aK), M)
    _, u3 = eig.smallest_eigenpair(fem.stiffness(n, 3.0 * aK), M)
    g = functional.G(n, u, M)
    assert abs(functional.G(n, -2.5 * u, M) - g) < 1e-15
    assert abs(functional.G(n, u3, M) - g) < 1e-12
    assert 0.5 < g < 1.0


def test_two_grid_G_approaches_direct_G():
    fam = problem1_family(6, 2.0)
    y = np.array([0.3, -0.2, 0.45, -0.4, 0.1, 0.0])
    h = 32
    M = fem.mass(h)
    _, u = twogrid.direct(h, 6, y, fam)
    g = functional.G(h, u, M)
    errs = []
    for H in (4, 8, 16):
        lam_H, u_H = twogrid.coarse_pair(H, 6, y, fam)
        _, w = twogrid.two_grid_update(h, 6, y, fam, lam_H, u_H, H)
        errs.append(abs(functional.G(h, w, M) - g))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_G_telescopes_over_direct_levels():
    fam = problem1_family(8, 2.0)
    levels = [LevelSpec(4, 4, 0, 0, 0, 0, 1), LevelSpec(8, 6, 0, 0, 4, 4, 1),
              LevelSpec(16, 8, 0, 0, 8, 6, 1)]
    y = np.array([0.1, -0.3, 0.2, 0.05, 0.4, -0.45, 0.0, 0.3])
    vals = [mlqmc.level_value(lv, y, fam) for lv in levels]
    tot = sum(v.G - v.G_prev for v in vals)
    _, u = twogrid.direct(16, 8, y, fam)
    assert abs(tot - functional.G(16, u, fem.mass(16))) < 1e-13
    assert vals[0].G_prev == 0.0
