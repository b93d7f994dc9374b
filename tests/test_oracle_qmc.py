"""Pins for the oracle's lattice points and estimator (eq. rqmc, eq. t_kl,
eq. sample_var, eq. mlqmc_R, eq. ml-var, Algorithm 2).

* a rank-1 lattice with odd z_j and N a power of two projects onto each
  coordinate as a permutation of {0, 1/N, ...};
* the character property: the rule integrates e^{2 pi i h.x} to 0 unless
  h.z = 0 mod N, when the shifted rule returns e^{2 pi i h.Delta};
* hand-computed shift averages and sample variances;
* the telescoping sum (eq. tele_sum) is exact sample by sample when all
  levels share points and use direct eigensolves;
* a degenerate two-grid level whose two meshes coincide gives Y = 0 at
  every point (the coarse pair and point are shared by both terms).
"""

import cmath
import math

import numpy as np
import pytest

from oracle import mlqmc, qmc, twogrid
from synth import LevelSpec, lattice_vector, problem1_family, shifts_for


@pytest.mark.parametrize("N,s", [(64, 8), (256, 16)])
def test_projections_are_permutations(N, s):
    z = lattice_vector(N, s)
    assert all(int(v) % 2 == 1 for v in z)
    pts = qmc.lattice_points(z, N, np.zeros(s))
    for j in range(s):
        assert sorted((pts[:, j] + 0.5).tolist()) == [k / N for k in range(N)]
    shift = shifts_for(99, 0, 1, s)[0]
    sp = qmc.lattice_points(z, N, shift)
    assert np.all(sp >= -0.5) and np.all(sp < 0.5)
    for j in range(s):
        want = sorted(((np.arange(N) / N + shift[j]) % 1.0).tolist())
        assert np.max(np.abs(np.sort(sp[:, j] + 0.5) - want)) < 1e-15


def test_character_property():
    N, s = 128, 16
    z = lattice_vector(N, s)
    shift = shifts_for(98, 0, 1, s)[0]
    pts = qmc.lattice_points(z, N, shift) + 0.5
    # frequency outside the dual lattice: integrated to zero
    h = np.zeros(s, dtype=np.int64)
    h[0], h[1] = 3, 1
    assert (h @ z) % N != 0
    val = sum(cmath.exp(2j * math.pi * float(h @ p)) for p in pts) / N
    assert abs(val) < 1e-12
    # dual-lattice frequency h = (-z_2 mod N, 1, 0, ...): z_1 = 1 so h.z = 0 mod N
    h = np.zeros(s, dtype=np.int64)
    h[0], h[1] = (-int(z[1])) % N, 1
    assert (h @ z) % N == 0
    val = sum(cmath.exp(2j * math.pi * float(h @ p)) for p in pts) / N
    assert abs(val - cmath.exp(2j * math.pi * float(h @ shift))) < 1e-10


def test_lattice_point_arithmetic_boundary_cases():
    z = [1, 3]
    # k z / N + shift crossing 1 wraps; k = 0 gives the shift itself
    y = qmc.lattice_point(z, 4, [0.75, 0.0], 1)     # t = (1/4, 3/4)
    assert y.tolist() == [0.0 - 0.5, 0.75 - 0.5]
    y0 = qmc.lattice_point(z, 4, [0.25, 0.5], 0)
    assert y0.tolist() == [-0.25, 0.0]


def test_sample_variance_hand_computed():
    # Q = (1, 2, 3, 4): mean 5/2, squared deviations 9/4+1/4+1/4+9/4 = 5,
    # divided by R (R-1) = 12
    assert qmc.shift_average([1.0, 2.0, 3.0, 4.0]) == 2.5
    assert abs(qmc.sample_variance([1.0, 2.0, 3.0, 4.0]) - 5.0 / 12.0) < 1e-16
    assert qmc.sample_variance([7.0, 7.0, 7.0]) == 0.0
    assert math.isnan(qmc.sample_variance([1.0]))
    est = mlqmc.combine([[1.0, 2.0, 3.0, 4.0], [0.5, 0.5, 0.5, 0.5]])
    assert est.Q_ml == 3.0 and abs(est.V_ml - 5.0 / 12.0) < 1e-16


def test_constant_integrand_and_identical_shifts():
    assert qmc.qmc_mean([3.25] * 16) == 3.25
    est = mlqmc.combine([[1.5] * 8])
    assert est.V[0] == 0.0 and est.Q_ml == 1.5


def test_telescoping_identity_direct_levels():
    fam = problem1_family(8, 2.0)
    N, s = 8, 8
    z = lattice_vector(64, 8)
    shift = shifts_for(97, 0, 1, s)[0]
    levels = [LevelSpec(4, 4, 0, 0, 0, 0, N), LevelSpec(8, 6, 0, 0, 4, 4, N),
              LevelSpec(16, 8, 0, 0, 8, 6, N)]
    pts = qmc.lattice_points(z, N, shift)
    for y in pts[:4]:
        tot = sum(mlqmc.level_value(lv, y, fam).Y for lv in levels)
        lam_L = twogrid.direct(16, 8, y, fam)[0]
        assert abs(tot - lam_L) < 1e-12 * lam_L


def test_degenerate_two_grid_level_is_zero():
    fam = problem1_family(8, 2.0)
    lv = LevelSpec(16, 8, 4, 4, 16, 8, 4)
    y = np.array([0.1, -0.3, 0.2, 0.05, 0.4, -0.45, 0.0, 0.3])
    v = mlqmc.level_value(lv, y, fam)
    assert v.Y == 0.0 and v.lam == v.lam_prev


def test_estimate_small_two_level():
    fam = problem1_family(8, 2.0)
    levels = [LevelSpec(4, 4, 0, 0, 0, 0, 4), LevelSpec(8, 8, 4, 4, 4, 4, 4)]
    zs = [lattice_vector(64, 4)[:4], lattice_vector(64, 8)]
    shifts = [shifts_for(96, 0, 2, 4), shifts_for(96, 1, 2, 8)]
    est = mlqmc.estimate(levels, zs, [4, 4], shifts, fam)
    assert est.Q_lr.shape == (2, 2)
    assert abs(est.Q_ml - est.Qhat.sum()) < 1e-14
    # level 0 values are direct eigenvalues of the coarse mesh, level 1 are
    # small corrections (variance reduction across levels)
    assert est.Qhat[0] > 10 and abs(est.Qhat[1]) < 0.2 * est.Qhat[0]
    assert est.V[1] < est.V[0]
