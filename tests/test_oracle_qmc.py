"""Pins for the oracle's lattice points and estimator (eq. rqmc, eq. t_kl,
eq. sample_var, eq. mlqmc_R, eq. ml-var, Algorithm 2).

* a rank-1 lattice with odd z_j and N a power of two projects onto each
  coordinate as a permutation of {0, 1/N, ...};
* the character property: the rule integrates e^{2 pi i h.x} to 0 unless
  h.z = 0 mod N, when the shifted rule returns e^{2 pi i h.Delta};
* hand-computed shift averages and sample variances;
* the estimator's assembly (Algorithm 2): on three levels with different z,
  N, truncations and shifts, each Q_l^(r) is the mean of the level values at
  exactly that cell's hand-listed points, so another level's z, N or shift
  fails it;
* the telescoping sum (eq. tele_sum) is exact sample by sample when all
  levels share points and use direct eigensolves;
* a degenerate two-grid level whose two meshes coincide gives Y = 0 at
  every point (the coarse pair and point are shared by both terms);
* embedded rules: hand-computed radical inverses and points, every prefix of
  2^m points is the plain rank-1 lattice with 2^m points, and each block of
  the enumeration fills exactly the gaps of the ones before;
* the nested estimator (shared shifts, nested points, H_l = h_0): the level
  terms telescope to the finest two-grid value point by point, its values
  are those of Algorithm 2's level evaluation at the same points, and the
  variance of the per-shift totals is at most the number of levels times
  sum_l V_l (Cauchy-Schwarz: the factor the paper states for shared shifts);
* extensible nested estimates: a point of the embedded rule does not depend on
  the rule's size (or on z being reduced modulo it), and level sums over
  disjoint blocks of points add up to the one-shot sums, N_l Q_l^(r).
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


# Hand-listed points of a three-level, two-shift estimate whose levels differ
# in z, N, s and shifts, and no level's points are a prefix of another's.
# y = {k z / N + Delta} - 1/2 worked out by hand per (level, shift, k), in
# units of 1/8.  Level 1's previous term differs from its coarse problem only
# through y_2, which is nonzero at all its points (y_2 = 0 would make that
# update exactly singular).
_EST_LEVELS = [LevelSpec(4, 2, 0, 0, 0, 0, 8),      # direct, h = 1/4, s = 2
               LevelSpec(8, 3, 4, 1, 4, 2, 4),      # two-grid 1/4 -> 1/8, prev on 1/4
               LevelSpec(16, 4, 4, 2, 8, 3, 2)]     # two-grid 1/4 -> 1/16, prev on 1/8
_EST_Z = [[1, 3], [3, 1, 1], [1, 1, 1, 1]]
_EST_SHIFTS = [[[1 / 8, 1 / 2], [5 / 8, 1 / 4]],
               [[0.0, 5 / 8, 1 / 2], [1 / 4, 1 / 8, 7 / 8]],
               [[1 / 4, 1 / 2, 3 / 4, 0.0], [1 / 8, 3 / 8, 5 / 8, 7 / 8]]]
_EST_POINTS = [
    # level 0, N = 8, z = (1, 3): t = (k/8, (3k mod 8)/8)
    [[(-3, 0), (-2, 3), (-1, -2), (0, 1), (1, -4), (2, -1), (3, 2), (-4, -3)],   # Delta (1/8, 1/2)
     [(1, -2), (2, 1), (3, -4), (-4, -1), (-3, 2), (-2, -3), (-1, 0), (0, 3)]],  # Delta (5/8, 1/4)
    # level 1, N = 4, z = (3, 1, 1): t = ((3k mod 4)/4, k/4, k/4)
    [[(-4, 1, 0), (2, 3, 2), (0, -3, -4), (-2, -1, -2)],        # Delta (0, 5/8, 1/2)
     [(-2, -3, 3), (-4, -1, -3), (2, 1, -1), (0, 3, 1)]],       # Delta (1/4, 1/8, 7/8)
    # level 2, N = 2, z = (1, 1, 1, 1): t = (k/2, k/2, k/2, k/2)
    [[(-2, 0, 2, -4), (2, -4, -2, 0)],                          # Delta (1/4, 1/2, 3/4, 0)
     [(-3, -1, 1, 3), (1, 3, -3, -1)]],                         # Delta (1/8, 3/8, 5/8, 7/8)
]


def test_estimate_assembles_each_level_and_shift():
    """Algorithm 2 / eq. mlqmc_R / eq. sample_var: Q_l^(r) is the mean of
    level_value over exactly the N_l points of (level l, shift r), Qhat_l the
    shift average, V_l = sum_r (Qhat_l - Q_l^(r))^2 / (R (R - 1)).  Taking
    another level's z, N, truncation or shift changes the point set (the
    hand-listed sets below are pairwise different) and fails the comparison."""
    fam = problem1_family(8, 2.0)
    Ns = [lv.N for lv in _EST_LEVELS]
    zs = [np.array(z, dtype=np.int64) for z in _EST_Z]
    shifts = [np.array(sh, dtype=np.float64) for sh in _EST_SHIFTS]
    est = mlqmc.estimate(_EST_LEVELS, zs, Ns, shifts, fam)
    # the point sets are pairwise distinct across (level, shift)
    sets = [frozenset(tuple(p) for p in _EST_POINTS[l][r]) for l in range(3) for r in range(2)]
    assert len(set(sets)) == 6
    Q = np.empty((3, 2))
    for l, lv in enumerate(_EST_LEVELS):
        for r in range(2):
            pts = _EST_POINTS[l][r]
            assert len(pts) == lv.N
            # the oracle's own point generator agrees with the hand list
            got = qmc.lattice_points(zs[l], lv.N, shifts[l][r])
            assert got.tolist() == [[v / 8 for v in p] for p in pts]
            ys = [mlqmc.level_value(lv, np.array(p, dtype=np.float64) / 8, fam).Y for p in pts]
            Q[l, r] = math.fsum(ys) / lv.N
            # ARPACK starts from a random vector: equal to round-off, not bitwise
            assert abs(est.Q_lr[l, r] - Q[l, r]) <= 1e-12 * abs(Q[l, r]) + 1e-14
        # the shift average and sample variance of the oracle's own Q_l^(r)
        q0, q1 = est.Q_lr[l]
        qh = (q0 + q1) / 2
        assert est.Qhat[l] == qh
        assert est.V[l] == ((qh - q0) ** 2 + (qh - q1) ** 2) / 2
        assert abs(est.V[l] - (Q[l, 0] - Q[l, 1]) ** 2 / 4) <= 1e-9 * est.V[l] + 1e-28
    assert est.Q_ml == math.fsum(est.Qhat)
    assert est.V_ml == math.fsum(est.V)
    # every cell carries its own value: a swap of points between cells shows
    assert len(set(Q.ravel().tolist())) == 6


def test_radical_inverse_hand_values():
    assert [qmc.radical_inverse_numerator(k, 3) for k in range(8)] == [0, 4, 2, 6, 1, 5, 3, 7]
    assert qmc.radical_inverse_numerator(1, 10) == 512
    assert qmc.radical_inverse_numerator(6, 4) == 6       # 0110 -> 0110
    assert qmc.radical_inverse_numerator(11, 5) == 26     # 01011 -> 11010
    with pytest.raises(ValueError):
        qmc.radical_inverse_numerator(8, 3)


def test_embedded_points_hand_computed():
    z, N, sh = [1, 3], 8, np.zeros(2)
    got = qmc.embedded_points(z, N, sh, 4)
    want = np.array([[-0.5, -0.5], [0.0, 0.0], [-0.25, 0.25], [0.25, -0.25]])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("N,s", [(64, 8), (256, 16)])
def test_embedded_prefixes_are_lattices_and_blocks_fill_gaps(N, s):
    z = lattice_vector(N, s)
    sh = shifts_for(98, 0, 1, s)[0]
    pts = [tuple(p) for p in qmc.embedded_points(z, N, sh, N)]
    assert len(set(pts)) == N
    m_max = N.bit_length() - 1
    prev = set()
    for m in range(m_max + 1):
        Nm = 1 << m
        plain = {tuple(p) for p in qmc.lattice_points(z, Nm, sh)}
        assert set(pts[:Nm]) == plain
        if m:
            assert set(pts[Nm // 2:Nm]) == plain - prev
        prev = plain


def _nested_levels(N):
    # level 0 direct on 1/4, levels 1-2 two-grid from (1/4, s_0)
    return [LevelSpec(4, 2, 0, 0, 0, 0, N[0]), LevelSpec(8, 3, 4, 2, 4, 2, N[1]),
            LevelSpec(16, 5, 4, 2, 8, 3, N[2])]


def test_nested_levels_telescope_to_finest_two_grid_value():
    fam = problem1_family(5, 2.0)
    N = [4, 4, 4]
    levels = _nested_levels(N)
    z = lattice_vector(64, 8)[:5]
    sh = shifts_for(99, 0, 1, 5)[0]
    lams = mlqmc.nested_values(levels, z, N, sh, fam)
    pts = qmc.embedded_points(z, N[0], sh, N[0])
    for k in range(N[0]):
        tot = sum(lams[l][k] - (lams[l - 1][k] if l else 0.0) for l in range(3))
        lam_L = twogrid.two_grid(16, 5, 4, 2, pts[k], fam)[0]
        assert abs(tot - lam_L) < 1e-12 * lam_L
        lam0 = twogrid.direct(4, 2, pts[k], fam)[0]
        assert abs(lams[0][k] - lam0) < 1e-13 * lam0


def test_nested_values_equal_algorithm2_values_at_the_same_points():
    fam = problem1_family(5, 2.0)
    N = [8, 4, 2]
    levels = _nested_levels(N)
    z = lattice_vector(64, 8)[:5]
    sh = shifts_for(99, 1, 1, 5)[0]
    lams = mlqmc.nested_values(levels, z, N, sh, fam)
    pts = qmc.embedded_points(z, N[0], sh, N[0])
    for l in range(1, 3):
        assert len(lams[l]) == N[l]
        for k in range(N[l]):
            v = mlqmc.level_value(levels[l], pts[k], fam)
            assert abs(v.lam - lams[l][k]) < 1e-12 * v.lam
            assert abs(v.lam_prev - lams[l - 1][k]) < 1e-12 * v.lam


def test_nested_estimate_variance_and_identical_shifts():
    fam = problem1_family(5, 2.0)
    N = [8, 4, 2]
    levels = _nested_levels(N)
    z = lattice_vector(64, 8)[:5]
    shifts = shifts_for(99, 2, 3, 5)
    est = mlqmc.estimate_nested(levels, z, N, shifts, fam)
    assert est.Q_lr.shape == (3, 3)
    assert abs(est.Q_ml - est.Qhat.sum()) < 1e-13 * abs(est.Q_ml)
    assert est.V_ml <= 3 * est.V.sum() * (1 + 1e-12)
    totals = est.Q_lr.sum(axis=0)
    assert abs(est.V_ml - np.var(totals, ddof=1) / 3) < 1e-12 * np.var(totals)
    same = mlqmc.estimate_nested(levels, z, N, np.repeat(shifts[:1], 2, axis=0), fam)
    # equal up to the eigensolver's last-bit differences between calls
    assert same.V_ml < 1e-26 and np.all(same.V < 1e-26)
    assert np.allclose(same.Q_lr[:, 0], est.Q_lr[:, 0], rtol=1e-13, atol=0)


def test_nested_level_list_checks():
    ok = _nested_levels([4, 4, 2])
    mlqmc.check_nested(ok, [4, 4, 2])
    with pytest.raises(ValueError):
        mlqmc.check_nested(ok, [4, 8, 2])
    bad = list(ok)
    bad[2] = LevelSpec(16, 5, 8, 3, 8, 3, 2)   # coarse mesh is not level 0's
    with pytest.raises(ValueError):
        mlqmc.check_nested(bad, [4, 4, 2])
    bad = list(ok)
    bad[2] = LevelSpec(16, 5, 4, 2, 4, 2, 2)   # previous term not on level 1's mesh
    with pytest.raises(ValueError):
        mlqmc.check_nested(bad, [4, 4, 2])


def test_nested_estimate_telescopes_per_shift():
    # with equal N the per-shift total is the plain QMC mean of the finest
    # two-grid value over the same points
    fam = problem1_family(5, 2.0)
    N = [4, 4, 4]
    levels = _nested_levels(N)
    z = lattice_vector(64, 8)[:5]
    shifts = shifts_for(99, 3, 2, 5)
    est = mlqmc.estimate_nested(levels, z, N, shifts, fam)
    for r in range(2):
        pts = qmc.embedded_points(z, 4, shifts[r], 4)
        want = np.mean([twogrid.two_grid(16, 5, 4, 2, y, fam)[0] for y in pts])
        assert abs(est.Q_lr[:, r].sum() - want) < 1e-12 * want


def test_nested_estimate_level_means_use_the_leading_points():
    # Q_l^(r) is Algorithm 2's level mean over the first N_l points of the
    # embedded rule (each Y_l evaluated afresh there)
    fam = problem1_family(5, 2.0)
    N = [8, 4, 2]
    levels = _nested_levels(N)
    z = lattice_vector(64, 8)[:5]
    shifts = shifts_for(99, 4, 2, 5)
    est = mlqmc.estimate_nested(levels, z, N, shifts, fam)
    for r in range(2):
        pts = qmc.embedded_points(z, 8, shifts[r], 8)
        for l in range(3):
            want = np.mean([mlqmc.level_value(levels[l], pts[k], fam).Y for k in range(N[l])])
            assert abs(est.Q_lr[l, r] - want) < 1e-12 * max(abs(want), 1.0)


def test_embedded_points_do_not_depend_on_the_rule_size():
    # the property that makes a nested estimate extensible: point k of the
    # embedded rule is the same for every rule of more than k points, with z
    # reduced modulo the rule size or not
    z = lattice_vector(1024, 8)
    sh = shifts_for(41, 0, 1, 8)[0]
    for N in (8, 32, 128):
        for k in range(N):
            a = qmc.embedded_point(z, N, sh, k)
            assert np.array_equal(a, qmc.embedded_point(z % N, N, sh, k))
            assert np.array_equal(a, qmc.embedded_point(z, 1024, sh, k))


def test_nested_block_sums_add_up_to_the_estimate():
    # sums over [0, N/2) and [N/2, N) per level give the one-shot level sums,
    # and those are N_l Q_l^(r) of the nested estimator; a level whose block
    # is empty adds 0
    N = [8, 4, 4]
    levels = _nested_levels(N)
    z = lattice_vector(64, 8)
    sh = shifts_for(42, 0, 1, 8)
    fam = problem1_family(8, 2.0)
    whole = mlqmc.nested_level_sums(levels, z, [0, 0, 0], N, sh[0], fam)
    half = [n // 2 for n in N]
    lo = mlqmc.nested_level_sums(levels, z, [0, 0, 0], half, sh[0], fam)
    hi = mlqmc.nested_level_sums(levels, z, half, N, sh[0], fam)
    # 1e-13: the direct eigensolve (ARPACK, random start) is reproducible to
    # about 1e-15 relative per eigenvalue, not bit for bit
    for l in range(3):
        assert abs(lo[l] + hi[l] - whole[l]) <= 1e-13 * max(1.0, abs(whole[l]))
    est = mlqmc.estimate_nested(levels, z, N, sh, fam)
    for l in range(3):
        assert abs(whole[l] / N[l] - est.Q_lr[l, 0]) <= 1e-13 * max(1.0, abs(est.Q_lr[l, 0]))
    assert mlqmc.nested_level_sums(levels, z, N, N, sh[0], fam) == [0.0, 0.0, 0.0]


def test_every_workload_reads_stored_generating_vectors():
    # the bench and the tests must not fall back to a component-by-component
    # search at run time: every (N, s) a workload uses has a stored vector
    # (or a longer one with the same N, whose prefix it is)
    import os
    from synth import CONFIGS
    store = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "synth", "lattice")
    have = {}
    for name in os.listdir(store):
        if name.startswith("cbc_N") and name.endswith(".txt"):
            N = int(name[5:name.index("_s")])
            s = int(name[name.index("_s") + 2:-4])
            have[N] = max(have.get(N, 0), s)
    for w in CONFIGS.values():
        pairs = ([(max(lv.N for lv in w.levels), w.s_max)] if w.nested else
                 [(lv.N, lv.s_fine) for lv in w.levels])
        for N, s in pairs:
            assert have.get(N, 0) >= s, (w.name, N, s)
