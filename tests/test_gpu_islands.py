"""GPU parity for Problem 2 of the numerical section (four interior islands:
region-wise diffusion a and reaction b), against the FP64 CPU oracle,
through the C ABI (mlqmc_create_islands).

The family runs on meshes 1/8 .. 1/32, every array of a solve in LDS, and as
the fine or previous mesh of a two-grid level on 1/64 .. 1/1024 (the batched
stencil kernels with the reaction term; 1/64, 1/128 and 1/256 here), in FP64
or mixed precision.  Tolerances as for Problem 1: eigenvalues relative 1e-10
per sample (mixed 1e-8), G(u) relative 1e-9 (mixed 1e-7), estimator sums from
the per-sample bound.  Both parameter
sets of the paper's complexity figure are covered: decays (4/3, 2, 4/3, 2)
and (2, 2, 2, 2) for (a on the islands, a outside, b on the islands, b
outside).
"""

import numpy as np
import pytest

import paper_2103_03407_amd as m
from oracle import mlqmc, qmc, twogrid
from synth import CONFIGS, LevelSpec, islands_family, lattice_vector, shifts_for

pytestmark = pytest.mark.gpu

LAM_RTOL = 1e-10
G_RTOL = 1e-9
PARS = {"p43": (4.0 / 3.0, 2.0, 4.0 / 3.0, 2.0), "p2": (2.0, 2.0, 2.0, 2.0)}


@pytest.fixture(scope="module", params=sorted(PARS))
def fam(request):
    return islands_family(64, *PARS[request.param])


@pytest.fixture(scope="module")
def ctx(fam):
    c = m.Context(fam)
    yield c
    c.close()


def _lv6(lv):
    return (lv.n_fine, lv.s_fine, lv.n_coarse, lv.s_coarse, lv.n_prev, lv.s_prev)


def _points(s, count, seed):
    z = lattice_vector(1024, 64)[:s]
    sh = shifts_for(seed, 0, 1, s)[0]
    return np.ascontiguousarray(qmc.lattice_points(z, 1024, sh, range(count)))


def _rel(a, b):
    return np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b)))


@pytest.mark.parametrize("n,s,count", [(8, 8, 17), (16, 16, 12), (32, 16, 9), (32, 64, 7),
                                       (16, 0, 3)])
def test_direct_eigenvalues(ctx, fam, n, s, count):
    Y = _points(max(s, 1), count, 31)[:, :s]
    Y = np.ascontiguousarray(Y)
    lam = np.empty(count)
    fl = np.zeros(count, np.uint8)
    rq = np.zeros(count, np.int32)
    ctx.eig_level((n, s, 0, 0, 0, 0), Y, lam, fl, rq_iters=rq)
    assert not fl.any(), fl
    ref = np.array([twogrid.direct(n, s, y, fam)[0] for y in Y])
    assert _rel(lam, ref) <= LAM_RTOL
    assert rq.min() >= 1 and rq.max() <= 8


def test_warm_and_cold_chains_agree(ctx, fam):
    Y = _points(32, 24, 32)
    out = {}
    for warm in (0, 1):
        lam = np.empty(24)
        fl = np.zeros(24, np.uint8)
        o = m.default_opts(chain_len=8)
        ctx.eig_level((32, 32, 0, 0, 0, 0), Y, lam, fl, warm_chain=warm, opts=o)
        assert not fl.any()
        out[warm] = lam
    assert _rel(out[1], out[0]) <= LAM_RTOL


@pytest.mark.parametrize("lv", [(16, 16, 8, 8, 0, 0), (32, 64, 16, 32, 0, 0),
                                (32, 32, 8, 16, 16, 16), (32, 32, 8, 8, 8, 8)])
def test_two_grid_level(ctx, fam, lv):
    # two-grid value, its coarse value and the level-(l-1) term (including
    # the degenerate previous mesh, which is the coarse mesh itself)
    spec = LevelSpec(*lv, 0)
    count = 10
    Y = _points(lv[1], count, 33)
    lam, lamc, lamp = np.empty(count), np.empty(count), np.empty(count)
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_coarse=lamc, lam_prev=lamp if lv[4] else None)
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= LAM_RTOL * v.lam, (k, lam[k], v.lam)
        assert abs(lamc[k] - v.lam_coarse) <= LAM_RTOL * v.lam_coarse
        if lv[4]:
            assert abs(lamp[k] - v.lam_prev) <= LAM_RTOL * v.lam_prev


@pytest.mark.parametrize("lv", [(32, 16, 0, 0, 16, 8), (32, 32, 8, 16, 16, 16)])
def test_functional(ctx, fam, lv):
    spec = LevelSpec(*lv, 0)
    count = 8
    Y = _points(lv[1], count, 34)
    lam, lamp, g, gp = (np.empty(count) for _ in range(4))
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_prev=lamp, g=g, g_prev=gp)
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= LAM_RTOL * v.lam
        assert abs(lamp[k] - v.lam_prev) <= LAM_RTOL * v.lam_prev
        assert abs(g[k] - v.G) <= G_RTOL * v.G, (k, g[k], v.G)
        assert abs(gp[k] - v.G_prev) <= G_RTOL * v.G_prev


def test_estimate_three_levels(ctx, fam):
    levels = [LevelSpec(8, 8, 0, 0, 0, 0, 16), LevelSpec(16, 16, 8, 8, 8, 8, 8),
              LevelSpec(32, 32, 8, 16, 16, 16, 4)]
    R = 3
    Ns = [16, 8, 4]
    zs = [lattice_vector(N, lv.s_fine) for N, lv in zip(Ns, levels)]
    shifts = [shifts_for(35, l, R, lv.s_fine) for l, lv in enumerate(levels)]
    st, Q, Qh, V, est = ctx.estimate([_lv6(lv) for lv in levels], Ns, R, zs, shifts)
    assert st == m.MLQMC_OK
    ref = mlqmc.estimate(levels, zs, Ns, shifts, fam)
    # each level value is a difference of two eigenvalues, each below 5 here
    lam_max = 5.0
    assert ref.Qhat[0] < lam_max
    dq = 2 * lam_max * LAM_RTOL
    assert np.max(np.abs(Q - ref.Q_lr)) <= dq
    assert np.max(np.abs(Qh - ref.Qhat)) <= dq
    assert abs(est[0] - ref.Q_ml) <= 3 * dq
    dq = 2 * dq
    for l in range(3):
        bound = 2.0 / (R * (R - 1)) * np.sum(np.abs(ref.Qhat[l] - ref.Q_lr[l]) * dq) + R * dq * dq
        assert abs(V[l] - ref.V[l]) <= bound + 1e-18


def test_nested_estimate(ctx, fam):
    N = [16, 8, 4]
    levels = [LevelSpec(8, 4, 0, 0, 0, 0, N[0]), LevelSpec(16, 6, 8, 4, 8, 4, N[1]),
              LevelSpec(32, 8, 8, 4, 16, 6, N[2])]
    R = 2
    z = lattice_vector(64, 8) % N[0]
    shifts = shifts_for(36, 0, R, 8)
    st, Q, Qh, V, est, lam = ctx.estimate_nested([_lv6(l) for l in levels], N, R, z, shifts,
                                                 lam_out=True)
    assert st == m.MLQMC_OK
    for r in range(R):
        ref = mlqmc.nested_values(levels, z, N, shifts[r], fam)
        for l in range(3):
            assert np.max(np.abs(lam[l][r] - ref[l]) / ref[l]) <= LAM_RTOL, (l, r)
    ref = mlqmc.estimate_nested(levels, z, N, shifts, fam)
    scale = ref.Qhat[0]
    assert np.max(np.abs(Q - ref.Q_lr)) <= 4 * LAM_RTOL * scale
    assert abs(est[0] - ref.Q_ml) <= 4 * LAM_RTOL * scale


@pytest.mark.parametrize("lv,prec", [((2048, 32, 16, 16, 0, 0), m.MLQMC_FP64),
                                     ((4, 4, 0, 0, 0, 0), m.MLQMC_FP64),
                                     ((128, 16, 64, 8, 0, 0), m.MLQMC_FP64),
                                     ((64, 8, 0, 0, 0, 0), m.MLQMC_FP64),
                                     ((64, 8, 0, 0, 0, 0), m.MLQMC_MIXED),
                                     ((16, 8, 0, 0, 64, 8), m.MLQMC_MIXED)])
def test_rejected_levels(ctx, lv, prec):
    # meshes outside 1/8 .. 1/1024, coarse meshes and direct levels above 1/32
    # are refused on the host
    Y = _points(max(lv[1], 1), 2, 37)
    lam = np.empty(2)
    fl = np.zeros(2, np.uint8)
    with pytest.raises(m.MlqmcError) as e:
        ctx.eig_level(lv, Y, lam, fl, opts=m.default_opts(prec=prec))
    assert e.value.code == m.MLQMC_EINVAL


def test_problem1_calls_refused(ctx):
    Y = _points(4, 2, 38)
    with pytest.raises(m.MlqmcError) as e:
        ctx.coefficient(8, 4, Y, np.empty((2, 128)))
    assert e.value.code == m.MLQMC_EINVAL


# ---------------- the Problem 2 workloads at full size, sampled ----------------

def _level_points(ctx, w, l):
    lv = w.levels[l]
    Y = np.empty((w.R * lv.N, lv.s_fine))
    for r in range(w.R):
        ctx.lattice_points(lv.N, w.z(l), w.shifts(l)[r], 0, lv.N, Y[r * lv.N:(r + 1) * lv.N])
    return Y


@pytest.fixture(scope="module")
def ctx_p2():
    c = m.Context(CONFIGS[7].family())
    yield c
    c.close()


def test_cfg7_full_batch_sampled(ctx_p2):
    # the bench workload of Problem 2: every sample of the step unflagged,
    # strided samples against the oracle, the estimator from the same values
    w = CONFIGS[7]
    fam = w.family()
    lv = w.levels[0]
    Y = _level_points(ctx_p2, w, 0)
    n = Y.shape[0]
    lam, lamc = np.empty(n), np.empty(n)
    fl = np.zeros(n, np.uint8)
    ctx_p2.eig_level(_lv6(lv), Y, lam, fl, lam_coarse=lamc)
    assert not fl.any()
    for i in range(0, n, 1021):
        lt, lH, _ = twogrid.two_grid(lv.n_fine, lv.s_fine, lv.n_coarse, lv.s_coarse, Y[i], fam)
        assert abs(lam[i] - lt) <= LAM_RTOL * lt, (i, lam[i], lt)
        assert abs(lamc[i] - lH) <= LAM_RTOL * lH
    st, Q, Qh, V, est = ctx_p2.estimate([_lv6(lv)], [lv.N], w.R, [w.z(0)],
                                        [w.shifts(0)])
    assert st == m.MLQMC_OK
    per_r = lam.reshape(w.R, lv.N).mean(axis=1)
    assert np.max(np.abs(Q[0] - per_r)) <= 1e-12 * np.max(per_r)


def test_cfg8_three_levels_sampled(ctx_p2):
    # the three-level Problem 2 workload (h = 1/8, 1/16, 1/32): per level, the
    # level values of every point unflagged, strided ones against the oracle,
    # and the estimator's level means equal to the means of those values
    w = CONFIGS[8]
    fam = w.family()
    st, Q, Qh, V, est = ctx_p2.estimate([_lv6(lv) for lv in w.levels],
                                        [lv.N for lv in w.levels], w.R,
                                        [w.z(l) for l in range(3)],
                                        [w.shifts(l) for l in range(3)])
    assert st == m.MLQMC_OK
    for l, lv in enumerate(w.levels):
        Y = _level_points(ctx_p2, w, l)
        n = Y.shape[0]
        lam, lamp = np.empty(n), np.empty(n)
        fl = np.zeros(n, np.uint8)
        ctx_p2.eig_level(_lv6(lv), Y, lam, fl, lam_prev=lamp if lv.n_prev else None)
        assert not fl.any()
        Yl = lam - lamp if lv.n_prev else lam
        for i in range(0, n, n // 5 + 7):
            v = mlqmc.level_value(lv, Y[i], fam)
            assert abs(lam[i] - v.lam) <= LAM_RTOL * v.lam, (l, i)
            assert abs(Yl[i] - v.Y) <= 2 * LAM_RTOL * v.lam, (l, i)
        per_r = Yl.reshape(w.R, lv.N).mean(axis=1)
        assert np.max(np.abs(Q[l] - per_r)) <= 1e-12 * np.max(lam)
    assert abs(est[0] - Qh.sum()) <= 1e-13 * abs(est[0])


# ---------------- mixed precision ----------------

def _mixed():
    return m.default_opts(prec=m.MLQMC_MIXED)


@pytest.mark.parametrize("n,s,count", [(8, 8, 9), (16, 16, 8), (32, 64, 7)])
def test_mixed_direct(ctx, fam, n, s, count):
    Y = _points(s, count, 60)
    lam = np.empty(count)
    fl = np.zeros(count, np.uint8)
    ctx.eig_level((n, s, 0, 0, 0, 0), Y, lam, fl, opts=_mixed())
    assert not fl.any(), fl
    ref = np.array([twogrid.direct(n, s, y, fam)[0] for y in Y])
    assert _rel(lam, ref) <= 1e-8


@pytest.mark.parametrize("lv", [(16, 16, 8, 8, 0, 0), (32, 64, 8, 8, 16, 32),
                                (32, 32, 8, 16, 8, 16)])
def test_mixed_two_grid_level(ctx, fam, lv):
    spec = LevelSpec(*lv, 0)
    count = 8
    Y = _points(lv[1], count, 61)
    lam, lamc, lamp = np.empty(count), np.empty(count), np.empty(count)
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_coarse=lamc, lam_prev=lamp if lv[4] else None,
                  opts=_mixed())
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= 1e-8 * v.lam, (k, lam[k], v.lam)
        assert abs(lamc[k] - v.lam_coarse) <= 1e-8 * v.lam_coarse
        if lv[4]:
            assert abs(lamp[k] - v.lam_prev) <= 1e-8 * v.lam_prev


def test_mixed_functional(ctx, fam):
    lv = (32, 32, 8, 16, 16, 16)
    spec = LevelSpec(*lv, 0)
    count = 6
    Y = _points(lv[1], count, 62)
    lam, lamp, g, gp = (np.empty(count) for _ in range(4))
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_prev=lamp, g=g, g_prev=gp, opts=_mixed())
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(g[k] - v.G) <= 1e-7 * v.G, (k, g[k], v.G)
        assert abs(gp[k] - v.G_prev) <= 1e-7 * v.G_prev


def test_mixed_cfg8_sampled(ctx_p2):
    # the three-level Problem 2 workload in mixed precision: every level value
    # unflagged, strided ones within 1e-8 of the oracle
    w = CONFIGS[8]
    fam = w.family()
    for l, lv in enumerate(w.levels):
        Y = _level_points(ctx_p2, w, l)
        n = Y.shape[0]
        lam, lamp = np.empty(n), np.empty(n)
        fl = np.zeros(n, np.uint8)
        ctx_p2.eig_level(_lv6(lv), Y, lam, fl, lam_prev=lamp if lv.n_prev else None,
                         opts=_mixed())
        assert not fl.any()
        Yl = lam - lamp if lv.n_prev else lam
        for i in range(0, n, n // 4 + 11):
            v = mlqmc.level_value(lv, Y[i], fam)
            assert abs(lam[i] - v.lam) <= 1e-8 * v.lam, (l, i)
            assert abs(Yl[i] - v.Y) <= 2e-8 * v.lam, (l, i)


# ---------------- two-grid updates on 1/64 (batched kernels with the reaction) ----------------

@pytest.mark.parametrize("lv", [(64, 32, 8, 8, 0, 0), (64, 64, 16, 16, 32, 32),
                                (64, 64, 8, 16, 8, 16)])
def test_two_grid_level_64(ctx, fam, lv):
    spec = LevelSpec(*lv, 0)
    count = 6
    Y = _points(lv[1], count, 70)
    lam, lamc, lamp = np.empty(count), np.empty(count), np.empty(count)
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_coarse=lamc, lam_prev=lamp if lv[4] else None)
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= LAM_RTOL * v.lam, (k, lam[k], v.lam)
        assert abs(lamc[k] - v.lam_coarse) <= LAM_RTOL * v.lam_coarse
        if lv[4]:
            assert abs(lamp[k] - v.lam_prev) <= LAM_RTOL * v.lam_prev


def test_functional_64(ctx, fam):
    lv = (64, 32, 8, 8, 32, 16)
    spec = LevelSpec(*lv, 0)
    count = 5
    Y = _points(lv[1], count, 71)
    lam, lamp, g, gp = (np.empty(count) for _ in range(4))
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_prev=lamp, g=g, g_prev=gp)
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= LAM_RTOL * v.lam
        assert abs(g[k] - v.G) <= G_RTOL * v.G, (k, g[k], v.G)
        assert abs(gp[k] - v.G_prev) <= G_RTOL * v.G_prev


def test_64_many_samples(ctx, fam):
    # a batch of 4100 samples (the first, the last and two in between against
    # the oracle)
    lv = (64, 16, 8, 8, 0, 0)
    n = 4100
    z = lattice_vector(16384, 16)
    sh = shifts_for(72, 0, 1, 16)[0]
    Y = np.ascontiguousarray(qmc.lattice_points(z, 16384, sh, range(n)))
    lam = np.empty(n)
    fl = np.zeros(n, np.uint8)
    ctx.eig_level(lv, Y, lam, fl)
    assert not fl.any()
    for k in (0, 4095, 4096, n - 1):
        ref = twogrid.two_grid(64, 16, 8, 8, Y[k], fam)[0]
        assert abs(lam[k] - ref) <= LAM_RTOL * ref, (k, lam[k], ref)


def test_estimate_four_levels(ctx, fam):
    # h = 1/8, 1/16, 1/32, 1/64 (h_l = 2^-(l+3)), H = 1/8: the paper's
    # Problem 2 hierarchy through level 3
    levels = [LevelSpec(8, 8, 0, 0, 0, 0, 16), LevelSpec(16, 16, 8, 8, 8, 8, 8),
              LevelSpec(32, 32, 8, 8, 16, 16, 4), LevelSpec(64, 32, 8, 8, 32, 32, 4)]
    R = 2
    Ns = [16, 8, 4, 4]
    zs = [lattice_vector(N, lv.s_fine) for N, lv in zip(Ns, levels)]
    shifts = [shifts_for(73, l, R, lv.s_fine) for l, lv in enumerate(levels)]
    st, Q, Qh, V, est = ctx.estimate([_lv6(lv) for lv in levels], Ns, R, zs, shifts)
    assert st == m.MLQMC_OK
    ref = mlqmc.estimate(levels, zs, Ns, shifts, fam)
    dq = 2 * 5.0 * LAM_RTOL
    assert np.max(np.abs(Q - ref.Q_lr)) <= dq
    assert abs(est[0] - ref.Q_ml) <= 4 * dq


@pytest.mark.parametrize("lv", [(64, 32, 8, 8, 0, 0), (64, 64, 16, 16, 32, 32)])
def test_mixed_two_grid_level_64(ctx, fam, lv):
    spec = LevelSpec(*lv, 0)
    count = 6
    Y = _points(lv[1], count, 74)
    lam, lamp = np.empty(count), np.empty(count)
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_prev=lamp if lv[4] else None, opts=_mixed())
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= 1e-8 * v.lam, (k, lam[k], v.lam)
        if lv[4]:
            assert abs(lamp[k] - v.lam_prev) <= 1e-8 * v.lam_prev


# ---------------- two-grid updates on 1/128 and 1/256 ----------------

@pytest.mark.parametrize("prec,tol", [("fp64", LAM_RTOL), ("mixed", 1e-8)])
@pytest.mark.parametrize("lv", [(128, 64, 8, 8, 0, 0), (128, 64, 16, 16, 64, 32)])
def test_two_grid_level_128(ctx, fam, lv, prec, tol):
    spec = LevelSpec(*lv, 0)
    count = 4
    Y = _points(lv[1], count, 80)
    lam, lamp = np.empty(count), np.empty(count)
    fl = np.zeros(count, np.uint8)
    o = m.default_opts(prec=m.MLQMC_FP64 if prec == "fp64" else m.MLQMC_MIXED)
    ctx.eig_level(lv, Y, lam, fl, lam_prev=lamp if lv[4] else None, opts=o)
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= tol * v.lam, (k, lam[k], v.lam)
        if lv[4]:
            assert abs(lamp[k] - v.lam_prev) <= tol * v.lam_prev


def test_128_two_batches(ctx, fam):
    # batches of 512 samples: both sides of the batch boundary
    lv = (128, 16, 8, 8, 0, 0)
    n = 520
    z = lattice_vector(16384, 16)
    sh = shifts_for(81, 0, 1, 16)[0]
    Y = np.ascontiguousarray(qmc.lattice_points(z, 16384, sh, range(n)))
    lam = np.empty(n)
    fl = np.zeros(n, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, opts=m.default_opts(batch=512))
    assert not fl.any()
    for k in (511, 512, n - 1):
        ref = twogrid.two_grid(128, 16, 8, 8, Y[k], fam)[0]
        assert abs(lam[k] - ref) <= LAM_RTOL * ref, (k, lam[k], ref)



@pytest.mark.parametrize("prec,tol", [("fp64", LAM_RTOL), ("mixed", 1e-8)])
@pytest.mark.parametrize("lv", [(256, 64, 8, 8, 0, 0), (256, 64, 16, 16, 128, 32)])
def test_two_grid_level_256(ctx, fam, lv, prec, tol):
    spec = LevelSpec(*lv, 0)
    count = 3
    Y = _points(lv[1], count, 82)
    lam, lamp = np.empty(count), np.empty(count)
    fl = np.zeros(count, np.uint8)
    o = m.default_opts(prec=m.MLQMC_FP64 if prec == "fp64" else m.MLQMC_MIXED)
    ctx.eig_level(lv, Y, lam, fl, lam_prev=lamp if lv[4] else None, opts=o)
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= tol * v.lam, (k, lam[k], v.lam)
        if lv[4]:
            assert abs(lamp[k] - v.lam_prev) <= tol * v.lam_prev


def test_functional_256(ctx, fam):
    lv = (256, 32, 8, 8, 64, 16)
    spec = LevelSpec(*lv, 0)
    count = 2
    Y = _points(lv[1], count, 83)
    lam, lamp, g, gp = (np.empty(count) for _ in range(4))
    fl = np.zeros(count, np.uint8)
    ctx.eig_level(lv, Y, lam, fl, lam_prev=lamp, g=g, g_prev=gp)
    assert not fl.any(), fl
    for k in range(count):
        v = mlqmc.level_value(spec, Y[k], fam)
        assert abs(lam[k] - v.lam) <= LAM_RTOL * v.lam
        assert abs(g[k] - v.G) <= G_RTOL * v.G, (k, g[k], v.G)
        assert abs(gp[k] - v.G_prev) <= G_RTOL * v.G_prev


def test_no_random_terms_on_64(ctx, fam):
    # s = S = 0: the background coefficients alone (the tables' base rows)
    lv = (64, 0, 8, 0, 0, 0)
    Y = np.zeros((3, 0))
    lam = np.empty(3)
    fl = np.zeros(3, np.uint8)
    ctx.eig_level(lv, Y, lam, fl)
    assert not fl.any()
    ref = twogrid.two_grid(64, 0, 8, 0, np.zeros(0), fam)[0]
    assert np.max(np.abs(lam - ref)) <= LAM_RTOL * ref


def test_nested_and_extended_with_a_64_level(ctx, fam):
    # shared shifts with level 3 on 1/64 (a batched update), grown in two
    # steps, against the oracle's nested estimate
    N = [8, 4, 4, 2]
    levels = [LevelSpec(8, 4, 0, 0, 0, 0, N[0]), LevelSpec(16, 6, 8, 4, 8, 4, N[1]),
              LevelSpec(32, 8, 8, 4, 16, 6, N[2]), LevelSpec(64, 8, 8, 4, 32, 8, N[3])]
    l6 = [_lv6(l) for l in levels]
    z = lattice_vector(64, 8)
    R = 2
    shifts = shifts_for(75, 0, R, 8)
    sums = np.zeros((4, R))
    ctx.estimate_nested_extend(l6, [0] * 4, [4, 2, 2, 1], R, z, shifts, sums)
    st, Q, Qh, V, est = ctx.estimate_nested_extend(l6, [4, 2, 2, 1], N, R, z, shifts, sums)
    assert st == m.MLQMC_OK
    ref = mlqmc.estimate_nested(levels, z, N, shifts, fam)
    scale = ref.Qhat[0]
    assert np.max(np.abs(Q - ref.Q_lr)) <= 4 * LAM_RTOL * scale
    assert abs(est[0] - ref.Q_ml) <= 4 * LAM_RTOL * scale


def test_cfg10_five_levels_sampled(ctx_p2):
    # the five-level Problem 2 workload (h = 1/8 .. 1/128, s = 16 .. 256) at
    # full size: the estimator's level means equal the means of the level
    # values, every value unflagged, strided ones against the oracle
    w = CONFIGS[10]
    fam = w.family()
    c = m.Context(fam)
    try:
        st, Q, Qh, V, est = c.estimate([_lv6(lv) for lv in w.levels], [lv.N for lv in w.levels],
                                       w.R, [w.z(l) for l in range(5)],
                                       [w.shifts(l) for l in range(5)])
        assert st == m.MLQMC_OK
        for l, lv in enumerate(w.levels):
            Y = _level_points(c, w, l)
            n = Y.shape[0]
            lam, lamp = np.empty(n), np.empty(n)
            fl = np.zeros(n, np.uint8)
            c.eig_level(_lv6(lv), Y, lam, fl, lam_prev=lamp if lv.n_prev else None)
            assert not fl.any()
            Yl = lam - lamp if lv.n_prev else lam
            for i in range(0, n, n // 3 + 5):
                v = mlqmc.level_value(lv, Y[i], fam)
                assert abs(lam[i] - v.lam) <= LAM_RTOL * v.lam, (l, i)
                assert abs(Yl[i] - v.Y) <= 2 * LAM_RTOL * v.lam, (l, i)
            per_r = Yl.reshape(w.R, lv.N).mean(axis=1)
            assert np.max(np.abs(Q[l] - per_r)) <= 2 * LAM_RTOL * np.max(lam)
    finally:
        c.close()


def test_cfg12_finest_level_sampled(ctx_p2):
    # the six-level Problem 2 workload's finest level (h = 1/256, s = 512,
    # previous term on 1/128) at full size: every value unflagged, three
    # strided ones against the oracle, the estimator's level mean equal to the
    # mean of the level values
    w = CONFIGS[12]
    fam = w.family()
    l = 5
    lv = w.levels[l]
    c = m.Context(fam)
    try:
        st, Q, Qh, V, est = c.estimate([_lv6(x) for x in w.levels], [x.N for x in w.levels],
                                       w.R, [w.z(i) for i in range(6)],
                                       [w.shifts(i) for i in range(6)])
        assert st == m.MLQMC_OK
        Y = _level_points(c, w, l)
        n = Y.shape[0]
        lam, lamp = np.empty(n), np.empty(n)
        fl = np.zeros(n, np.uint8)
        c.eig_level(_lv6(lv), Y, lam, fl, lam_prev=lamp)
        assert not fl.any()
        Yl = lam - lamp
        for i in (0, n // 2 + 7, n - 1):
            v = mlqmc.level_value(lv, Y[i], fam)
            assert abs(lam[i] - v.lam) <= LAM_RTOL * v.lam, (i, lam[i], v.lam)
            assert abs(Yl[i] - v.Y) <= 2 * LAM_RTOL * v.lam, (i, Yl[i], v.Y)
        per_r = Yl.reshape(w.R, lv.N).mean(axis=1)
        assert np.max(np.abs(Q[l] - per_r)) <= 2 * LAM_RTOL * np.max(lam)
    finally:
        c.close()
