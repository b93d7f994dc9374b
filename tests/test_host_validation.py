"""Argument checking of every entry point, on the CPU.

A context created with ``MLQMC_HOST_ONLY`` touches no device: each call runs
the same argument checks as on a GPU context and then returns MLQMC_EINVAL
(invalid arguments, with a message) or MLQMC_EDEVICE (valid arguments; it
never computes).  So every rejection below is the library's own code path,
and the valid cases prove the checks do not reject what the GPU tests run."""

import ctypes as C

import numpy as np
import pytest

import paper_2103_03407_amd as m
from synth import coeff_family
from synth.family import islands_family

HOST = m.MLQMC_HOST_ONLY


@pytest.fixture(scope="module")
def ctx():
    c = m.Context(coeff_family(32), device=HOST)
    yield c
    c.close()


@pytest.fixture(scope="module")
def isl():
    c = m.Context(islands_family(16, 4 / 3, 2.0, 4 / 3, 2.0), device=HOST)
    yield c
    c.close()


def _code(fn, *a, **k):
    try:
        fn(*a, **k)
    except m.MlqmcError as e:
        return e.code, str(e)
    return m.MLQMC_OK, ""


def _level_call(c, level, n=4, opts=None, nan=False, lam_prev=True):
    s = level[1]
    Y = np.zeros((n, s))
    if nan and n * s:
        Y[0, 0] = np.nan
    lam = np.zeros(n)
    fl = np.zeros(n, np.uint8)
    lp = np.zeros(n) if lam_prev else None
    return _code(c.eig_level, level, Y, lam, fl, lam_prev=lp, opts=opts)


def test_host_only_context_is_not_a_fallback(ctx):
    code, msg = _level_call(ctx, (16, 8, 0, 0, 0, 0))
    assert code == m.MLQMC_EDEVICE and "host-only" in msg


@pytest.mark.parametrize("level", [
    (16, 8, 0, 0, 0, 0),        # direct
    (64, 16, 0, 0, 32, 8),      # direct with a direct previous level
    (128, 32, 32, 8, 0, 0),     # two-grid
    (1024, 32, 64, 23, 512, 16),  # two-grid with a previous two-grid term
    (64, 16, 16, 8, 16, 8),     # degenerate previous mesh
])
def test_valid_levels_reach_the_device(ctx, level):
    assert _level_call(ctx, level)[0] == m.MLQMC_EDEVICE


@pytest.mark.parametrize("level,what", [
    ((24, 8, 0, 0, 0, 0), "power of two"),
    ((16, 33, 0, 0, 0, 0), "s_fine"),
    ((128, 8, 0, 0, 0, 0), "direct levels"),
    ((2, 8, 0, 0, 0, 0), "direct levels"),
    ((64, 8, 64, 4, 0, 0), "n_coarse < n_fine"),
    ((2048, 8, 64, 4, 0, 0), "n_coarse < n_fine"),
    ((128, 8, 128 // 3, 4, 0, 0), "n_coarse"),
    ((128, 8, 32, 9, 0, 0), "s_coarse"),
    ((128, 8, 32, 4, 16, 4), "n_coarse <= n_prev"),
    ((128, 8, 32, 4, 64, 9), "s_prev"),
    ((32, 8, 0, 0, 128, 4), "direct previous"),
    ((32, 8, 0, 0, 48, 4), "power of two"),
])
def test_invalid_levels(ctx, level, what):
    code, msg = _level_call(ctx, level)
    assert code == m.MLQMC_EINVAL and what in msg, msg


def test_non_finite_point_and_sizes(ctx):
    code, msg = _level_call(ctx, (16, 8, 0, 0, 0, 0), nan=True)
    assert code == m.MLQMC_EINVAL and "non-finite" in msg
    code, msg = _level_call(ctx, (128, 8, 32, 4, 64, 4), lam_prev=False)
    assert code == m.MLQMC_EINVAL and "lam_prev" in msg
    # no points: valid, and nothing to do before the device is needed
    assert _level_call(ctx, (16, 8, 0, 0, 0, 0), n=0)[0] == m.MLQMC_EDEVICE


@pytest.mark.parametrize("field,value,what", [
    ("prec", 7, "precision"),
    ("eig_rtol", 0.0, "tolerances"),
    ("eig_atol", -1e-8, "tolerances"),
    ("lin_rtol", -1.0, "tolerances"),
    ("lam_rtol", float("nan"), "tolerances"),
    ("rq_lin_rtol", 0.0, "tolerances"),
    ("max_rq_iter", 0, "caps"),
    ("max_lin_iter", 0, "caps"),
    ("device_mem_cap", -1, "device_mem_cap"),
])
def test_invalid_options(ctx, field, value, what):
    o = m.default_opts()
    setattr(o, field, value)
    code, msg = _level_call(ctx, (16, 8, 0, 0, 0, 0), opts=o)
    assert code == m.MLQMC_EINVAL and what in msg, msg


def test_components(ctx, isl):
    z = np.array([1, 5, 7], np.int64)
    sh = np.array([0.1, 0.2, 0.3])
    Y = np.zeros((4, 3))
    assert _code(ctx.lattice_points, 8, z, sh, 0, 4, Y)[0] == m.MLQMC_EDEVICE
    assert _code(ctx.embedded_points, 8, z, sh, 0, 4, Y)[0] == m.MLQMC_EDEVICE
    code, msg = _code(ctx.lattice_points, 12, z, sh, 0, 4, Y)
    assert code == m.MLQMC_EINVAL and "power of two" in msg
    code, msg = _code(ctx.lattice_points, 8, np.array([1, 8, 7]), sh, 0, 4, Y)
    assert code == m.MLQMC_EINVAL and "z[1]" in msg
    code, msg = _code(ctx.lattice_points, 8, z, np.array([0.1, 1.0, 0.3]), 0, 4, Y)
    assert code == m.MLQMC_EINVAL and "shift[1]" in msg
    code, msg = _code(ctx.lattice_points, 8, z, sh, 6, 4, Y)
    assert code == m.MLQMC_EINVAL and "k0" in msg
    aK = np.zeros((4, 2 * 16 * 16))
    assert _code(ctx.coefficient, 16, 3, Y, aK)[0] == m.MLQMC_EDEVICE
    code, msg = _code(ctx.coefficient, 16, 33, np.zeros((4, 33)), aK)
    assert code == m.MLQMC_EINVAL and "s_max" in msg
    code, msg = _code(isl.coefficient, 16, 3, Y, aK)
    assert code == m.MLQMC_EINVAL and "Problem 1" in msg
    code, msg = _code(ctx.prolong, 16, 12, np.zeros((2, 225)), np.zeros((2, 121)))
    assert code == m.MLQMC_EINVAL and "powers of two" in msg


def _estimate_args():
    levels = [(16, 8, 0, 0, 0, 0), (64, 16, 16, 8, 16, 8)]
    N = [16, 8]
    z = [np.array([1, 3, 5, 7, 9, 11, 13, 15]), np.tile([1, 3, 5, 7], 4)]
    R = 2
    sh = [np.full((R, 8), 0.25), np.full((R, 16), 0.5)]
    return levels, N, R, z, sh


def test_estimate(ctx):
    levels, N, R, z, sh = _estimate_args()
    assert _code(ctx.estimate, levels, N, R, z, sh)[0] == m.MLQMC_EDEVICE
    code, msg = _code(ctx.estimate, levels, [16, 12], R, z, sh)
    assert code == m.MLQMC_EINVAL and "N[1]" in msg
    bad = [z[0], z[1].copy()]
    bad[1][3] = 8
    code, msg = _code(ctx.estimate, levels, N, R, bad, sh)
    assert code == m.MLQMC_EINVAL and "z of level 1" in msg
    bad = [sh[0], sh[1].copy()]
    bad[1][1, 2] = -0.1
    code, msg = _code(ctx.estimate, levels, N, R, z, bad)
    assert code == m.MLQMC_EINVAL and "shift of level 1" in msg
    code, msg = _code(ctx.estimate, [levels[0], (64, 16, 16, 17, 16, 8)], N, R, z, sh)
    assert code == m.MLQMC_EINVAL and "s_coarse" in msg


def _nested_args():
    levels = [(16, 8, 0, 0, 0, 0), (32, 16, 16, 8, 16, 8), (64, 16, 16, 8, 32, 16)]
    N = [32, 16, 8]
    R = 2
    z = np.arange(1, 33, 2, dtype=np.int64)[:16]
    sh = np.full((R, 16), 0.5)
    return levels, N, R, z, sh


def test_nested(ctx):
    levels, N, R, z, sh = _nested_args()
    assert _code(ctx.estimate_nested, levels, N, R, z, sh)[0] == m.MLQMC_EDEVICE
    code, msg = _code(ctx.estimate_nested, levels, [16, 32, 8], R, z, sh)
    assert code == m.MLQMC_EINVAL and "must not increase" in msg
    code, msg = _code(ctx.estimate_nested, [(16, 8, 0, 0, 8, 4)] + levels[1:], N, R, z, sh)
    assert code == m.MLQMC_EINVAL and "level 0" in msg
    code, msg = _code(ctx.estimate_nested, [levels[0], (32, 16, 8, 8, 16, 8), levels[2]], N, R,
                      z, sh)
    assert code == m.MLQMC_EINVAL and "coarse mesh" in msg
    code, msg = _code(ctx.estimate_nested, [levels[0], levels[1], (64, 16, 16, 8, 16, 8)], N, R,
                      z, sh)
    assert code == m.MLQMC_EINVAL and "previous term" in msg
    zb = z.copy()
    zb[2] = -1
    code, msg = _code(ctx.estimate_nested, levels, N, R, zb, sh)
    assert code == m.MLQMC_EINVAL and "z[2]" in msg
    sums = np.zeros((3, R))
    assert _code(ctx.estimate_nested_extend, levels, [8, 8, 4], N, R, z, sh,
                 sums)[0] == m.MLQMC_EDEVICE
    code, msg = _code(ctx.estimate_nested_extend, levels, [8, 32, 4], N, R, z, sh, sums)
    assert code == m.MLQMC_EINVAL and "N_done[1]" in msg


def test_adaptive(ctx):
    levels, _, R, z, sh = _nested_args()
    run = ctx.estimate_adaptive
    assert _code(run, levels, R, z, sh, eps=0.01)[0] == m.MLQMC_EDEVICE
    code, msg = _code(run, levels, 1, z, sh[:1], eps=0.01)
    assert code == m.MLQMC_EINVAL and "R >= 2" in msg
    for kw in ({"eps": 0.0}, {"eps": 0.01, "N_init": 12}, {"eps": 0.01, "N_init": 64,
                                                            "N_max": 32},
               {"eps": 0.01, "gamma": -1.0}):
        code, msg = _code(run, levels, R, z, sh, **kw)
        assert code == m.MLQMC_EINVAL and "adaptive options" in msg, kw
    # a level the rule may add later is checked up front
    code, msg = _code(run, levels[:2] + [(64, 16, 16, 8, 16, 8)], R, z, sh, eps=0.01)
    assert code == m.MLQMC_EINVAL and "previous term" in msg


def test_islands_meshes(isl):
    assert _level_call(isl, (32, 16, 0, 0, 16, 8))[0] == m.MLQMC_EDEVICE
    assert _level_call(isl, (1024, 16, 8, 8, 512, 16))[0] == m.MLQMC_EDEVICE
    for level, what in [((64, 16, 0, 0, 0, 0), "direct"),
                        ((128, 16, 64, 8, 0, 0), "coarse"),
                        ((16, 8, 4, 4, 0, 0), "1/8"),
                        ((2048, 16, 8, 8, 0, 0), "n_coarse < n_fine")]:
        code, msg = _level_call(isl, level)
        assert code == m.MLQMC_EINVAL and what in msg, (level, msg)


def test_noalloc_limits(ctx):
    lib, h = ctx._lib, ctx._h
    o = m.default_opts()
    lam = np.zeros(4)
    fl = np.zeros(4, np.uint8)
    Y = np.zeros((4, 8))

    def call(level, on_dev, n=4):
        o.io_on_device = on_dev
        lv = m.Level(*level)
        st = lib.mlqmc_eig_level_noalloc(h, C.byref(lv), C.byref(o), n,
                                         C.c_void_p(Y.ctypes.data), 1,
                                         C.c_void_p(lam.ctypes.data), None, None, None, None,
                                         C.c_void_p(fl.ctypes.data))
        return st, lib.mlqmc_last_error(h).decode()

    st, msg = call((16, 8, 0, 0, 0, 0), 0)
    assert st == m.MLQMC_EINVAL and "device pointers" in msg
    st, msg = call((64, 8, 16, 8, 0, 0), 1)
    assert st == m.MLQMC_EINVAL and "1/32" in msg
    st, msg = call((32, 8, 16, 8, 0, 0), 1, n=1 << 22)
    assert st == m.MLQMC_EINVAL and "MLQMC_NOALLOC_SCRATCH_BYTES" in msg
    st, msg = call((32, 8, 16, 8, 0, 0), 1)
    assert st == m.MLQMC_EDEVICE and "host-only" in msg


def test_timing_and_tuning(ctx):
    assert _code(ctx.set_tuning, 48, m.MLQMC_FP64, 1024)[0] == m.MLQMC_EINVAL
    assert _code(ctx.set_tuning, 128, 5, 1024)[0] == m.MLQMC_EINVAL
    assert _code(ctx.set_tuning, 128, m.MLQMC_FP64, 1024)[0] == m.MLQMC_OK
    assert ctx._lib.mlqmc_set_timing(ctx._h, 99) == m.MLQMC_EINVAL
    assert ctx._lib.mlqmc_get_timing(ctx._h, None, None, None, None) == m.MLQMC_EDEVICE
