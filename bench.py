#!/usr/bin/env python3
"""Throughput of the two-grid MLQMC eigen-sample path on one MI355X.

One step = one pass of the whole hot path over one batch: lattice points ->
coefficient expansion -> warm-started coarse RQ eigensolve -> prolongation ->
projected-PCG shifted fine solve -> Rayleigh quotient -> level accumulation,
i.e. one ``mlqmc_estimate`` call.  The default workload is the largest that
fits one GPU: the two-grid level H = 1/64 -> h = 1/1024 (1 046 529 fine
unknowns), s = 512, S = 23, coefficients decaying as j^-2, N = 1024 lattice
points x R = 8 shifts (8192 eigen-samples), all synthetic (CBC lattice,
seeded shifts), in FP64.  On that workload (and on ``--cfg 2``) the line also
carries: the other batched kernels' rates, the mixed-precision path, the FP64
path stopped at the mixed path's tolerances (equal accuracy), each with its
error against the oracle, and the two-grid 1/32 -> 1/128 workload (s = 64).

``--cfg`` selects another workload of ``synth/configs.py``: 4 and 6 are the
five-level estimators (independent and shared shifts), 7 to 10 and 12
Problem 2 (the islands) as one two-grid level H = 1/8 -> h = 1/32 and as the
three- to six-level estimators on h = 1/8 .. 1/32, 1/64, 1/128 and 1/256.
Updates on meshes up to 1/32 run per sample in LDS (the roofline is then
those kernels' rate against the vector peak of the precision); finer ones on
the batched stencil kernels (HBM roofline).

Prints one JSON line.  ``value`` = eigen-samples per second on one GPU.
Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
PEAK_FP64_MFMA_TFS = 78.6  # MI355X dense FP64 matrix, published
PEAK_FP64_VALU_TFS = 78.6  # MI355X FP64 vector, published
PEAK_FP32_VALU_TFS = 157.3  # MI355X FP32 vector, published
# LDS: 128 bytes per clock per compute unit x 256 units x 2.4 GHz
PEAK_LDS_TBS = 128 * 256 * 2.4e9 / 1e12


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cfg", type=int, default=5,
                    help="workload id (5: two-grid 1/64 -> 1/1024, s = 512; 2: 1/32 -> 1/128)")
    ap.add_argument("--kernel-class", default=None,
                    choices=["post", "pre", "apply", "coeff", "lds", "rqi"],
                    help="kernel timed for the roofline (default: post, the dominant kernel of "
                         "the batched path; lds, the per-sample two-grid update, for workloads "
                         "without batched levels; rqi, the eigensolve, for direct-only ones)")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"],
                    help="fp64, or mixed (FP32 fine PCG/V-cycle, FP64 residual and RQ)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the main leg (no other kernel classes, no second precision, no "
                         "equal-accuracy FP64 leg, no 1/32 -> 1/128 workload)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the untimed accuracy pass (for profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES bytes (counter calibration)")
    ap.add_argument("--plain-vs-enhanced", action="store_true",
                    help="only compare, per level of the workload (direct solves up to 1/64), the "
                         "enhanced method (two-grid update, warm-started RQ) with plain MLQMC "
                         "(direct eigensolves, cold start) on the same points")
    return ap.parse_args()


def _lv6(lv):
    return (lv.n_fine, lv.s_fine, lv.n_coarse, lv.s_coarse, lv.n_prev, lv.s_prev)


def _flat(w, i):
    """The i-th sample of workload w in (level, shift r, lattice index k) order."""
    for l, lv in enumerate(w.levels):
        n = w.R * lv.N
        if i < n:
            r, k = divmod(i, lv.N)
            return l, r, k
        i -= n
    raise IndexError(i)


def _oracle_worker(args):
    # CPU baseline: the oracle as it stands, one sample per call
    cfg_id, l, r, k = args
    from oracle import mlqmc, qmc
    from synth import CONFIGS
    w = CONFIGS[cfg_id]
    lv = w.levels[l]
    y = qmc.lattice_point(w.z(l), lv.N, w.shifts(l)[r], k)
    v = mlqmc.level_value(lv, y, w.family())
    return v.Y, v.lam


def _oracle_nested_worker(args):
    # CPU baseline of a nested workload: the oracle's evaluation of one point
    # of shift r (every level whose N_l exceeds k), as its nested estimator
    # runs it
    cfg_id, r, k = args
    from oracle import mlqmc
    from synth import CONFIGS
    w = CONFIGS[cfg_id]
    lams = mlqmc.nested_point(list(w.levels), w.z_shared(), [lv.N for lv in w.levels],
                              w.shifts_shared()[r], k, w.family())
    return [(l, lam - (lams[l - 1] if l else 0.0), lam) for l, lam in enumerate(lams)]


def cpu_baseline_nested(cfg_id: int, seconds: float, cores: int):
    import multiprocessing as mp
    from synth import CONFIGS
    w = CONFIGS[cfg_id]
    N0 = w.levels[0].N
    t0 = time.perf_counter()
    _oracle_nested_worker((cfg_id, 0, 0))            # a point on every level
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    _oracle_nested_worker((cfg_id, 0, N0 - 1))       # a level-0-only point
    t_one = time.perf_counter() - t0
    share = w.levels[-1].N / N0
    per = share * t_all + (1 - share) * t_one
    count = max(cores, min(N0, int(seconds * cores / max(per, 1e-3))))
    pts = [(cfg_id, i % w.R, (i * 7919) % N0) for i in range(count)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        vals = pool.map(_oracle_nested_worker, pts, chunksize=1)
    dt = time.perf_counter() - t0
    idx, ref = [], []
    for (_, r, k), lv in zip(pts, vals):
        for l, y, lam in lv:
            assert math.isfinite(y)
            idx.append((l, r, k))
            ref.append((y, lam))
    base = {"value": len(idx) / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{count} of the {w.R * N0} points of the nested rule (strided), "
                      f"{len(idx)} level samples Y_l, scipy/SuperLU FP64, {cores} processes, "
                      f"{dt:.1f} s"}
    return base, idx, ref


def _worker_bytes(w) -> float:
    """Peak memory of one oracle worker on workload w: the [s, 2 n^2] table of
    coefficient terms (oracle.coeff.basis_at) or the sparse LU factors of the
    finest mesh, whichever is larger, plus the interpreter."""
    peak = 0.0
    for lv in w.levels:
        n, s = lv.n_fine, lv.s_fine
        peak = max(peak, 8.0 * s * 2 * n * n, 4e9 * (n / 1024.0) ** 2)
    return peak + 1e9


def _oracle_pool_size(w) -> int:
    """Oracle processes: every affinity core, as many as the host memory
    holds (MemAvailable, at most 240 GiB) at the workload's peak per worker."""
    cores = len(os.sched_getaffinity(0))
    avail = 240 * 2.0 ** 30
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemAvailable:"):
                avail = min(avail, float(line.split()[1]) * 1024.0 - 8e9)
    except OSError:
        pass
    return max(1, min(cores, int(avail // _worker_bytes(w))))


def cpu_baseline(cfg_id: int, seconds: float):
    """The oracle as it stands on the host cores: a strided sample of the
    workload's points, one per task, in rounds of at least one point per
    process until about `seconds` have passed (a workload whose single point
    takes longer runs one round)."""
    import multiprocessing as mp
    from synth import CONFIGS
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    w = CONFIGS[cfg_id]
    cores = _oracle_pool_size(w)
    if w.nested:
        return cpu_baseline_nested(cfg_id, seconds, cores)
    n_total = w.n_samples()
    order = [(i * 7919) % n_total for i in range(n_total)]
    idx, vals = [], []
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        take = cores
        while len(idx) < n_total:
            chunk = [(cfg_id, *_flat(w, i)) for i in order[len(idx):len(idx) + take]]
            got = []
            for v in pool.imap(_oracle_worker, chunk, chunksize=1):
                got.append(v)
                if len(got) % cores == 0 or len(got) == len(chunk):
                    _log(f"oracle: {len(idx) + len(got)} samples, "
                         f"{time.perf_counter() - t0:.0f} s")
            vals += got
            idx += chunk
            el = time.perf_counter() - t0
            if el >= seconds:
                break
            rate = len(idx) / el
            take = max(cores, int((seconds - el) * rate))
    dt = time.perf_counter() - t0
    assert all(math.isfinite(v[0]) for v in vals)
    count = len(idx)
    kind = "two-grid eigen-samples" if len(w.levels) == 1 else "level samples Y_l"
    base = {"value": count / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{count} of the {n_total} {kind} of the workload (strided indices), "
                      f"scipy/SuperLU FP64, {cores} processes (affinity cores, capped by host "
                      f"memory at {_worker_bytes(w) / 1e9:.1f} GB each), {dt:.1f} s"}
    return base, [i[1:] for i in idx], vals


def golden_points(cfg_id: int):
    """Stored oracle values of workload cfg_id (tests/golden, written by a
    script that calls only the oracle): ([(level, r, k)], [(Y, lambda)])."""
    if cfg_id != 5:
        return [], []
    idx, ref = [], []
    for name in ("large_twogrid_samples.json", "large_twogrid_chain.json"):
        p = os.path.join(ROOT, "tests", "golden", name)
        if not os.path.exists(p):
            continue
        for x in json.load(open(p))["samples"]:
            idx.append((0, int(x["r"]), int(x["k"])))
            ref.append((float(x["lambda"]), float(x["lambda"])))
    return idx, ref


def per_level(ctx, m, w, opts, idx=None, ref=None, bound=None):
    """Untimed pass over every level with mlqmc_eig_level and the bench
    options: samples/s per level and, given oracle values of the CPU-baseline
    sample, the per-sample error of Y_l (relative to lambda) against them."""
    import numpy as np
    import torch
    out, errs = [], []
    ys = {}
    for l, lv in enumerate(w.levels):
        n = w.R * lv.N
        Y = np.empty((n, max(lv.s_fine, 1)))
        for r in range(w.R):
            ctx.lattice_points(lv.N, w.z(l), w.shifts(l)[r], 0, lv.N, Y[r * lv.N:(r + 1) * lv.N])
        lam, lp = np.empty(n), np.empty(n)
        fl = np.zeros(n, np.uint8)
        prev = lp if lv.n_prev else None
        ctx.eig_level(_lv6(lv), Y, lam, fl, lam_prev=prev, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.eig_level(_lv6(lv), Y, lam, fl, lam_prev=prev, opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.append({"level": l, "h": f"1/{lv.n_fine}", "H": f"1/{lv.n_coarse}" if lv.n_coarse else None,
                    "s": lv.s_fine, "samples": n, "samples_per_s": round(n / dt, 1),
                    "flagged": int((fl != 0).sum())})
        ys[l] = (lam - lp) if lv.n_prev else lam, lam
    acc = None
    if idx is not None:
        lev_err = {}
        for (l, r, k), (yref, lref) in zip(idx, ref):
            yv = ys[l][0][r * w.levels[l].N + k]
            errs.append(abs(yv - yref) / abs(lref))
            lev_err.setdefault(l, []).append(errs[-1])
        for x in out:
            le = lev_err.get(x["level"])
            x["max_rel_err"] = float(max(le)) if le else None
            x["oracle_samples"] = len(le) if le else 0
        e = np.asarray(errs)
        acc = {"max_rel_err": float(e.max()), "median_rel_err": float(np.median(e)),
               "samples": int(e.size), "flagged": int(sum(x["flagged"] for x in out)),
               "bound": bound or (1e-10 if opts.prec == m.MLQMC_FP64 else 1e-8),
               "quantity": "Y_l = lambda^l - lambda^(l-1), error relative to lambda^l"
               if len(w.levels) > 1 else "lambda"}
    return out, acc


def per_level_nested(ctx, m, w, opts, idx=None, ref=None):
    """Untimed nested estimate with the per-point values: flags and, given
    oracle values of the CPU-baseline sample, the per-sample error of Y_l."""
    import numpy as np
    levels = [_lv6(lv) for lv in w.levels]
    Ns = [lv.N for lv in w.levels]
    st, Q, Qh, V, est, lam = ctx.estimate_nested(levels, Ns, w.R, w.z_shared(),
                                                 w.shifts_shared(), opts=opts, lam_out=True)
    out = [{"level": l, "h": f"1/{lv.n_fine}",
            "H": f"1/{lv.n_coarse}" if lv.n_coarse else None, "s": lv.s_fine,
            "samples": w.R * lv.N, "Qhat": float(Qh[l]), "V": float(V[l])}
           for l, lv in enumerate(w.levels)]
    acc = None
    if idx is not None:
        errs, lev_err = [], {}
        for (l, r, k), (yref, lref) in zip(idx, ref):
            yv = lam[l][r, k] - (lam[l - 1][r, k] if l else 0.0)
            errs.append(abs(yv - yref) / abs(lref))
            lev_err.setdefault(l, []).append(errs[-1])
        for x in out:
            le = lev_err.get(x["level"])
            x["max_rel_err"] = float(max(le)) if le else None
            x["oracle_samples"] = len(le) if le else 0
        e = np.asarray(errs)
        acc = {"max_rel_err": float(e.max()), "median_rel_err": float(np.median(e)),
               "samples": int(e.size), "flagged": int(st != m.MLQMC_OK),
               "bound": 1e-10 if opts.prec == m.MLQMC_FP64 else 1e-8,
               "quantity": "Y_l = lambda^l - lambda^(l-1), error relative to lambda^l"}
    return out, acc


def lds_update_flops(n: int, rows: int, its: int, reaction: bool) -> int:
    """Algorithmic FP64 flops of one two-grid update on mesh 1/n in LDS
    (k_tg_small) that took `its` projected-PCG iterations, counted per
    interior node (one add or multiply = 1; a divide = 1):

    * operator (A [+ R]) x: 11 (4 differences, 4 products, 3 sums), with the
      reaction 30 (six sums x_k + x_j, six products, 5 sums, the h^2/12 scale,
      1 sum); mass M x: 8;
    * V-cycle, per node of each level 1/n .. 1/2: three Jacobi sweeps (op + 4),
      the first from zero (2), the residual (op + 1), restriction (2) and
      prolongation (3): 4 op + 20;
    * PCG iteration on the top level: q = (A - mu M) p (op + mass + 2), three
      dots (6), three tracking dots (6), t and r updates (6), three dots after
      the V-cycle (6), p update (4): op + 38, plus one V-cycle;
    * per sample: the weights (2 rows segs P, segs = 5 with the reaction, 2
      without), the initial residual and V-cycle, and two Rayleigh quotients
      (2 (op + mass + 4))."""
    D = (n - 1) ** 2
    P = (n + 1) * n + 1
    op = 30 if reaction else 11
    mass = 8
    levels, c = 0, n
    while c >= 2:
        levels += (c - 1) ** 2
        c //= 2
    vcycle = (4 * op + 20) * levels
    weights = 2 * rows * (5 if reaction else 2) * P
    init = (op + mass + 3) * D + vcycle + 8 * D
    rq = 2 * (op + mass + 4) * D
    return weights + init + rq + its * ((op + 38) * D + vcycle)


def plain_vs_enhanced(m, w, opts):
    """Time of each level's values with the enhanced method (Algorithm 2: the
    two-grid update from the coarse pair, warm-started RQ chains) and with
    plain MLQMC (a direct, cold-started eigensolve on the level's fine and
    previous meshes), on the same points; the paper compares the two in its
    numerical section.  Direct solves run up to 1/64 (Problem 2: 1/32), so
    levels beyond are skipped."""
    import numpy as np
    import torch
    ctx = m.Context(w.family(), device=0)

    def timed(L, Y, warm, reps=3):
        n = Y.shape[0]
        lam, lp = np.empty(n), np.empty(n)
        fl = np.zeros(n, np.uint8)
        prev = lp if L[4] else None
        ctx.eig_level(L, Y, lam, fl, lam_prev=prev, warm_chain=warm, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.eig_level(L, Y, lam, fl, lam_prev=prev, warm_chain=warm, opts=opts)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, float(((lam - lp) if L[4] else lam).mean())

    out, te_all, tp_all = [], 0.0, 0.0
    for l, lv in enumerate(w.levels):
        if lv.n_fine > (32 if w.problem == 2 else 64):
            continue
        n = w.R * lv.N
        Y = np.empty((n, max(lv.s_fine, 1)))
        for r in range(w.R):
            ctx.lattice_points(lv.N, w.z(l), w.shifts(l)[r], 0, lv.N, Y[r * lv.N:(r + 1) * lv.N])
        enh = _lv6(lv)
        plain = (lv.n_fine, lv.s_fine, 0, 0, lv.n_prev, lv.s_prev)
        te, ye = timed(enh, Y, 1)
        tp, yp = timed(plain, Y, 0)
        te_all += te
        tp_all += tp
        out.append({"level": l, "h": f"1/{lv.n_fine}", "samples": n,
                    "enhanced_ms": round(te * 1e3, 3), "plain_ms": round(tp * 1e3, 3),
                    "plain_over_enhanced": round(tp / te, 3),
                    "mean_Y_enhanced": ye, "mean_Y_plain": yp})
    ctx.close()
    return {"workload": w.name, "precision": "fp64" if opts.prec == m.MLQMC_FP64 else "mixed",
            "levels": out, "plain_over_enhanced": round(tp_all / max(te_all, 1e-30), 3)}


def rqi_sample_flops(n: int, rows: int, rq: int, lin: int, reaction: bool) -> int:
    """Algorithmic FP64 flops of one warm-started RQ eigensolve on mesh 1/n in
    LDS (k_rqi) that took `rq` RQ steps and `lin` inner PCG iterations in all,
    with the per-node counts of lds_update_flops: the weights, the starting
    Rayleigh quotient, and per RQ step one correction solve's set-up (the
    initial residual, V-cycle and dots) and one Rayleigh quotient with its
    normalisation (op + mass + 5 per node), plus `lin` PCG iterations."""
    D = (n - 1) ** 2
    P = (n + 1) * n + 1
    op = 30 if reaction else 11
    mass = 8
    levels, c = 0, n
    while c >= 2:
        levels += (c - 1) ** 2
        c //= 2
    vcycle = (4 * op + 20) * levels
    weights = 2 * rows * (5 if reaction else 2) * P
    setup = (op + mass + 3) * D + vcycle + 8 * D
    rq_eval = (op + mass + 5) * D
    return (weights + rq_eval + rq * (setup + rq_eval) +
            lin * ((op + 38) * D + vcycle))


def lds_words(n: int, its: int, rq: int, reaction: bool, solve: str) -> int:
    """LDS traffic of one per-sample solve on mesh 1/n, in array elements read
    or written (the same operation structure as the flop counts), per
    interior node:

    * operator A [+ R] x: 5 x reads and 4 weights (with the reaction 7 x reads
      and 10 weights), 1 write: 10 (18); mass M x: 7 reads + 1 write = 8;
    * V-cycle, per node of each level: the first sweep (right-hand side,
      weights, write: 6 (12)), three sweeps (operator reads + rhs + write:
      11 (19) each), the residual (operator reads + rhs: 10 (18)), the
      restriction (2) and the prolongation (4): 55 (93);
    * PCG iteration on the top level: q = (A - mu M) p (12 (18)), the six
      dots and the t, r updates (13), the three dots after the V-cycle (3),
      the p update (4): 32 (38), plus one V-cycle;
    * per solve: staging the weights (2 (5) writes per node), the initial
      residual (20 (26)) and V-cycle, and two Rayleigh quotients (16 (24)
      each); an RQ eigensolve adds, per RQ step, a correction set-up and a
      quotient.
    solve = "update" (k_tg_small, `its` PCG iterations) or "rqi" (k_rqi,
    `rq` RQ steps and `its` inner iterations in all)."""
    D = (n - 1) ** 2
    levels, c = 0, n
    while c >= 2:
        levels += (c - 1) ** 2
        c //= 2
    vcyc = (93 if reaction else 55) * levels
    stage = (5 if reaction else 2) * D
    init = (26 if reaction else 20) * D + vcyc
    rq_eval = (24 if reaction else 16) * D
    it = (38 if reaction else 32) * D + vcyc
    if solve == "update":
        return stage + init + 2 * rq_eval + its * it
    return stage + rq_eval + rq * (init + rq_eval) + its * it


def rqi_step_flops(ctx, m, w, opts, with_words=False):
    """Algorithmic flops of every k_rqi launch of one step of a direct-only
    workload, from the RQ-step and inner-iteration counts of the same points
    (an untimed pass)."""
    import numpy as np
    total = 0
    words = [0]
    reaction = w.problem == 2
    for l, lv in enumerate(w.levels):
        n = w.R * lv.N
        Y = np.empty((n, max(lv.s_fine, 1)))
        for r in range(w.R):
            ctx.lattice_points(lv.N, w.z(l), w.shifts(l)[r], 0, lv.N, Y[r * lv.N:(r + 1) * lv.N])
        lam = np.empty(n)
        fl = np.zeros(n, np.uint8)
        for nm, sm in [(lv.n_fine, lv.s_fine)] + ([(lv.n_prev, lv.s_prev)] if lv.n_prev else []):
            rq = np.zeros(n, np.int32)
            li = np.zeros(n, np.int32)
            ctx.eig_level((nm, sm, 0, 0, 0, 0), np.ascontiguousarray(Y[:, :sm]), lam, fl,
                          rq_iters=rq, lin_iters=li, opts=opts)
            rows = sm + 1 if reaction else sm
            for q, k in zip(rq.tolist(), li.tolist()):
                total += rqi_sample_flops(nm, rows, q, k, reaction)
                words[0] += lds_words(nm, k, q, reaction, "rqi")
    return (total, words[0]) if with_words else total


def lds_step_flops(ctx, m, w, opts, with_words=False):
    """Algorithmic flops of every k_tg_small launch of one step of workload w,
    from the PCG iteration counts of the same points (an untimed pass; the
    solves are deterministic).  mlqmc_eig_level reports the coarse eigensolve's
    inner iterations plus the fine update's; the direct coarse eigensolve alone
    on the same points gives the first part (on Problem 2 with the one-step
    refinement of its vectors that the two-grid levels apply, which a
    requested G switches on)."""
    import numpy as np
    total = 0
    words = 0
    reaction = w.problem == 2
    for l, lv in enumerate(w.levels):
        if not lv.n_coarse:
            continue
        n = w.R * lv.N
        Y = np.empty((n, max(lv.s_fine, 1)))
        for r in range(w.R):
            ctx.lattice_points(lv.N, w.z(l), w.shifts(l)[r], 0, lv.N, Y[r * lv.N:(r + 1) * lv.N])
        lam = np.empty(n)
        fl = np.zeros(n, np.uint8)
        base = np.zeros(n, np.int32)
        Yc = np.ascontiguousarray(Y[:, :lv.s_coarse])
        ctx.eig_level((lv.n_coarse, lv.s_coarse, 0, 0, 0, 0), Yc, lam, fl, lin_iters=base,
                      opts=opts, g=np.empty(n) if reaction else None)
        updates = [(lv.n_fine, lv.s_fine)]
        if lv.n_prev and not (lv.n_prev == lv.n_coarse and lv.s_prev == lv.s_coarse):
            updates.append((lv.n_prev, lv.s_prev))
        for nm, sm in updates:
            if nm > 32:
                continue  # the batched kernels: not this kernel class
            li = np.zeros(n, np.int32)
            ctx.eig_level((nm, sm, lv.n_coarse, lv.s_coarse, 0, 0),
                          np.ascontiguousarray(Y[:, :sm]), lam, fl, lin_iters=li, opts=opts)
            its = (li - base).astype(np.int64)
            if its.min() < 0:
                raise RuntimeError("iteration counts of the coarse eigensolve differ")
            rows = sm + 1 if reaction else sm
            total += n * lds_update_flops(nm, rows, 0, reaction)
            total += int(its.sum()) * (lds_update_flops(nm, rows, 1, reaction) -
                                       lds_update_flops(nm, rows, 0, reaction))
            words += n * lds_words(nm, 0, 0, reaction, "update")
            words += int(its.sum()) * (lds_words(nm, 1, 0, reaction, "update") -
                                       lds_words(nm, 0, 0, reaction, "update"))
    return (total, words) if with_words else total


def _traffic(kernel: str, prec: str = "fp64", cfg: int = 2):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel, precision and workload, or None when there is none or the
    kernel source changed since the counters were taken."""
    name = f"traffic_{kernel}" + ("" if prec == "fp64" else f"_{prec}")
    if cfg != 2:
        name += f"_cfg{cfg}"
    p = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        src = open(os.path.join(ROOT, d["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != d["source_sha256"]:
            return None
        return float(d["bytes_per_launch"])
    except Exception:
        return None


def _workload_opts(m, prec: str, **kw):
    return m.default_opts(prec=m.MLQMC_MIXED if prec == "mixed" else m.MLQMC_FP64, **kw)


def _default_class(w) -> str:
    per_sample = all(lv.n_fine <= 32 for lv in w.levels)
    if not any(lv.n_coarse for lv in w.levels):
        return "rqi"
    return "lds" if per_sample else "post"


KCLS_NAME = {"post": "k_post", "pre": "k_pre", "apply": "k_pupdate_apply",
             "coeff": "k_expand_mfma", "lds": "k_tg_small", "rqi": "k_rqi"}


def timed_leg(ctx, m, w, opts, steps: int, warmup: int, kernel_class: str):
    """`warmup` untimed and `steps` timed estimates of workload w (one step =
    one mlqmc_estimate over all its levels), the launches of `kernel_class`
    in which every sample is active bracketed by HIP events on the library's
    stream.  Returns samples/s, ms per step, the last estimate and the live
    kernel timing."""
    import torch
    levels = [_lv6(lv) for lv in w.levels]
    Ns = [lv.N for lv in w.levels]
    if w.nested:
        z_sh, sh_sh = w.z_shared(), w.shifts_shared()
    else:
        zs = [w.z(l) for l in range(len(w.levels))]
        shs = [w.shifts(l) for l in range(len(w.levels))]

    def step():
        if w.nested:
            st, Q, Qh, V, est, _ = ctx.estimate_nested(levels, Ns, w.R, z_sh, sh_sh, opts=opts)
        else:
            st, Q, Qh, V, est = ctx.estimate(levels, Ns, w.R, zs, shs, opts=opts)
        if st != m.MLQMC_OK:
            raise RuntimeError(f"estimate flagged samples (status {st})")
        return est

    for _ in range(warmup):
        step()
    kcls = {"post": m.K_SMOOTH, "pre": m.K_PRE, "apply": m.K_APPLY, "coeff": m.K_COEFF,
            "lds": m.K_TG_LDS, "rqi": m.K_COARSE}[kernel_class]
    ctx.set_timing(kcls)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est = None
    for _ in range(steps):
        est = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms, kbytes, kflops = ctx.get_timing(flops=True)
    ctx.set_timing(m.K_NONE)
    return {"value": w.n_samples() * steps / dt, "ms_per_step": 1e3 * dt / steps, "est": est,
            "launches": launches, "kms": kms, "kbytes": kbytes, "kflops": kflops,
            "steps": steps}


def roofline(ctx, m, w, opts, prec: str, kernel_class: str, leg, cfg: int):
    """The roofline object of one kernel class from a timed leg: achieved =
    algorithmic bytes (or flops) per launch / live average launch time."""
    launches, kms, kbytes, steps = leg["launches"], leg["kms"], leg["kbytes"], leg["steps"]
    if not (launches > 0 and kms > 0):
        return None
    kname = KCLS_NAME[kernel_class]
    avg_ms = kms / launches
    if kernel_class in ("rqi", "lds"):
        # LDS-resident solvers: vector arithmetic on data in LDS, against the
        # vector peak of the precision they compute in; beside it the LDS
        # traffic of the same solves against the LDS peak (neither bounds
        # them: they wait on LDS latency and workgroup barriers)
        fl, words = (rqi_step_flops if kernel_class == "rqi" else lds_step_flops)(
            ctx, m, w, opts, with_words=True)
        flops_per_launch = fl * steps / launches
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        peak = PEAK_FP64_VALU_TFS if prec == "fp64" else PEAK_FP32_VALU_TFS
        lds_bytes = words * (8 if prec == "fp64" else 4) * steps / launches
        lds_rate = lds_bytes / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "avg_launch_us": round(avg_ms * 1e3, 2), "launches": launches,
                "algorithmic_flops_per_launch": flops_per_launch,
                "lds": {"achieved": round(lds_rate, 3), "peak": PEAK_LDS_TBS, "unit": "TB/s",
                        "frac": round(lds_rate / PEAK_LDS_TBS, 4),
                        "bytes_per_launch": lds_bytes}}
    if kernel_class == "coeff":
        # the coefficient expansion: the product the library formed (the dense
        # Y Phi, 2 s E flops per sample, or the separable one, two element
        # products of kx terms per node plus the row sums), both on FP64 MFMA;
        # flops from the library's model
        flops_per_launch = leg["kflops"] / launches
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        fam = w.family()

        def separable(s):
            kx, ky = int(max(fam["k1"][:s])), int(max(fam["k2"][:s]))
            return 4 * kx < s and kx <= 32 and kx * ky <= 1024

        dense = w.problem == 2 or not all(separable(lv.s_fine) for lv in w.levels if lv.n_coarse)
        peak = PEAK_FP64_MFMA_TFS
        tkey = kname
        if not dense:
            kname, tkey = "k_sep_march+k_sep_rows", "k_sep"
        return {"bound": "mfma", "kernel": kname,
                "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "traffic": _traffic(tkey, prec, cfg), "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches": launches, "algorithmic_flops_per_launch": flops_per_launch,
                "hbm_GBs": round(kbytes / launches / (avg_ms * 1e-3) / 1e9, 1)}
    bytes_per_launch = kbytes / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = _traffic(kname, prec, cfg)
    roof = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic, "avg_launch_us": round(avg_ms * 1e3, 2), "launches": launches,
            "algorithmic_bytes_per_launch": bytes_per_launch}
    if traffic:
        # the counted HBM bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)
        # over the same live launch time: what the memory system moved
        tg = traffic / (avg_ms * 1e-3) / 1e9
        roof["traffic_GBs"] = round(tg, 1)
        roof["traffic_frac"] = round(tg / PEAK_HBM_GBS, 4)
    return roof


def rq_counts(ctx, m, w, opts, count: int = 256):
    """RQ iterations of the coarse eigensolve of the first two-grid level on
    `count` consecutive points of shift 0: at the paper's criterion (section 5:
    |sigma_k - sigma_{k-1}| <= 5e-8, exact inner solves, here to 1e-12) from
    the fixed start and from the previous point's eigenvector (section 4.3),
    and with the library's own settings (relative 1e-8, inner solves to the
    bench options' rq_lin_rtol) from the previous point."""
    import numpy as np
    lv = next((lv for lv in w.levels if lv.n_coarse), None)
    if lv is None or w.nested:
        return None
    l = list(w.levels).index(lv)
    count = min(count, lv.N)
    full = np.empty((count, lv.s_fine))
    ctx.lattice_points(lv.N, w.z(l), w.shifts(l)[0], 0, count, full)
    Y = np.ascontiguousarray(full[:, :lv.s_coarse]) if lv.s_coarse else np.zeros((count, 1))
    out = {"mesh": f"1/{lv.n_coarse}", "S": lv.s_coarse, "points": count}
    runs = [("paper_cold", 0, m.default_opts(prec=opts.prec, eig_atol=5e-8, rq_lin_rtol=1e-12,
                                             max_lin_iter=400, chain_len=count)),
            ("paper_nearby", 1, m.default_opts(prec=opts.prec, eig_atol=5e-8, rq_lin_rtol=1e-12,
                                               max_lin_iter=400, chain_len=count)),
            ("library_nearby", 1, m.default_opts(prec=opts.prec, chain_len=count))]
    for name, warm, o in runs:
        lam = np.empty(count)
        fl = np.zeros(count, np.uint8)
        rq = np.zeros(count, np.int32)
        ctx.eig_level((lv.n_coarse, lv.s_coarse, 0, 0, 0, 0), Y, lam, fl, rq_iters=rq,
                      warm_chain=warm, opts=o)
        out[name] = {"mean": round(float(rq.mean()), 3),
                     "histogram": {int(k): int(v) for k, v in
                                   zip(*np.unique(rq, return_counts=True))},
                     "flagged": int((fl != 0).sum())}
    return out


def _brief(roof):
    if not roof:
        return None
    keep = ("kernel", "achieved", "peak", "unit", "frac", "avg_launch_us", "launches",
            "traffic_frac")
    return {k: roof[k] for k in keep if k in roof}


def main():
    a = _parse()
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU only; --gpus {a.gpus} is not supported "
              "(samples would shard across GPUs by warm-start chain, with one all-reduce of "
              "the per-level sums)",
              file=sys.stderr)
        return 2
    import numpy as np  # noqa: F401
    import torch
    if a.copy_probe:
        # plain copy kernel of known size: calibrates the HBM byte counters
        n = a.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 8 * n, "copies": 3}), flush=True)
        return 0
    import paper_2103_03407_amd as m
    from synth import CONFIGS

    w = CONFIGS[a.cfg]
    torch.cuda.init()
    if a.plain_vs_enhanced:
        print(json.dumps(plain_vs_enhanced(m, w, _workload_opts(m, a.prec))), flush=True)
        return 0
    extras = (not a.no_extras) and a.cfg in (2, 5)
    ctx = m.Context(w.family(), device=0)
    tuned = ctx.apply_tuning()  # the autotuner's table for this device, if shipped
    opts = _workload_opts(m, a.prec)
    kclass = a.kernel_class or _default_class(w)
    _log(f"{w.name} {a.prec}: {a.warmup} warm-up + {a.steps} timed steps")
    main_leg = timed_leg(ctx, m, w, opts, a.steps, a.warmup, kclass)
    roof = roofline(ctx, m, w, opts, a.prec, kclass, main_leg, a.cfg)

    extra = {}
    legs = {}
    if extras:
        # the other batched kernels of the same step (one timed step each)
        rates = {}
        for kc in ("pre", "apply", "coeff"):
            _log(f"{w.name} {a.prec}: kernel class {kc}")
            leg = timed_leg(ctx, m, w, opts, 1, 0, kc)
            rates[KCLS_NAME[kc]] = _brief(roofline(ctx, m, w, opts, a.prec, kc, leg, a.cfg))
        extra["kernels"] = rates
        # mixed precision, and FP64 stopped at the mixed path's tolerances
        # (equal accuracy), on the same workload
        k2 = min(a.steps, 5)
        other = "mixed" if a.prec == "fp64" else "fp64"
        o_other = _workload_opts(m, other)
        _log(f"{w.name} {other}: 1 warm-up + {k2} timed steps")
        legs[other] = (o_other, timed_leg(ctx, m, w, o_other, k2, 1, kclass))
        extra["rq_iterations"] = rq_counts(ctx, m, w, opts)
        o_eq = _workload_opts(m, "fp64", lam_rtol=5e-10, lin_rtol=1e-7)
        _log(f"{w.name} fp64 at the mixed tolerances: 1 warm-up + {k2} timed steps")
        legs["fp64_mixed_tol"] = (o_eq, timed_leg(ctx, m, w, o_eq, k2, 1, kclass))

    cpu = None
    idx = ref = None
    if not a.no_cpu_baseline:
        _log(f"oracle CPU baseline ({_oracle_pool_size(w)} processes)")
        cpu, idx, ref = cpu_baseline(a.cfg, a.cpu_seconds)
    gi, gr = golden_points(a.cfg)
    aidx = (idx or []) + gi
    aref = (ref or []) + gr
    _log("accuracy pass")
    if a.no_accuracy:
        levels_out, acc = None, None
    elif w.nested:
        levels_out, acc = per_level_nested(ctx, m, w, opts, idx, ref)
    else:
        levels_out, acc = per_level(ctx, m, w, opts, aidx or None, aref or None)
    if acc is not None and gi:
        acc["golden_samples"] = len(gi)
    if extras:
        for name, (o, leg) in legs.items():
            lo, lacc = per_level(ctx, m, w, o, aidx or None, aref or None, bound=1e-8)
            prec_name = "mixed" if o.prec == m.MLQMC_MIXED else "fp64"
            extra[name] = {"samples_per_s": round(leg["value"], 1),
                           "ms_per_step": round(leg["ms_per_step"], 3), "steps": leg["steps"],
                           "estimate": leg["est"][0],
                           "roofline": _brief(roofline(ctx, m, w, o, prec_name, kclass, leg,
                                                       a.cfg)),
                           "accuracy_vs_oracle": lacc}
        if "mixed" in extra:
            fp64_v = main_leg["value"] if a.prec == "fp64" else legs["fp64"][1]["value"]
            mixed_v = legs["mixed"][1]["value"] if a.prec == "fp64" else main_leg["value"]
            extra["mixed_over_fp64"] = round(mixed_v / fp64_v, 3)
            extra["mixed_over_fp64_at_mixed_tolerances"] = round(
                mixed_v / legs["fp64_mixed_tol"][1]["value"], 3)
    ctx.close()
    if extras and a.cfg != 2:
        # the two-grid 1/32 -> 1/128 workload (s = 64), both precisions
        w2 = CONFIGS[2]
        c2 = m.Context(w2.family(), device=0)
        c2.apply_tuning()
        small = {}
        for prec in ("fp64", "mixed"):
            _log(f"{w2.name} {prec}")
            o2 = _workload_opts(m, prec)
            leg = timed_leg(c2, m, w2, o2, max(a.steps, 5), 1, "post")
            small[prec] = {"samples_per_s": round(leg["value"], 1),
                           "ms_per_step": round(leg["ms_per_step"], 3),
                           "roofline": _brief(roofline(c2, m, w2, o2, prec, "post", leg, 2))}
        c2.close()
        extra[w2.name] = small

    out = {
        "metric": "two-grid eigen-samples/sec per level; stencil HBM GB/s in roofline"
                  if w.problem == 1 else
                  "two-grid eigen-samples/sec per level (Problem 2, islands); "
                  + ("LDS-update TFLOP/s" if kclass in ("lds", "rqi") else "stencil HBM GB/s")
                  + " in roofline",
        "value": round(main_leg["value"], 1), "unit": "samples/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(main_leg["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.prec == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "problem": w.problem, "levels": len(w.levels),
                   "h": [f"1/{lv.n_fine}" for lv in w.levels],
                   "H": [f"1/{lv.n_coarse}" if lv.n_coarse else None for lv in w.levels],
                   "s": [lv.s_fine for lv in w.levels], "S": [lv.s_coarse for lv in w.levels],
                   "N": [lv.N for lv in w.levels], "R": w.R,
                   "samples_per_step": w.n_samples(), "nested_shared_shifts": bool(w.nested),
                   "estimate": main_leg["est"][0], "variance": main_leg["est"][1]},
        "roofline": roof, "cpu_baseline": cpu, "accuracy_vs_oracle": acc,
        "per_level": levels_out, "tuning_entries_applied": tuned,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    return 0


def _log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    sys.exit(main())
