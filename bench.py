#!/usr/bin/env python3
"""Throughput of the two-grid MLQMC eigen-sample path on one MI355X.

One step = one pass of the whole hot path over one batch: lattice points ->
coefficient expansion -> warm-started coarse RQ eigensolve -> prolongation ->
projected-PCG shifted fine solve -> Rayleigh quotient -> level accumulation,
i.e. one ``mlqmc_estimate`` call on the single-level two-grid workload
H = 1/32 -> h = 1/128, s = 64, S = 8, N = 1024 lattice points x R = 8 shifts
(8192 eigen-samples), all synthetic (CBC lattice, seeded shifts).

Prints one JSON line.  ``value`` = eigen-samples per second on one GPU.
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


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cfg", type=int, default=2, help="workload id (2: two-grid 1/32->1/128)")
    ap.add_argument("--kernel-class", default="post",
                    choices=["post", "pre", "apply", "coeff"],
                    help="kernel timed for the roofline (post: the dominant kernel)")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"],
                    help="fp64, or mixed (FP32 fine PCG/V-cycle, FP64 residual and RQ)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES bytes (counter calibration)")
    return ap.parse_args()


def _oracle_worker(args):
    # CPU baseline: the oracle as it stands, one sample per call
    cfg_id, idx = args
    from oracle import mlqmc, qmc
    from synth import CONFIGS
    w = CONFIGS[cfg_id]
    lv = w.levels[0]
    fam = w.family()
    r, k = divmod(int(idx), lv.N)
    y = qmc.lattice_point(w.z(0), lv.N, w.shifts(0)[r], k)
    return mlqmc.level_value(lv, y, fam).Y


def cpu_baseline(cfg_id: int, seconds: float):
    import multiprocessing as mp
    from synth import CONFIGS
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    cores = len(os.sched_getaffinity(0))
    cores = min(cores, 16)
    w = CONFIGS[cfg_id]
    n_total = w.R * w.levels[0].N
    # calibrate: one sample on this process, then size the sample to ~`seconds`
    t0 = time.perf_counter()
    _oracle_worker((cfg_id, 0))
    per = time.perf_counter() - t0
    count = max(cores, int(seconds * cores / max(per, 1e-3)))
    count = min(count, n_total)
    idx = [(cfg_id, (i * 7919) % n_total) for i in range(count)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        vals = pool.map(_oracle_worker, idx, chunksize=1)
    dt = time.perf_counter() - t0
    assert all(math.isfinite(v) for v in vals)
    base = {"value": count / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{count} of the {n_total} two-grid eigen-samples of the workload "
                      f"(strided lattice indices), scipy/SuperLU FP64, {cores} processes, "
                      f"{dt:.1f} s"}
    return base, [i for _, i in idx], vals


def accuracy(ctx, m, w, opts, idx, ref):
    """Per-sample relative eigenvalue error of the GPU path against the
    oracle values of the CPU-baseline sample (same lattice indices), from one
    untimed eig_level call over the whole workload with the bench options."""
    import numpy as np
    lv = w.levels[0]
    z, sh = w.z(0), w.shifts(0)
    n = w.R * lv.N
    Y = np.empty((n, lv.s_fine))
    for r in range(w.R):
        ctx.lattice_points(lv.N, z, sh[r], 0, lv.N, Y[r * lv.N:(r + 1) * lv.N])
    lam = np.empty(n)
    fl = np.zeros(n, np.uint8)
    level = (lv.n_fine, lv.s_fine, lv.n_coarse, lv.s_coarse, lv.n_prev, lv.s_prev)
    ctx.eig_level(level, Y, lam, fl, opts=opts)
    ref = np.asarray(ref)
    err = np.abs(lam[np.asarray(idx)] - ref) / np.abs(ref)
    return {"max_rel_err": float(err.max()), "median_rel_err": float(np.median(err)),
            "samples": int(err.size), "flagged": int((fl != 0).sum()),
            "bound": 1e-10 if opts.prec == m.MLQMC_FP64 else 1e-8}


def _traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
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


def main():
    a = _parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {a.gpus} is not supported "
              "(samples shard across GPUs by warm-start chain, see the design notes)",
              file=sys.stderr)
        return 2
    import numpy as np
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
    if len(w.levels) != 1:
        raise SystemExit("bench workload must be single-level")
    lv = w.levels[0]
    fam = w.family()
    torch.cuda.init()
    ctx = m.Context(fam, device=0)
    z, sh = w.z(0), w.shifts(0)
    level = (lv.n_fine, lv.s_fine, lv.n_coarse, lv.s_coarse, lv.n_prev, lv.s_prev)
    opts = m.default_opts(prec=m.MLQMC_MIXED if a.prec == "mixed" else m.MLQMC_FP64)
    n_samples = w.R * lv.N

    def step():
        st, Q, Qh, V, est = ctx.estimate([level], [lv.N], w.R, [z], [sh], opts=opts)
        if st != m.MLQMC_OK:
            raise RuntimeError(f"estimate flagged samples (status {st})")
        return est

    for _ in range(a.warmup):
        step()
    kcls = {"post": m.K_SMOOTH, "pre": m.K_PRE, "apply": m.K_APPLY,
            "coeff": m.K_COEFF}[a.kernel_class]
    ctx.set_timing(kcls)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est = None
    for _ in range(a.steps):
        est = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms, kbytes = ctx.get_timing()
    ctx.set_timing(m.K_NONE)
    ms_per_step = 1e3 * dt / a.steps
    value = n_samples * a.steps / dt

    kname = {"post": "k_post", "pre": "k_pre", "apply": "k_pupdate_apply",
             "coeff": "k_expand_mfma"}[a.kernel_class]
    roof = None
    if launches > 0 and kms > 0 and a.kernel_class == "coeff":
        # the coefficient product on FP64 MFMA: 2 s E flops per sample, every
        # sample expanded once per step (E = edge weights of the padded mesh)
        avg_ms = kms / launches
        ew = 2 * (lv.n_fine + 2) * lv.n_fine
        flops_per_launch = 2.0 * lv.s_fine * ew * n_samples * a.steps / launches
        achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": kname, "achieved": round(achieved, 2),
                "peak": PEAK_FP64_MFMA_TFS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_MFMA_TFS, 4), "traffic": _traffic(kname),
                "avg_launch_us": round(avg_ms * 1e3, 2), "launches": launches,
                "algorithmic_flops_per_launch": flops_per_launch,
                "hbm_GBs": round(kbytes / launches / (avg_ms * 1e-3) / 1e9, 1)}
    elif launches > 0 and kms > 0:
        avg_ms = kms / launches
        bytes_per_launch = kbytes / launches
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": _traffic(kname), "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches": launches, "algorithmic_bytes_per_launch": bytes_per_launch}

    cpu = acc = None
    if not a.no_cpu_baseline:
        cpu, idx, ref = cpu_baseline(a.cfg, a.cpu_seconds)
        acc = accuracy(ctx, m, w, opts, idx, ref)

    out = {
        "metric": "two-grid eigen-samples/sec per level; stencil HBM GB/s in roofline",
        "value": round(value, 1), "unit": "samples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.prec == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "h": f"1/{lv.n_fine}", "H": f"1/{lv.n_coarse}",
                   "s": lv.s_fine, "S": lv.s_coarse, "N": lv.N, "R": w.R,
                   "samples_per_step": n_samples, "estimate": est[0]},
        "roofline": roof, "cpu_baseline": cpu, "accuracy_vs_oracle": acc,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
