"""Writes oracle eigenvalues for a few lattice points of the large two-grid
workload (H = 1/64 -> h = 1/1024, s = 512, S = 23, coefficients decaying as
j^-2), where one oracle sample takes minutes.  Calls only oracle/ (and the
input generators in synth/); the GPU parity test reads the stored values.

    python tests/golden/make_large_samples.py   # writes large_twogrid_samples.json
"""

from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import qmc, twogrid  # noqa: E402
from synth import CONFIGS  # noqa: E402

CFG = 5
POINTS = [(0, 0), (0, 1), (3, 517), (7, 1023)]  # (shift r, lattice index k)


def one(rk):
    r, k = rk
    w = CONFIGS[CFG]
    lv = w.levels[0]
    y = qmc.lattice_point(w.z(0), lv.N, w.shifts(0)[r], k)
    lam, lam_H, _ = twogrid.two_grid(lv.n_fine, lv.s_fine, lv.n_coarse, lv.s_coarse, y, w.family())
    return {"r": r, "k": k, "lambda": lam, "lambda_H": lam_H}


def main():
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    with mp.get_context("fork").Pool(len(POINTS)) as pool:
        rows = pool.map(one, POINTS, chunksize=1)
    w = CONFIGS[CFG]
    out = {"workload": w.name, "source": "oracle.twogrid.two_grid (Algorithm 1), FP64, SuperLU",
           "samples": rows}
    with open(os.path.join(HERE, "large_twogrid_samples.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
