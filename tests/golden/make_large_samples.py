"""Writes oracle eigenvalues for lattice points of the large two-grid
workload (H = 1/64 -> h = 1/1024, s = 512, S = 23, coefficients decaying as
j^-2), where one oracle sample takes minutes.  Calls only oracle/ (and the
input generators in synth/); the GPU parity tests read the stored values.

    python tests/golden/make_large_samples.py            # large_twogrid_samples.json
    python tests/golden/make_large_samples.py --chain    # large_twogrid_chain.json

The first set is four scattered points; the second is eight consecutive
points of one shift, so that warm-start chains (each eigensolve started from
the previous point's eigenvector, section 4.3) can be checked at this size.
One worker holds about 9 GB; --workers caps the pool.
"""

from __future__ import annotations

import argparse
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
CHAIN = [(2, k) for k in range(300, 308)]       # consecutive points of shift 2


def one(rk):
    r, k = rk
    w = CONFIGS[CFG]
    lv = w.levels[0]
    y = qmc.lattice_point(w.z(0), lv.N, w.shifts(0)[r], k)
    lam, lam_H, _ = twogrid.two_grid(lv.n_fine, lv.s_fine, lv.n_coarse, lv.s_coarse, y, w.family())
    return {"r": r, "k": k, "lambda": lam, "lambda_H": lam_H}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--chain", action="store_true")
    ap.add_argument("--workers", type=int, default=4)
    a = ap.parse_args()
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    pts = CHAIN if a.chain else POINTS
    with mp.get_context("fork").Pool(min(a.workers, len(pts))) as pool:
        rows = pool.map(one, pts, chunksize=1)
    w = CONFIGS[CFG]
    out = {"workload": w.name, "source": "oracle.twogrid.two_grid (Algorithm 1), FP64, SuperLU",
           "samples": rows}
    name = "large_twogrid_chain.json" if a.chain else "large_twogrid_samples.json"
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
