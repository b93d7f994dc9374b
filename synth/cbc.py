"""Rank-1 lattice generating vectors by a plain component-by-component search.

The paper builds its randomly shifted lattice rules (eq. rqmc) from a
published embedded generating vector that is not available here, so the
workloads use vectors built by the CBC algorithm of the quasi-Monte Carlo
background section instead.  The criterion is the shift-averaged worst-case
error in the unanchored weighted Sobolev space of eq. (W-norm) with product
weights gamma_j:

    e^2(z) = -1 + (1/N) sum_{k<N} prod_j (1 + gamma_j B2({k z_j / N})),
    B2(x) = x^2 - x + 1/6,

minimised one component at a time over odd z_j < N (N a power of two),
with z_1 = 1.  Cost O(s N^2 / 2), done once per (N, s) and stored as text.

Run ``python -m synth.cbc`` to (re)write the stored vectors.
"""

from __future__ import annotations

import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_STORE = os.path.join(_HERE, "lattice")

# (N, s) pairs the workloads need; gamma_j = j^-2 throughout.
NEEDED = [(256, 16), (1024, 64), (16384, 16), (8192, 32), (2048, 64),
          (1024, 128), (256, 256), (1024, 512), (64, 8), (128, 16), (512, 32),
          (16384, 256), (4096, 32), (512, 256), (256, 512)]


def _b2(x: np.ndarray) -> np.ndarray:
    return x * x - x + 1.0 / 6.0


def cbc_vector(N: int, s: int, gamma_decay: float = 2.0) -> np.ndarray:
    """Plain CBC generating vector for N a power of two (int64[s])."""
    if N < 2 or N & (N - 1):
        raise ValueError("N must be a power of two >= 2")
    if s < 1:
        raise ValueError("s must be >= 1")
    k = np.arange(N, dtype=np.int64)
    cand = np.arange(1, N, 2, dtype=np.int64)
    z = np.zeros(s, dtype=np.int64)
    z[0] = 1
    prod = 1.0 + 1.0 * _b2(k / N)  # gamma_1 = 1
    chunk = max(1, (1 << 24) // N)
    for d in range(1, s):
        gam = float(d + 1) ** (-gamma_decay)
        best_val, best_z = np.inf, 1
        for c0 in range(0, cand.size, chunk):
            cc = cand[c0:c0 + chunk]
            omega = _b2(((np.outer(cc, k)) % N) / N)   # [chunk, N]
            err = omega @ prod                         # sum_k prod_k B2(...)
            i = int(np.argmin(err))
            if err[i] < best_val:
                best_val, best_z = float(err[i]), int(cc[i])
        z[d] = best_z
        prod = prod * (1.0 + gam * _b2(((k * best_z) % N) / N))
    return z


def _path(N: int, s: int) -> str:
    return os.path.join(_STORE, f"cbc_N{N}_s{s}.txt")


def lattice_vector(N: int, s: int) -> np.ndarray:
    """Stored CBC vector for (N, s) if present (or a longer stored one with the
    same N, whose leading components are the CBC vector for s); else compute."""
    p = _path(N, s)
    if os.path.exists(p):
        return np.loadtxt(p, dtype=np.int64, ndmin=1)
    if os.path.isdir(_STORE):
        for name in sorted(os.listdir(_STORE)):
            if name.startswith(f"cbc_N{N}_s"):
                s_have = int(name.split("_s")[1].split(".")[0])
                if s_have >= s:
                    return np.loadtxt(os.path.join(_STORE, name),
                                      dtype=np.int64, ndmin=1)[:s]
    return cbc_vector(N, s)


def main(argv=None) -> int:
    """Writes the stored vectors: all of NEEDED, or the (N, s) pairs given as
    N:s arguments."""
    os.makedirs(_STORE, exist_ok=True)
    todo = NEEDED
    if argv:
        todo = [tuple(int(v) for v in a.split(":")) for a in argv]
    for N, s in todo:
        z = cbc_vector(N, s)
        np.savetxt(_path(N, s), z, fmt="%d",
                   header=f"CBC generating vector N={N} s={s} gamma_j=j^-2")
        print(f"N={N} s={s} z[:8]={z[:8].tolist()}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
