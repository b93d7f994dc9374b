"""Workload descriptions and seeded random shifts.

Each workload is a list of levels; a level fixes the fine mesh h = 1/n_fine
and truncation s, the coarse mesh H = 1/n_coarse and truncation S of the
two-grid-truncation method (Algorithm 1; n_coarse = 0 means a direct
eigensolve on the fine mesh), the previous-level mesh and truncation used for
the level difference (Algorithm 2; n_prev = 0 means no previous level), and
the number of lattice points N.  All levels share R random shifts.

Shifts are independent per level and per replicate, drawn uniformly on
[0, 1)^s from ``numpy.random.default_rng([210303407, cfg, level, r])``.

Problem 2 workloads (``problem=2``) use the islands family with the decays
(p_a, p_a', p_b, p_b') of the left panel of the paper's Problem 2 complexity
figure, (4/3, 2, 4/3, 2), and meshes h_l = 2^-(l+3) up to 1/32.

A nested workload (end of section 4.3) shares one set of R shifts (level 0's
seeds, s_max components) and one generating vector (the CBC vector for the
largest N with s_max components, enumerated as an embedded base-2 rule)
across its levels; levels l >= 1 take level 0's mesh and truncation as the
coarse pair.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .cbc import lattice_vector
from .family import coeff_family, islands_family, problem1_family

SEED_ROOT = 210303407


@dataclass(frozen=True)
class LevelSpec:
    n_fine: int
    s_fine: int
    n_coarse: int
    s_coarse: int
    n_prev: int
    s_prev: int
    N: int


@dataclass(frozen=True)
class Workload:
    name: str
    cfg_id: int
    precision: str            # "fp64" or "mixed"
    decay: float
    levels: tuple
    R: int
    description: str = ""
    a0: float = 1.0
    nested: bool = False
    problem: int = 1              # 1: benchmark / Problem 1 table; 2: islands
    decays: tuple = ()            # Problem 2: (p_a, p_a', p_b, p_b')
    p1_decay: float = 0.0         # > 0: Problem 1's own table (k1 = j, k2 = j + 1) with this decay

    @property
    def s_max(self) -> int:
        return max(lv.s_fine for lv in self.levels)

    def family(self):
        if self.problem == 2:
            return islands_family(self.s_max, *self.decays)
        if self.p1_decay > 0:
            return problem1_family(self.s_max, self.p1_decay)
        return coeff_family(self.s_max, decay=self.decay, a0=self.a0)

    def z(self, level: int) -> np.ndarray:
        lv = self.levels[level]
        return lattice_vector(lv.N, lv.s_fine)

    def shifts(self, level: int) -> np.ndarray:
        lv = self.levels[level]
        return shifts_for(self.cfg_id, level, self.R, lv.s_fine)

    def z_shared(self) -> np.ndarray:
        """Nested workloads: one vector for every level (first s_l used)."""
        return lattice_vector(max(lv.N for lv in self.levels), self.s_max)

    def shifts_shared(self) -> np.ndarray:
        """Nested workloads: R shifts with s_max components for every level."""
        return shifts_for(self.cfg_id, 0, self.R, self.s_max)

    def n_samples(self) -> int:
        return self.R * sum(lv.N for lv in self.levels)


def shifts_for(cfg_id: int, level: int, R: int, s: int) -> np.ndarray:
    """R independent uniform shifts in [0, 1)^s, float64 [R, s]."""
    out = np.empty((R, s), dtype=np.float64)
    for r in range(R):
        out[r] = np.random.default_rng([SEED_ROOT, cfg_id, level, r]).random(s)
    return out


def coarse_rule(n_fine: int) -> int:
    """H = sqrt(h) rounded to a power of two, ties to the finer mesh:
    h = 2^-k  ->  H = 2^-ceil(k/2)."""
    k = int(round(math.log2(n_fine)))
    return 1 << ((k + 1) // 2)


def coarse_trunc(s_fine: int, s0: int) -> int:
    """S_l = max(ceil(s_l^(1/2)), s_0) (two-grid level rule, section 4.3)."""
    return max(int(math.ceil(math.sqrt(s_fine) - 1e-12)), s0)


def _cfg4_levels():
    ns = [16, 32, 64, 128, 256]
    ss = [16, 32, 64, 128, 256]
    Ns = [1 << 14, 1 << 13, 1 << 11, 1 << 10, 1 << 8]
    out = []
    for l, (n, s, N) in enumerate(zip(ns, ss, Ns)):
        if l == 0:
            out.append(LevelSpec(n, s, 0, 0, 0, 0, N))
        else:
            out.append(LevelSpec(n, s, coarse_rule(n), coarse_trunc(s, ss[0]),
                                 ns[l - 1], ss[l - 1], N))
    return tuple(out)


def _islands_levels():
    """h_l = 1/8, 1/16, 1/32 (h_l = 2^-(l+3)), s_l = 16, 32, 64; H_l = 1/8 (the
    coarsest mesh that resolves the islands) and S_l = s_0 = 16 for l >= 1."""
    ns, ss, Ns = [8, 16, 32], [16, 32, 64], [1 << 13, 1 << 12, 1 << 11]
    out = [LevelSpec(8, 16, 0, 0, 0, 0, Ns[0])]
    for l in (1, 2):
        out.append(LevelSpec(ns[l], ss[l], 8, coarse_trunc(ss[l], ss[0]), ns[l - 1], ss[l - 1],
                             Ns[l]))
    return tuple(out)


P2_DECAYS = (4.0 / 3.0, 2.0, 4.0 / 3.0, 2.0)


def _islands_levels4():
    """_islands_levels plus level 3 on h = 1/64 (s = 128, N = 2^10)."""
    lv = list(_islands_levels())
    lv.append(LevelSpec(64, 128, 8, coarse_trunc(128, 16), 32, 64, 1 << 10))
    return tuple(lv)


def _islands_levels5():
    """_islands_levels4 plus level 4 on h = 1/128 (s = 256, N = 2^9)."""
    lv = list(_islands_levels4())
    lv.append(LevelSpec(128, 256, 8, coarse_trunc(256, 16), 64, 128, 1 << 9))
    return tuple(lv)


def _islands_levels6():
    """_islands_levels5 plus level 5 on h = 1/256 (s = 512, N = 2^8)."""
    lv = list(_islands_levels5())
    lv.append(LevelSpec(256, 512, 8, coarse_trunc(512, 16), 128, 256, 1 << 8))
    return tuple(lv)


def _nested_levels(base):
    """The levels of ``base`` with H_l = h_0 and S_l = s_0 for l >= 1."""
    l0 = base[0]
    return tuple([l0] + [LevelSpec(lv.n_fine, lv.s_fine, l0.n_fine, l0.s_fine, lv.n_prev,
                                   lv.s_prev, lv.N) for lv in base[1:]])


CONFIGS = {
    1: Workload("cfg1-direct-h32-s16", 1, "fp64", 2.5,
                (LevelSpec(32, 16, 0, 0, 0, 0, 256),), 4,
                "single-level QMC, direct eigensolve on h=1/32, s=16, N=256 x R=4"),
    2: Workload("cfg2-twogrid-H32-h128-s64", 2, "fp64", 2.5,
                (LevelSpec(128, 64, 32, 8, 0, 0, 1024),), 8,
                "single-level two-grid, H=1/32 -> h=1/128, s=64, S=8, N=1024 x R=8"),
    3: Workload("cfg3-direct-h32-s16-mixed", 3, "mixed", 2.5,
                (LevelSpec(32, 16, 0, 0, 0, 0, 256),), 4,
                "cfg1 in mixed precision"),
    4: Workload("cfg4-mlqmc-5level", 4, "fp64", 2.5, _cfg4_levels(), 8,
                "five-level two-grid MLQMC, h=1/16..1/256, s=16..256"),
    5: Workload("cfg5-twogrid-H64-h1024-s512", 5, "mixed", 2.0,
                (LevelSpec(1024, 512, 64, 23, 0, 0, 1024),), 8,
                "large fine level, H=1/64 -> h=1/1024, s=512, S=23, decay j^-2"),
    6: Workload("cfg6-mlqmc-5level-nested", 6, "fp64", 2.5, _nested_levels(_cfg4_levels()), 8,
                "cfg4's meshes, truncations and N_l with shared shifts, one embedded rule "
                "and H_l = h_0 = 1/16, S_l = s_0 = 16 (end of section 4.3)", nested=True),
    7: Workload("cfg7-islands-twogrid-H8-h32-s64", 7, "fp64", 0.0,
                (LevelSpec(32, 64, 8, 8, 0, 0, 1024),), 8,
                "Problem 2 (islands), single-level two-grid H=1/8 -> h=1/32, s=64, S=8, "
                "N=1024 x R=8", problem=2, decays=P2_DECAYS),
    8: Workload("cfg8-islands-mlqmc-3level", 8, "fp64", 0.0, _islands_levels(), 8,
                "Problem 2 (islands), three-level two-grid MLQMC, h=1/8..1/32, s=16..64, "
                "H=1/8, S=16", problem=2, decays=P2_DECAYS),
    9: Workload("cfg9-islands-mlqmc-4level", 9, "fp64", 0.0, _islands_levels4(), 8,
                "Problem 2 (islands), four-level two-grid MLQMC, h=1/8..1/64, s=16..128, "
                "H=1/8, S=16", problem=2, decays=P2_DECAYS),
    10: Workload("cfg10-islands-mlqmc-5level", 10, "fp64", 0.0, _islands_levels5(), 8,
                 "Problem 2 (islands), five-level two-grid MLQMC, h=1/8..1/128, s=16..256, "
                 "H=1/8, S=16", problem=2, decays=P2_DECAYS),
    11: Workload("cfg11-problem1-mlqmc-3level", 11, "fp64", 2.0, _islands_levels(), 8,
                 "Problem 1 of the numerical section (decay 2) on workload 8's meshes, "
                 "truncations and N_l", p1_decay=2.0),
    12: Workload("cfg12-islands-mlqmc-6level", 12, "fp64", 0.0, _islands_levels6(), 8,
                 "Problem 2 (islands), six-level two-grid MLQMC, h=1/8..1/256, s=16..512, "
                 "H=1/8, S=16", problem=2, decays=P2_DECAYS),
}


def workload(cfg_id: int) -> Workload:
    return CONFIGS[cfg_id]
