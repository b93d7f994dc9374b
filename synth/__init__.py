"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds input data only: the coefficient family tables, the
lattice generating vectors (built by a component-by-component search), the
seeded random shifts and the workload descriptions.  It holds none of the
method's arithmetic: the lattice points, the coefficient values, the finite
element operators, the eigensolves and the estimator are computed separately
by ``oracle/`` (plain CPU reference) and by the HIP library.
"""

from .family import coeff_family, islands_family, problem1_family, pair_ordering
from .cbc import cbc_vector, lattice_vector
from .configs import CONFIGS, LevelSpec, Workload, workload, shifts_for

__all__ = [
    "coeff_family",
    "problem1_family",
    "islands_family",
    "pair_ordering",
    "cbc_vector",
    "lattice_vector",
    "CONFIGS",
    "LevelSpec",
    "Workload",
    "workload",
    "shifts_for",
]
