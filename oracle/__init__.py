"""Plain FP64 CPU oracle for two-grid MLQMC eigen-samples (Gilbert & Scheichl,
"Multilevel quasi-Monte Carlo for random elliptic eigenvalue problems II:
efficient algorithms and numerical results").

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does, and it shares no code with the HIP library (its only
shared inputs come from the seeded generators in ``synth``).

Every step follows the paper's statement in FP64 with library primitives
(scipy sparse assembly, ARPACK shift-invert Lanczos, SuperLU):

* ``mesh``     uniform triangulation of the unit square ("/" diagonals)
* ``coeff``    truncated affine coefficient (eq. coeff, eq. coeff_s)
* ``fem``      P1 stiffness and mass matrices (section 2.3, eq. fe-evp)
* ``eig``      smallest eigenpair of the generalised EVP (section 2.4)
* ``twogrid``  two-grid-truncation method (Algorithm 1, eq. 2grid_src_ell)
* ``rqi``      counted RQ iteration from the fixed or the nearby-point start
               (section 4.3; section 5's absolute tolerance)
* ``qmc``      randomly shifted rank-1 lattice points (eq. rqmc, eq. t_kl),
               shift average and sample variance (eq. sample_var)
* ``mlqmc``    level differences and the estimator (Algorithm 2,
               eq. mlqmc_R, eq. tg-mlqmc, eq. ml-var)

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, textbook identities, invariants or brute force, except
the final multilevel estimate itself, whose value the paper does not print
(its pins are the telescoping identity and the hand-computed estimator).
"""

from . import mesh, coeff, fem, eig, twogrid, qmc, mlqmc, rqi  # noqa: F401
