"""Pins for the oracle's counted RQ iteration (section 4.3; section 5's
absolute tolerance 5e-8):

* the converged value is the smallest eigenvalue: against the shift-invert
  Lanczos eigenpair and, on a 3 x 3 interior mesh, dense LAPACK;
* started from the converged eigenvector of the same point it stops after
  one iteration;
* cubic convergence: each eigenvalue error is at most a modest multiple of
  the cube of the previous one (relative), until round-off;
* the counts the paper prints for Problem 1 (section 5): 3 iterations from
  the fixed start in almost all cases, and 2 when started from the previous
  QMC point's eigenvector in almost all cases.
"""

import numpy as np
import pytest

from oracle import eig, fem, qmc, rqi, twogrid
from synth import lattice_vector, problem1_family, shifts_for


def _pts(count, k0=100):
    z = lattice_vector(1024, 64)
    sh = shifts_for(2, 0, 1, 64)[0]
    return qmc.lattice_points(z, 1024, sh, range(k0, k0 + count))


def test_converges_to_the_smallest_eigenvalue():
    fam = problem1_family(64, 2.0)
    for y in _pts(3):
        for n in (4, 8):
            A = twogrid.operator(n, 8, y, fam)
            M = fem.mass(n)
            sig, v, its, _ = rqi.rq_iteration(A, M, rqi.sine_start(n), 5e-8)
            lam = eig.smallest_eigenpair(A, M)[0]
            assert abs(sig - lam) <= 1e-13 * lam
            if n == 4:
                assert abs(sig - eig.dense_spectrum(A, M)[0]) <= 1e-12 * lam
            assert abs(float(v @ (M @ v)) - 1.0) < 1e-13


def test_exact_start_takes_one_iteration():
    fam = problem1_family(64, 2.0)
    y = _pts(1)[0]
    A = twogrid.operator(8, 8, y, fam)
    M = fem.mass(8)
    _, u = eig.smallest_eigenpair(A, M)
    _, _, its, hist = rqi.rq_iteration(A, M, u, 5e-8)
    assert its == 1 and abs(hist[1] - hist[0]) <= 1e-12 * hist[0]


def test_cubic_convergence():
    fam = problem1_family(64, 2.0)
    y = _pts(1)[0]
    A = twogrid.operator(16, 8, y, fam)
    M = fem.mass(16)
    lam = eig.smallest_eigenpair(A, M)[0]
    _, _, _, hist = rqi.rq_iteration(A, M, rqi.sine_start(16), 0.0, max_iter=4)
    e = [abs(h - lam) / lam for h in hist]
    assert e[0] > 1e-4                     # a real start, not a converged one
    for a, b in zip(e, e[1:]):
        if a < 1e-5:
            break                          # the next error is round-off
        assert b <= 100.0 * a ** 3, e


@pytest.mark.parametrize("p", [2.0, 4.0 / 3.0])
def test_paper_iteration_counts_problem1(p):
    # Problem 1 (s = 64, S = 8, H = 1/8), 32 consecutive points of one shift
    fam = problem1_family(64, p)
    cold, warm, lc, lw = rqi.chain_counts(8, 8, _pts(32), fam, tol=5e-8)
    assert np.all(cold == 3)
    assert warm[0] == cold[0]              # the chain's first point starts cold
    nearby = warm[1:]
    assert np.median(nearby) == 2 and np.mean(nearby == 2) >= 0.7
    assert np.all(nearby <= 3)
    assert np.max(np.abs(lc - lw) / lc) <= 1e-13


def test_one_step_on_two_eigenvectors():
    # from v0 = u1 + b u2 (M-orthonormal eigenvectors of the pencil, dense
    # LAPACK) one step stays in their span, each component divided by its
    # eigenvalue minus the Rayleigh quotient sigma_0 of v0
    import scipy.linalg as sla
    fam = problem1_family(64, 2.0)
    y = _pts(1)[0]
    A = twogrid.operator(8, 8, y, fam)
    M = fem.mass(8)
    lam, U = sla.eigh(A.toarray(), M.toarray())
    b = 0.3
    v0 = U[:, 0] + b * U[:, 1]
    sig0 = (lam[0] + b * b * lam[1]) / (1.0 + b * b)
    _, v1, its, hist = rqi.rq_iteration(A, M, v0, 0.0, max_iter=1)
    assert its == 1 and abs(hist[0] - sig0) <= 1e-13 * sig0
    c = U.T @ (M @ v1)                     # coefficients in the eigenbasis
    assert np.max(np.abs(c[2:])) <= 1e-10 * np.max(np.abs(c[:2]))
    want = (b / (lam[1] - sig0)) / (1.0 / (lam[0] - sig0))
    assert abs(c[1] / c[0] - want) <= 1e-9 * abs(want)
