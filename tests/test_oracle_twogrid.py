"""Pins for the oracle's two-grid-truncation method (section 3, Algorithm 1).

* prolongation: exact P1 interpolation (injection at coarse nodes, edge
  midpoints average their end values, nesting under repeated halving) and
  the Galerkin identities P^T M_h P = M_H, P^T A_h(1) P = A_H(1) that hold
  because V_H is a subspace of V_h;
* Lemma RQ-diff holds for any w, with B = A_s(y) and B~ = A_s'(y);
* with S = s the two-grid value is an upper bound (Lemma RQ-diff with
  B = B~) and converges like H^8 (eq. tg_lam_err).
"""

import numpy as np
import pytest

from oracle import coeff, eig, fem, twogrid
from synth import coeff_family, problem1_family


def _P(nH, nh):
    mH = (nH - 1) ** 2
    cols = [twogrid.prolong(np.eye(mH)[k], nH, nh) for k in range(mH)]
    return np.array(cols).T


def test_prolong_injection_and_edge_midpoints():
    nH, nh = 4, 8
    rng = np.random.default_rng(0)
    u = rng.standard_normal((nH - 1) ** 2)
    v = twogrid.prolong(u, nH, nh)
    U = np.zeros((nH + 1, nH + 1))
    U[1:nH, 1:nH] = u.reshape(nH - 1, nH - 1)
    V = np.zeros((nh + 1, nh + 1))
    V[1:nh, 1:nh] = v.reshape(nh - 1, nh - 1)
    for J in range(nH + 1):
        for I in range(nH + 1):
            assert V[2 * J, 2 * I] == U[J, I]
    for J in range(nH + 1):
        for I in range(nH):
            assert abs(V[2 * J, 2 * I + 1] - 0.5 * (U[J, I] + U[J, I + 1])) < 1e-15   # horizontal
    for J in range(nH):
        for I in range(nH + 1):
            assert abs(V[2 * J + 1, 2 * I] - 0.5 * (U[J, I] + U[J + 1, I])) < 1e-15   # vertical
    for J in range(nH):
        for I in range(nH):
            assert abs(V[2 * J + 1, 2 * I + 1] - 0.5 * (U[J, I] + U[J + 1, I + 1])) < 1e-15  # "/"


def test_prolong_nests():
    rng = np.random.default_rng(1)
    u = rng.standard_normal(9)
    direct = twogrid.prolong(u, 4, 16)
    twice = twogrid.prolong(twogrid.prolong(u, 4, 8), 8, 16)
    assert np.max(np.abs(direct - twice)) < 1e-14


@pytest.mark.parametrize("nH,nh", [(4, 8), (4, 16)])
def test_galerkin_identities(nH, nh):
    P = _P(nH, nh)
    MH, Mh = fem.mass(nH).toarray(), fem.mass(nh).toarray()
    AH = fem.stiffness(nH, np.ones(2 * nH * nH)).toarray()
    Ah = fem.stiffness(nh, np.ones(2 * nh * nh)).toarray()
    assert np.max(np.abs(P.T @ Mh @ P - MH)) < 1e-15
    assert np.max(np.abs(P.T @ Ah @ P - AH)) < 1e-12


def test_lemma_rq_diff_identity():
    n = 16
    fam = coeff_family(32)
    rng = np.random.default_rng(2)
    y = rng.random(32) - 0.5
    B = fem.stiffness(n, coeff.coefficient(n, y[:8], fam))
    Bt = fem.stiffness(n, coeff.coefficient(n, y[:32], fam))
    M = fem.mass(n)
    lam, u = eig.smallest_eigenpair(B, M)
    for _ in range(3):
        w = u + 0.3 * rng.standard_normal(u.size)
        nw = w @ (M @ w)
        d = u - w
        lhs = (w @ (Bt @ w)) / nw - lam
        rhs = ((d @ (Bt @ d)) / nw - lam * (d @ (M @ d)) / nw
               + ((u @ (B @ (u - 2 * w))) - (u @ (Bt @ (u - 2 * w)))) / nw)
        assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_two_grid_upper_bound_and_h8_rate():
    # S = s: the two-grid value is a Rayleigh quotient of the fine problem,
    # so it bounds lambda_h from above; its error decays like H^8.
    fam = problem1_family(4, 2.0)
    y = np.array([0.3, -0.2, 0.1, 0.4])
    nh = 64
    lam_h = twogrid.direct(nh, 4, y, fam)[0]
    errs = []
    for nH in (4, 8, 16):
        lam_tg = twogrid.two_grid(nh, 4, nH, 4, y, fam)[0]
        assert lam_tg >= lam_h * (1 - 1e-14)
        errs.append(lam_tg - lam_h)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 100 < r1 < 600 and 100 < r2 < 600, (errs, r1, r2)


def test_two_grid_close_to_direct_fine_value():
    fam = coeff_family(64)
    y = np.random.default_rng(3).random(64) - 0.5
    lam_h = twogrid.direct(64, 64, y, fam)[0]
    lam_tg, lam_H, _ = twogrid.two_grid(64, 64, 16, 8, y, fam)
    assert lam_H > lam_h                         # coarse FE value is above the fine one
    assert abs(lam_tg - lam_h) < 1e-3 * abs(lam_H - lam_h)
