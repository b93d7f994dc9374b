"""RQ iteration counts at the paper's criterion (section 5: absolute
tolerance 5e-8) on the device against the oracle's counted RQ iteration, from
the fixed start and from the previous QMC point's eigenvector (section 4.3).
The inner solves run to 1e-12, so the device iteration is the exact-solve RQ
iteration of the oracle; counts are then compared point by point (a count can
differ only where |sigma_k - sigma_{k-1}| lies within round-off of 5e-8)."""

import numpy as np
import pytest

import paper_2103_03407_amd as m
from oracle import qmc, rqi
from synth import coeff_family, lattice_vector, problem1_family, shifts_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fam_name,n,S", [("p1-2", 8, 8), ("p1-4/3", 8, 8), ("bench", 16, 16),
                                          ("bench", 32, 8)])
def test_rq_counts_match_oracle(fam_name, n, S):
    fam = {"p1-2": problem1_family(64, 2.0), "p1-4/3": problem1_family(64, 4.0 / 3.0),
           "bench": coeff_family(64, 2.5)}[fam_name]
    cnt = 32
    z = lattice_vector(1024, 64)
    sh = shifts_for(2, 0, 1, 64)[0]
    Y = np.ascontiguousarray(qmc.lattice_points(z, 1024, sh, range(100, 100 + cnt))[:, :S])
    cold_o, warm_o, lam_o, _ = rqi.chain_counts(n, S, Y, fam, tol=5e-8)
    ctx = m.Context(fam)
    try:
        got = {}
        for warm in (0, 1):
            lam = np.empty(cnt)
            fl = np.zeros(cnt, np.uint8)
            rq = np.zeros(cnt, np.int32)
            o = m.default_opts(eig_atol=5e-8, rq_lin_rtol=1e-12, max_lin_iter=200, chain_len=cnt)
            ctx.eig_level((n, S, 0, 0, 0, 0), Y, lam, fl, rq_iters=rq, warm_chain=warm, opts=o)
            assert not fl.any(), fl
            assert np.max(np.abs(lam - lam_o) / lam_o) <= 1e-10
            got[warm] = rq
    finally:
        ctx.close()
    assert np.mean(got[0] == cold_o) >= 0.9, (got[0], cold_o)
    assert np.mean(got[1] == warm_o) >= 0.9, (got[1], warm_o)
    assert got[1][1:].mean() < got[0][1:].mean()
