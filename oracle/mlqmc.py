"""Level differences and the MLQMC estimator (section 4; Algorithm 2).

For a level (n_fine=1/h_l, s_fine=s_l, n_coarse=1/H_l, s_coarse=S_l,
n_prev=1/h_{l-1}, s_prev=s_{l-1}) and a parameter value y:

* two-grid levels (n_coarse > 0): one coarse pair (lambda_{H_l,S_l}, u_{H_l,S_l})
  feeds both two-grid updates, lambda^l on (h_l, s_l) and lambda^{l-1} on
  (h_{l-1}, s_{l-1}) for the same point (Algorithm 2 reuses the coarse pair
  for level l-1);
* direct levels (n_coarse = 0): lambda^l = lambda_{h_l,s_l} by a direct
  eigensolve, and lambda^{l-1} = lambda_{h_{l-1},s_{l-1}} likewise (the basic
  estimator eq. mlqmc0; on level 0 of the two-grid estimator
  lambda^0 = lambda_{h_0,s_0});
* n_prev = 0 means lambda^{l-1} = 0 (lambda_{-1} = 0).

Estimator (eq. mlqmc_R / eq. tg-mlqmc with eq. ml-var):
  Q_l^(r) = (1/N_l) sum_{k<N_l} (lambda^l - lambda^{l-1})(y_{l,r,k}),
  Qhat_l = (1/R) sum_r Q_l^(r),  V_l = eq. sample_var,
  Q^ML = sum_l Qhat_l,  V = sum_l V_l.
The loop over k runs over k = 0 .. N_l - 1 (eq. rqmc), and the level-(l-1)
term is evaluated at the same point t_{l,k}.

Shared shifts with nested rules (end of section 4.3): one set of R shifts
and one embedded rule serve every level, so t_{l,k} = t_{0,k} (the first N_l
points of the rule, N_0 >= N_1 >= ...).  Then H_l = h_0 (and S_l = s_0): the
coarse pair of every level is the level-0 direct pair at the same point, and
lambda^{l-1} at level l is the value level l-1 already computed there.  The
level terms of one shift are no longer independent, so the variance of Q^ML
is estimated from the R per-shift totals sum_l Q_l^(r) (eq. sample_var
applied to them); sum_l V_l bounds it only up to the factor L the paper
gives.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fem, functional, qmc, twogrid


@dataclass
class LevelValue:
    Y: float          # lambda^l - lambda^{l-1}
    lam: float        # lambda^l
    lam_prev: float   # lambda^{l-1}
    lam_coarse: float # lambda_{H_l,S_l}, NaN for direct levels
    G: float = float("nan")       # G(u^l), the functional of oracle.functional
    G_prev: float = 0.0           # G(u^{l-1}) (0 without a previous level)


def _G(n, u):
    return functional.G(n, u, fem.mass(n))


def level_value(lv, y, fam) -> LevelValue:
    y = np.asarray(y, dtype=np.float64)
    if lv.n_coarse == 0:
        lam, u = twogrid.direct(lv.n_fine, lv.s_fine, y, fam)
        lam_prev, G_prev = 0.0, 0.0
        if lv.n_prev:
            lam_prev, up = twogrid.direct(lv.n_prev, lv.s_prev, y, fam)
            G_prev = _G(lv.n_prev, up)
        return LevelValue(lam - lam_prev, lam, lam_prev, float("nan"), _G(lv.n_fine, u), G_prev)
    lam_H, u_H = twogrid.coarse_pair(lv.n_coarse, lv.s_coarse, y, fam)
    lam, w = twogrid.two_grid_update(lv.n_fine, lv.s_fine, y, fam, lam_H, u_H, lv.n_coarse)
    lam_prev, G_prev = 0.0, 0.0
    if lv.n_prev:
        if lv.n_prev == lv.n_coarse and lv.s_prev == lv.s_coarse:
            # (A - lambda_H M) is exactly singular here; its two-grid value is lambda_H
            # (and its eigenfunction u_H)
            lam_prev, G_prev = lam_H, _G(lv.n_coarse, u_H)
        else:
            lam_prev, wp = twogrid.two_grid_update(lv.n_prev, lv.s_prev, y, fam, lam_H, u_H,
                                                   lv.n_coarse)
            G_prev = _G(lv.n_prev, wp)
    return LevelValue(lam - lam_prev, lam, lam_prev, lam_H, _G(lv.n_fine, w), G_prev)


def level_samples(lv, z, N: int, shift, fam, ks=None):
    """LevelValue for the points y_k (default k = 0..N-1) of one shift."""
    pts = qmc.lattice_points(z, N, shift, ks)
    return [level_value(lv, y, fam) for y in pts]


@dataclass
class Estimate:
    Q_lr: np.ndarray   # [L+1, R]
    Qhat: np.ndarray   # [L+1]
    V: np.ndarray      # [L+1]
    Q_ml: float
    V_ml: float


def combine(Q_lr) -> Estimate:
    """Shift averages, sample variances and the multilevel sums from Q_l^(r)."""
    Q_lr = np.asarray(Q_lr, dtype=np.float64)
    Qhat = np.array([qmc.shift_average(row) for row in Q_lr])
    V = np.array([qmc.sample_variance(row) for row in Q_lr])
    return Estimate(Q_lr, Qhat, V, math.fsum(Qhat), math.fsum(V))


def estimate(levels, zs, Ns, shifts, fam, with_G: bool = False):
    """Algorithm 2: levels[l], zs[l] (int[s_l]), Ns[l], shifts[l] (float[R, s_l]).
    With with_G, also the same estimator for G(u) (the telescoping sum of the
    introduction with Y_l = G(u^l) - G(u^{l-1})): returns (lambda, G)."""
    L1 = len(levels)
    R = np.asarray(shifts[0]).shape[0]
    Q_lr = np.empty((L1, R))
    QG_lr = np.empty((L1, R))
    for l in range(L1):
        for r in range(R):
            vals = level_samples(levels[l], zs[l], Ns[l], shifts[l][r], fam)
            Q_lr[l, r] = qmc.qmc_mean(v.Y for v in vals)
            QG_lr[l, r] = qmc.qmc_mean(v.G - v.G_prev for v in vals)
    if with_G:
        return combine(Q_lr), combine(QG_lr)
    return combine(Q_lr)


def check_nested(levels, Ns) -> None:
    """The level list the nested estimator accepts: level 0 direct, level
    l >= 1 two-grid from the level-0 mesh and truncation, its previous term
    on level l-1's mesh and truncation, N non-increasing."""
    l0 = levels[0]
    if l0.n_coarse != 0 or l0.n_prev != 0:
        raise ValueError("level 0 must be a direct level without a previous term")
    for l in range(1, len(levels)):
        lv, pv = levels[l], levels[l - 1]
        if (lv.n_coarse, lv.s_coarse) != (l0.n_fine, l0.s_fine):
            raise ValueError("level %d: coarse mesh and truncation must be level 0's" % l)
        if (lv.n_prev, lv.s_prev) != (pv.n_fine, pv.s_fine):
            raise ValueError("level %d: previous term must be on level %d's mesh" % (l, l - 1))
        if Ns[l] > Ns[l - 1]:
            raise ValueError("N must not increase with the level")


def nested_point(levels, z, Ns, shift, k: int, fam):
    """lambda^l(t_k) for l = 0 .. (the last level with k < N_l), at point k
    of the embedded rule with N_0 points: the level-0 direct pair, then the
    two-grid update from it on each finer level."""
    l0 = levels[0]
    y = qmc.embedded_point(z, Ns[0], shift, k)
    lam0, u0 = twogrid.direct(l0.n_fine, l0.s_fine, y, fam)
    out = [lam0]
    for l in range(1, len(levels)):
        if k >= Ns[l]:
            break
        lv = levels[l]
        out.append(twogrid.two_grid_update(lv.n_fine, lv.s_fine, y, fam, lam0, u0,
                                           l0.n_fine)[0])
    return out


def nested_values(levels, z, Ns, shift, fam):
    """lambda^l(t_k) for one shift: lams[l][k], k < N_l, l = 0..L, on the
    first N_l points of the embedded rule with N_0 points (z of length
    max_l s_l; level l reads y_{1:s_l})."""
    check_nested(levels, Ns)
    lams = [np.empty(N) for N in Ns]
    for k in range(Ns[0]):
        for l, v in enumerate(nested_point(levels, z, Ns, shift, k, fam)):
            lams[l][k] = v
    return lams


def nested_level_sums(levels, z, N_done, Ns, shift, fam):
    """For one shift, per level l: the sum of Y_l(t_k) = lambda^l(t_k) -
    lambda^{l-1}(t_k) over k in [N_done[l], Ns[l]), summed exactly rounded.
    This is what an extensible nested estimate adds when it grows from
    N_done[l] to Ns[l] points: the points of the embedded rule do not depend
    on its size (sections 2.5 and 5), so the sums over disjoint blocks add up
    to the sum over all points."""
    check_nested(levels, Ns)
    cache = {}
    out = []
    for l in range(len(levels)):
        terms = []
        for k in range(N_done[l], Ns[l]):
            if k not in cache:
                cache[k] = nested_point(levels, z, Ns, shift, k, fam)
            lams = cache[k]
            terms.append(lams[l] - (lams[l - 1] if l else 0.0))
        out.append(math.fsum(terms))
    return out


def estimate_nested(levels, z, Ns, shifts, fam) -> Estimate:
    """Nested estimator: Y_l(t_k) = lambda^l(t_k) - lambda^{l-1}(t_k)
    (lambda^{-1} = 0), Q_l^(r) their mean over k < N_l, Qhat_l and V_l as in
    Algorithm 2, Q^ML = sum_l Qhat_l, and V_ml the sample variance of the
    per-shift totals."""
    L1 = len(levels)
    R = np.asarray(shifts).shape[0]
    Q_lr = np.empty((L1, R))
    for r in range(R):
        lams = nested_values(levels, z, Ns, shifts[r], fam)
        for l in range(L1):
            prev = lams[l - 1][:Ns[l]] if l else np.zeros(Ns[l])
            Q_lr[l, r] = qmc.qmc_mean(lams[l] - prev)
    est = combine(Q_lr)
    totals = [math.fsum(Q_lr[:, r]) for r in range(R)]
    return Estimate(Q_lr, est.Qhat, est.V, est.Q_ml, qmc.sample_variance(totals))
