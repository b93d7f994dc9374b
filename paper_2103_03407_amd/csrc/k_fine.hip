// Batched fine-mesh kernels of the two-grid update (Algorithm 1 steps 2-4) for
// meshes too large for LDS.  Grid: x = blocks of kFineNT interior nodes, y = sample.
// Every sample carries its own coefficient, shift and prolongated coarse
// eigenvector; per-sample scalars live in FineState.  Samples whose projected
// PCG has finished are skipped (active[b] == 0).
//
// The projected PCG (see lds_mg.h for the algebra) keeps v unnormalised and
// carries vs = ||v||_M^{-1}, so v_n = vs * v below.
#include "../../include/mlqmc.h"
#include "common.h"
#include "kernels.h"

namespace mlqmc {
namespace {

constexpr int NT = kFineNT;

struct Geo {
  int n, m, D;
  __device__ __forceinline__ void ij(int id, int& i, int& j) const {
    j = id / m + 1;
    i = id - (j - 1) * m + 1;
  }
};

// Block reduction of K partial sums; thread 0 writes part[(b*nblk + blk)*K + k].
template <int K>
__device__ __forceinline__ void write_partials(double (&s)[K], double* part) {
  __shared__ double red[K * (NT / 64)];
  block_sums<NT, K>(s, red);
  if (threadIdx.x == 0) {
    const int64_t base = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * K;
#pragma unroll
    for (int k = 0; k < K; ++k) part[base + k] = s[k];
  }
}

__global__ __launch_bounds__(NT) void k_prolong(int nH, int nh, const double* __restrict__ uH,
                                                double* __restrict__ uh) {
  const int mH = nH - 1, mh = nh - 1, Dh = mh * mh;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= Dh) return;
  const int64_t b = blockIdx.y;
  const int j = id / mh + 1, i = id - (j - 1) * mh + 1;
  uh[b * Dh + id] = interp_coarse(uH + b * (int64_t)(mH * mH), nH, nh / nH, i, j);
}

__global__ __launch_bounds__(NT) void k_coarsen(int n, const double* __restrict__ w,
                                                double* __restrict__ wc) {
  const int nc = n / 2, mc = nc - 1;
  const int EX = (n - 1) * n, EW = 2 * EX;
  const int EXc = (nc - 1) * nc, EWc = 2 * EXc;
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= EWc) return;
  const int64_t b = blockIdx.y;
  const double* wx = w + b * EW;
  const double* wy = wx + EX;
  double val;
  if (e < EXc) {
    const int J = e / nc + 1, I = e % nc;
    val = coarsen_wx(wx, n, I, J);
  } else {
    const int f = e - EXc;
    const int J = f / mc, I = f % mc + 1;
    val = coarsen_wy(wy, n, I, J);
  }
  wc[b * EWc + e] = val;
}

// partials: v.M12 v, v.A v  (raw v)
__global__ __launch_bounds__(NT) void k_setup_dots(Geo g, const double* __restrict__ v,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ part) {
  const int64_t b = blockIdx.y;
  const int id = blockIdx.x * NT + threadIdx.x;
  const int EX = (g.n - 1) * g.n;
  double s[2] = {0.0, 0.0};
  if (id < g.D) {
    int i, j;
    g.ij(id, i, j);
    const double* vb = v + b * g.D;
    const double* wx = w + b * (2 * EX);
    double d;
    const double av = stencil_A(vb, wx, wx + EX, g.n, i, j, id, d);
    s[0] = vb[id] * stencil_M12(vb, g.n, i, j, id);
    s[1] = vb[id] * av;
  }
  write_partials<2>(s, part);
}

// r = -(A v_n - rho M v_n), t = 0, zb = omega r / diag (first smoothing sweep)
__global__ __launch_bounds__(NT) void k_setup_rhs(Geo g, const double* __restrict__ v,
                                                  const double* __restrict__ w, FineState S,
                                                  double* __restrict__ r, double* __restrict__ t,
                                                  double* __restrict__ zb) {
  const int64_t b = blockIdx.y;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= g.D) return;
  const int EX = (g.n - 1) * g.n;
  int i, j;
  g.ij(id, i, j);
  const double* vb = v + b * g.D;
  const double* wx = w + b * (2 * EX);
  double d;
  const double av = stencil_A(vb, wx, wx + EX, g.n, i, j, id, d);
  const double mv = mass_scale(g.n) * stencil_M12(vb, g.n, i, j, id);
  const double vs = S.vs[b];
  const double rv = -vs * (av - S.rho[b] * mv);
  r[b * g.D + id] = rv;
  t[b * g.D + id] = 0.0;
  zb[b * g.D + id] = kOmega * rv / d;
}

// q = (A - mu M) p; partials p.q, v_n.q, p.M v_n
__global__ __launch_bounds__(NT) void k_apply_dots(Geo g, const double* __restrict__ p,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ w, FineState S,
                                                   double* __restrict__ q,
                                                   double* __restrict__ part) {
  const int64_t b = blockIdx.y;
  if (!S.active[b]) return;
  const int id = blockIdx.x * NT + threadIdx.x;
  const int EX = (g.n - 1) * g.n;
  double s[3] = {0.0, 0.0, 0.0};
  if (id < g.D) {
    int i, j;
    g.ij(id, i, j);
    const double* pb = p + b * g.D;
    const double* vb = v + b * g.D;
    const double* wx = w + b * (2 * EX);
    const double hm = mass_scale(g.n), vs = S.vs[b];
    double d;
    const double ap = stencil_A(pb, wx, wx + EX, g.n, i, j, id, d);
    const double qv = ap - S.mu[b] * hm * stencil_M12(pb, g.n, i, j, id);
    q[b * g.D + id] = qv;
    s[0] = pb[id] * qv;
    s[1] = vs * vb[id] * qv;
    s[2] = pb[id] * vs * hm * stencil_M12(vb, g.n, i, j, id);
  }
  write_partials<3>(s, part);
}

// t += alpha p; r -= alpha (q - c M v_n); zb = omega r / diag
__global__ __launch_bounds__(NT) void k_update(Geo g, const double* __restrict__ p,
                                               const double* __restrict__ q,
                                               const double* __restrict__ v,
                                               const double* __restrict__ w, FineState S,
                                               double* __restrict__ t, double* __restrict__ r,
                                               double* __restrict__ zb) {
  const int64_t b = blockIdx.y;
  if (!S.active[b]) return;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= g.D) return;
  const int EX = (g.n - 1) * g.n;
  int i, j;
  g.ij(id, i, j);
  const int64_t o = b * g.D + id;
  const double* vb = v + b * g.D;
  const double* wx = w + b * (2 * EX);
  const double alpha = S.alpha[b];
  const double mv = S.vs[b] * mass_scale(g.n) * stencil_M12(vb, g.n, i, j, id);
  t[o] += alpha * p[o];
  const double rn = r[o] - alpha * (q[o] - S.c[b] * mv);
  r[o] = rn;
  zb[o] = kOmega * rn / stencil_diag(wx, wx + EX, g.n, i, j);
}

__global__ __launch_bounds__(NT) void k_jacobi_first(Geo g, const double* __restrict__ w,
                                                     const double* __restrict__ rhs,
                                                     double* __restrict__ X,
                                                     const uint8_t* __restrict__ active) {
  const int64_t b = blockIdx.y;
  if (active && !active[b]) return;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= g.D) return;
  const int EX = (g.n - 1) * g.n;
  int i, j;
  g.ij(id, i, j);
  const double* wx = w + b * (2 * EX);
  X[b * g.D + id] = kOmega * rhs[b * g.D + id] / stencil_diag(wx, wx + EX, g.n, i, j);
}

__global__ __launch_bounds__(NT) void k_jacobi(Geo g, const double* __restrict__ w,
                                               const double* __restrict__ rhs,
                                               const double* __restrict__ Xin,
                                               double* __restrict__ Xout,
                                               const uint8_t* __restrict__ active) {
  const int64_t b = blockIdx.y;
  if (active && !active[b]) return;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= g.D) return;
  const int EX = (g.n - 1) * g.n;
  int i, j;
  g.ij(id, i, j);
  const double* xb = Xin + b * g.D;
  const double* wx = w + b * (2 * EX);
  double d;
  const double ax = stencil_A(xb, wx, wx + EX, g.n, i, j, id, d);
  Xout[b * g.D + id] = xb[id] + kOmega * (rhs[b * g.D + id] - ax) / d;
}

// rhs_c = P^T (rhs - A X) on the next coarser mesh (7 fine residuals per coarse node)
__global__ __launch_bounds__(NT) void k_resid_restrict(Geo g, const double* __restrict__ w,
                                                       const double* __restrict__ rhs,
                                                       const double* __restrict__ X,
                                                       double* __restrict__ rhs_c,
                                                       const uint8_t* __restrict__ active) {
  const int64_t b = blockIdx.y;
  if (active && !active[b]) return;
  const int nc = g.n / 2, mc = nc - 1, Dc = mc * mc;
  const int idc = blockIdx.x * NT + threadIdx.x;
  if (idc >= Dc) return;
  const int J = idc / mc + 1, I = idc - (J - 1) * mc + 1;
  const int EX = (g.n - 1) * g.n;
  const double* xb = X + b * g.D;
  const double* rb = rhs + b * g.D;
  const double* wx = w + b * (2 * EX);
  const double* wy = wx + EX;
  auto res = [&](int i, int j) -> double {
    const int id = (j - 1) * g.m + (i - 1);
    double d;
    return rb[id] - stencil_A(xb, wx, wy, g.n, i, j, id, d);
  };
  const int i0 = 2 * I, j0 = 2 * J;
  const double v = res(i0, j0) + 0.5 * (res(i0 - 1, j0) + res(i0 + 1, j0) + res(i0, j0 - 1) +
                                        res(i0, j0 + 1) + res(i0 + 1, j0 + 1) +
                                        res(i0 - 1, j0 - 1));
  rhs_c[b * Dc + idc] = v;
}

__global__ __launch_bounds__(NT) void k_prolong_add(Geo g, const double* __restrict__ Xc,
                                                    double* __restrict__ X,
                                                    const uint8_t* __restrict__ active) {
  const int64_t b = blockIdx.y;
  if (active && !active[b]) return;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= g.D) return;
  int i, j;
  g.ij(id, i, j);
  const int nc = g.n / 2, Dc = (nc - 1) * (nc - 1);
  X[b * g.D + id] += prolong2_at(Xc + b * Dc, nc, i, j);
}

// partials r.z, M v_n . z, r . v_n
__global__ __launch_bounds__(NT) void k_dots3(Geo g, const double* __restrict__ r,
                                              const double* __restrict__ z,
                                              const double* __restrict__ v, FineState S,
                                              double* __restrict__ part) {
  const int64_t b = blockIdx.y;
  if (!S.active[b]) return;
  const int id = blockIdx.x * NT + threadIdx.x;
  double s[3] = {0.0, 0.0, 0.0};
  if (id < g.D) {
    int i, j;
    g.ij(id, i, j);
    const int64_t o = b * g.D + id;
    const double* vb = v + b * g.D;
    const double vs = S.vs[b];
    const double zz = z[o], rr = r[o];
    s[0] = rr * zz;
    s[1] = vs * mass_scale(g.n) * stencil_M12(vb, g.n, i, j, id) * zz;
    s[2] = rr * vs * vb[id];
  }
  write_partials<3>(s, part);
}

// p = z - c2 v_n + beta p
__global__ __launch_bounds__(NT) void k_pupdate(Geo g, const double* __restrict__ z,
                                                const double* __restrict__ v, FineState S,
                                                double* __restrict__ p) {
  const int64_t b = blockIdx.y;
  if (!S.active[b]) return;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= g.D) return;
  const int64_t o = b * g.D + id;
  p[o] = z[o] - S.c2[b] * S.vs[b] * v[o] + S.beta[b] * p[o];
}

// w = v_n + t: partials w.A w, w.M12 w
__global__ __launch_bounds__(NT) void k_final_dots(Geo g, const double* __restrict__ v,
                                                   const double* __restrict__ t,
                                                   const double* __restrict__ w, FineState S,
                                                   double* __restrict__ part) {
  const int64_t b = blockIdx.y;
  const int id = blockIdx.x * NT + threadIdx.x;
  const int EX = (g.n - 1) * g.n;
  double s[2] = {0.0, 0.0};
  if (id < g.D) {
    int i, j;
    g.ij(id, i, j);
    const int m = g.m, n = g.n;
    const double* vb = v + b * g.D;
    const double* tb = t + b * g.D;
    const double vs = S.vs[b];
    auto W = [&](int k) -> double { return vs * vb[k] + tb[k]; };
    const double wc = W(id);
    const double ww = (i > 1) ? W(id - 1) : 0.0, we = (i < m) ? W(id + 1) : 0.0;
    const double ws = (j > 1) ? W(id - m) : 0.0, wn = (j < m) ? W(id + m) : 0.0;
    const double wne = (i < m && j < m) ? W(id + m + 1) : 0.0;
    const double wsw = (i > 1 && j > 1) ? W(id - m - 1) : 0.0;
    const double* wx = w + b * (2 * EX);
    const double* wy = wx + EX;
    const double aw = wx[(j - 1) * n + (i - 1)] * (wc - ww) + wx[(j - 1) * n + i] * (wc - we) +
                      wy[(j - 1) * m + (i - 1)] * (wc - ws) + wy[j * m + (i - 1)] * (wc - wn);
    const double mw = 6.0 * wc + ww + we + ws + wn + wne + wsw;
    s[0] = wc * aw;
    s[1] = wc * mw;
  }
  write_partials<2>(s, part);
}

// one wavefront per sample: sum the sample's block partials in fixed order
__global__ __launch_bounds__(256) void k_scalar(int phase, int n, int64_t B, int nblk,
                                                const double* __restrict__ part, FineState S,
                                                double rtol, int max_it) {
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  int K = 3;
  if (phase == PH_SETUP || phase == PH_FINAL) K = 2;
  if (phase != PH_SETUP && phase != PH_FINAL && phase != PH_FIRST_RZ && !S.active[b]) return;
  double s[3] = {0.0, 0.0, 0.0};
  for (int k = lane; k < nblk; k += 64)
    for (int c = 0; c < K; ++c) s[c] += part[((int64_t)b * nblk + k) * K + c];
  for (int c = 0; c < K; ++c) s[c] = wave_sum(s[c]);
  if (lane != 0) return;
  const double hm = mass_scale(n);
  switch (phase) {
    case PH_SETUP: {  // s0 = v.M12v, s1 = v.Av (raw v)
      const double g = s[0] * hm;
      S.vs[b] = 1.0 / sqrt(g);
      S.rho[b] = s[1] / g;
      S.active[b] = 1;
      S.its[b] = 0;
      break;
    }
    case PH_FIRST_RZ: {  // s0 = r.z, s1 = Mv.z, s2 = r.v
      const double rz = s[0] - s[2] * s[1];
      S.rz[b] = rz;
      S.rz0[b] = rz;
      S.c2[b] = s[1];
      S.beta[b] = 0.0;
      if (!(rz > 0.0)) S.active[b] = 0;  // zero right-hand side: t = 0 is exact
      break;
    }
    case PH_ALPHA: {  // s0 = p.q, s1 = v.q, s2 = p.Mv
      const double pq = s[0] - s[2] * s[1];
      if (!(pq > 0.0)) {
        S.flags[b] |= MLQMC_FLAG_BREAKDOWN;
        S.active[b] = 0;
        S.alpha[b] = 0.0;
        break;
      }
      S.alpha[b] = S.rz[b] / pq;
      S.c[b] = s[1];
      break;
    }
    case PH_BETA: {  // s0 = r.z, s1 = Mv.z, s2 = r.v
      const double rzn = s[0] - s[2] * s[1];
      const int it = S.its[b] + 1;
      S.its[b] = it;
      if (sqrt(fabs(rzn / S.rz0[b])) <= rtol) {
        S.active[b] = 0;
        break;
      }
      if (it >= max_it) {
        S.flags[b] |= MLQMC_FLAG_LIN_NOCONV;
        S.active[b] = 0;
        break;
      }
      S.beta[b] = rzn / S.rz[b];
      S.rz[b] = rzn;
      S.c2[b] = s[1];
      break;
    }
    case PH_FINAL: {  // s0 = w.Aw, s1 = w.M12w
      const double lam = s[0] / (s[1] * hm);
      S.lam[b] = lam;
      if (S.lin_acc) S.lin_acc[b] += S.its[b];
      if (!isfinite(lam)) S.flags[b] |= MLQMC_FLAG_NONFINITE;
      break;
    }
  }
}

__global__ __launch_bounds__(NT) void k_apply_plain(Geo g, const double* __restrict__ w,
                                                    const double* __restrict__ sigma,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ out) {
  const int64_t b = blockIdx.y;
  const int id = blockIdx.x * NT + threadIdx.x;
  if (id >= g.D) return;
  const int EX = (g.n - 1) * g.n;
  int i, j;
  g.ij(id, i, j);
  const double* xb = x + b * g.D;
  const double* wx = w + b * (2 * EX);
  double d;
  const double ax = stencil_A(xb, wx, wx + EX, g.n, i, j, id, d);
  out[b * g.D + id] = ax - sigma[b] * mass_scale(g.n) * stencil_M12(xb, g.n, i, j, id);
}

inline Geo geo(int n) { return Geo{n, n - 1, (n - 1) * (n - 1)}; }
inline dim3 grid_for(int D, int64_t B) { return dim3((unsigned)fine_blocks(D), (unsigned)B); }

}  // namespace

hipError_t launch_prolong(int nH, int nh, int64_t B, const double* uH, double* uh,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_prolong, grid_for((nh - 1) * (nh - 1), B), dim3(NT), 0, st, nH, nh, uH, uh);
  return hipGetLastError();
}

hipError_t launch_coarsen(int n, int64_t B, const double* w, double* wc, hipStream_t st) {
  const int nc = n / 2;
  hipLaunchKernelGGL(k_coarsen, grid_for(2 * (nc - 1) * nc, B), dim3(NT), 0, st, n, w, wc);
  return hipGetLastError();
}

hipError_t launch_setup_dots(int n, int64_t B, const double* v, const double* w, double* part,
                             hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_setup_dots, grid_for(g.D, B), dim3(NT), 0, st, g, v, w, part);
  return hipGetLastError();
}

hipError_t launch_setup_rhs(int n, int64_t B, const double* v, const double* w,
                            const FineState& S, double* r, double* t, double* zb,
                            hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_setup_rhs, grid_for(g.D, B), dim3(NT), 0, st, g, v, w, S, r, t, zb);
  return hipGetLastError();
}

hipError_t launch_apply_dots(int n, int64_t B, const double* p, const double* v, const double* w,
                             const FineState& S, double* q, double* part, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_apply_dots, grid_for(g.D, B), dim3(NT), 0, st, g, p, v, w, S, q, part);
  return hipGetLastError();
}

hipError_t launch_update(int n, int64_t B, const double* p, const double* q, const double* v,
                         const double* w, const FineState& S, double* t, double* r, double* zb,
                         hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_update, grid_for(g.D, B), dim3(NT), 0, st, g, p, q, v, w, S, t, r, zb);
  return hipGetLastError();
}

hipError_t launch_jacobi_first(int n, int64_t B, const double* w, const double* rhs, double* X,
                               const uint8_t* active, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_jacobi_first, grid_for(g.D, B), dim3(NT), 0, st, g, w, rhs, X, active);
  return hipGetLastError();
}

hipError_t launch_jacobi(int n, int64_t B, const double* w, const double* rhs, const double* Xin,
                         double* Xout, const uint8_t* active, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_jacobi, grid_for(g.D, B), dim3(NT), 0, st, g, w, rhs, Xin, Xout, active);
  return hipGetLastError();
}

hipError_t launch_resid_restrict(int n, int64_t B, const double* w, const double* rhs,
                                 const double* X, double* rhs_c, const uint8_t* active,
                                 hipStream_t st) {
  const Geo g = geo(n);
  const int mc = n / 2 - 1;
  hipLaunchKernelGGL(k_resid_restrict, grid_for(mc * mc, B), dim3(NT), 0, st, g, w, rhs, X,
                     rhs_c, active);
  return hipGetLastError();
}

hipError_t launch_prolong_add(int n, int64_t B, const double* Xc, double* X,
                              const uint8_t* active, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_prolong_add, grid_for(g.D, B), dim3(NT), 0, st, g, Xc, X, active);
  return hipGetLastError();
}

hipError_t launch_dots3(int n, int64_t B, const double* r, const double* z, const double* v,
                        const FineState& S, double* part, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_dots3, grid_for(g.D, B), dim3(NT), 0, st, g, r, z, v, S, part);
  return hipGetLastError();
}

hipError_t launch_pupdate(int n, int64_t B, const double* z, const double* v,
                          const FineState& S, double* p, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_pupdate, grid_for(g.D, B), dim3(NT), 0, st, g, z, v, S, p);
  return hipGetLastError();
}

hipError_t launch_final_dots(int n, int64_t B, const double* v, const double* t,
                             const double* w, const FineState& S, double* part, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_final_dots, grid_for(g.D, B), dim3(NT), 0, st, g, v, t, w, S, part);
  return hipGetLastError();
}

hipError_t launch_scalar(int phase, int n, int64_t B, int nblk, const double* part,
                         const FineState& S, double rtol, int max_it, hipStream_t st) {
  const unsigned blocks = (unsigned)((B + 3) / 4);
  hipLaunchKernelGGL(k_scalar, dim3(blocks), dim3(256), 0, st, phase, n, B, nblk, part, S, rtol,
                     max_it);
  return hipGetLastError();
}

hipError_t launch_apply_plain(int n, int64_t B, const double* w, const double* sigma,
                              const double* x, double* out, hipStream_t st) {
  const Geo g = geo(n);
  hipLaunchKernelGGL(k_apply_plain, grid_for(g.D, B), dim3(NT), 0, st, g, w, sigma, x, out);
  return hipGetLastError();
}

}  // namespace mlqmc
