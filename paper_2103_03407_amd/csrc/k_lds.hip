// Per-sample LDS kernels: the warm-started Rayleigh-quotient eigensolve on a
// coarse (or direct-level) mesh, the two-grid update on small fine meshes, and
// the bottom of the batched V-cycle.  One workgroup owns one sample (or one
// warm-start chain of samples) and keeps every vector in LDS.
#include <type_traits>

#include "../../include/mlqmc.h"
#include "kernels.h"
#include "lds_mg.h"

namespace mlqmc {
namespace {

constexpr int kMaxStagedS = 512;

template <int N>
constexpr int threads_for() {
  return N >= 32 ? 256 : (N >= 16 ? 128 : 64);
}
// With the reaction term the 1/32 two-grid update holds 110 KB of LDS, one
// workgroup per CU: twice the threads keep two waves on each SIMD.  (The
// eigensolve keeps 256: at 512 its live state no longer fits the registers.)
template <int N>
constexpr int threads_for_reaction() {
  return N >= 32 ? 512 : threads_for<N>();
}

// v = sin(pi x1) sin(pi x2) at the interior nodes
template <int NT, int n, typename T>
__device__ __forceinline__ void init_sine(T* v) {
  LDS_FOR_NODES(NT, n, k) {
    const int i = k & (n - 1), j = k >> lds::Mesh<n>::lg;
    v[k] = (T)(sinpi(double(i) / n) * sinpi(double(j) / n));
  }
  __syncthreads();
}

// M-overlap of the M-normalised v with the normalised sine mode
template <int NT, int n, typename T>
__device__ __forceinline__ double sine_overlap(const T* v, double* red) {
  constexpr int m = n - 1;
  double s[2] = {0.0, 0.0};
  LDS_FOR_NODES(NT, n, k) {
    const int i = k & (n - 1), j = k >> lds::Mesh<n>::lg;
    auto ph = [&](int a, int b) -> double {
      return (a >= 1 && a <= m && b >= 1 && b <= m) ? sinpi(double(a) / n) * sinpi(double(b) / n)
                                                     : 0.0;
    };
    const double p0 = ph(i, j);
    const double mp = 6.0 * p0 + ph(i - 1, j) + ph(i + 1, j) + ph(i, j - 1) + ph(i, j + 1) +
                      ph(i + 1, j + 1) + ph(i - 1, j - 1);
    s[0] += (double)v[k] * mp;
    s[1] += p0 * mp;
  }
  block_sums<NT, 2>(s, red);
  const double hm = mass_scale(n);
  return fabs(s[0] * hm) / sqrt(s[1] * hm);
}

// Share of the l1 norm of v carried by its dominant sign: 1 for a vector of
// one sign, as the discrete ground state of Problem 2 is; an excited state
// changes sign and scores well below.
template <int NT, int n, typename T>
__device__ __forceinline__ double sign_share(const T* v, double* red) {
  double s[2] = {0.0, 0.0};
  LDS_FOR_NODES(NT, n, k) {
    const double x = (double)v[k];
    s[0] += x;
    s[1] += fabs(x);
  }
  block_sums<NT, 2>(s, red);
  return s[1] > 0.0 ? fabs(s[0]) / s[1] : 0.0;
}

// Stages the point of sample i into s_y and forms the level's weights.
// Problem 1: w = a0 + sum_{j<S} y_j Phi_j.  Problem 2 (kR): the tables carry
// the background values as row 0, so s_y = (1, y_1, ..., y_S) weights S + 1
// rows of both the diffusion table [WX | WY] and the reaction table
// [RX | RY | RD]; with FP32 storage the FP64 block goes to w64 (for the
// Rayleigh quotients) and its rounding to a.wx.
template <int N, int NT, bool kR, typename T>
__device__ __forceinline__ void stage_weights(const double* Y, int64_t ldY, int64_t i, int S,
                                              const double* phi, const double* rphi, double a0,
                                              const lds::PcgArrays<T>& a, double* s_y,
                                              double* w64) {
  constexpr int P = lds::Mesh<N>::P;
  if constexpr (kR) {
    for (int j = threadIdx.x; j <= S; j += NT) s_y[j] = j == 0 ? 1.0 : Y[i * ldY + j - 1];
    __syncthreads();
    if constexpr (std::is_same_v<T, double>) {
      lds::weights_from_table<NT, N>(phi, s_y, S + 1, 0.0, a.wx);
      lds::weights_from_table<NT, N, T, 3>(rphi, s_y, S + 1, 0.0, a.wx + 2 * P);
    } else {
      lds::weights_from_table<NT, N>(phi, s_y, S + 1, 0.0, w64);
      lds::weights_from_table<NT, N, double, 3>(rphi, s_y, S + 1, 0.0, w64 + 2 * P);
      for (int e = threadIdx.x; e < 5 * P; e += NT) a.wx[e] = (T)w64[e];
      __syncthreads();
    }
  } else {
    for (int j = threadIdx.x; j < S; j += NT) s_y[j] = Y[i * ldY + j];
    __syncthreads();
    lds::weights_from_table<NT, N>(phi, s_y, S, a0, a.wx);
  }
  lds::coarsen_all<NT, N, T, kR>(a.wx, a.wy, a.mg);
}

// The chain of samples [blockIdx.x * chain_len, ...) on mesh N: arrays in `a`
// (zero padding), the staged point in s_y.
template <int N, int NT, bool kR = false, typename T, class WF>
__device__ void rqi_chain(const RqiArgs& A, const lds::PcgArrays<T>& a, double* s_y,
                          const WF& wf, double* w64 = nullptr) {
  using Mh = lds::Mesh<N>;
  constexpr int m = N - 1;
  T* const s_v = a.v;
  const int64_t i0 = (int64_t)blockIdx.x * A.chain_len;
  const int64_t i1 = (i0 + A.chain_len < A.n) ? i0 + A.chain_len : A.n;
  bool have_prev = false;
  for (int64_t i = i0; i < i1; ++i) {
    stage_weights<N, NT, kR>(A.Y, A.ldY, i, A.S, A.phi, A.rphi, A.a0, a, s_y, w64);
    if (!(A.warm && have_prev)) init_sine<NT, N>(s_v);

    double vMv, vAv;
    lds::rayleigh_parts<NT, N, T, WF, kR>(a, s_v, wf, vMv, vAv);
    lds::scale_vec<NT, N>(s_v, 1.0 / sqrt(vMv));
    double sigma = vAv / vMv;  // sigma_0 = A(t_k; v0, v0) for the M-normalised start

    int rq = 0, lin = 0;
    bool conv = false;
    uint8_t fl = 0;
    while (rq < A.max_rq) {
      ++rq;
      bool c, b;
      lin += lds::jd_pcg<NT, N, false, kR>(a, sigma, sigma, A.lin_rtol, A.max_lin, &c, &b);
      LDS_FOR_NODES(NT, N, k) s_v[k] += a.t[k];
      __syncthreads();
      lds::rayleigh_parts<NT, N, T, WF, kR>(a, s_v, wf, vMv, vAv);
      lds::scale_vec<NT, N>(s_v, 1.0 / sqrt(vMv));
      const double sig_new = vAv / vMv;
      const double tol = A.eig_atol > 0.0 ? A.eig_atol : A.eig_rtol * fabs(sig_new);
      const bool done = fabs(sig_new - sigma) <= tol;
      sigma = sig_new;
      if (!isfinite(sigma)) break;
      if (done) {
        conv = true;
        break;
      }
    }
    if (!conv) fl |= MLQMC_FLAG_RQ_NOCONV;
    if (!isfinite(sigma)) fl |= MLQMC_FLAG_NONFINITE;
    // The inexact inner solves leave the vector's error near the square root
    // of sigma's.  G is linear in the vector (here, or through the two-grid
    // update that starts from it): one correction solve at the converged
    // sigma to the linear tolerance (a Newton step) makes it as accurate as
    // the two-grid vectors; lambda stays the converged sigma
    const bool refine = conv && A.g_lin_rtol > 0.0 && (A.g_out || A.refine);
    if (refine) {
      bool c, b;
      lin += lds::jd_pcg<NT, N, false, kR>(a, sigma, sigma, A.g_lin_rtol, A.max_lin, &c, &b);
      if (!c) fl |= MLQMC_FLAG_LIN_NOCONV;
      LDS_FOR_NODES(NT, N, k) s_v[k] += a.t[k];
      __syncthreads();
    }
    if (A.g_out || refine) {
      double sm, mn;
      lds::sum_and_mnorm<NT, N>(a, s_v, sm, mn);
      if (A.g_out && threadIdx.x == 0) A.g_out[i] = fabs(sm) / ((double)N * N * sqrt(mn));
      lds::scale_vec<NT, N>(s_v, 1.0 / sqrt(mn));
    }
    // ground-state check: overlap with the first sine mode (Problem 1), or
    // one sign (Problem 2, whose islands can pull the ground state away from
    // the sine mode)
    if constexpr (kR) {
      if (!(sign_share<NT, N>(s_v, a.red) >= 0.9)) fl |= MLQMC_FLAG_WRONG_PAIR;
    } else {
      if (!(sine_overlap<NT, N>(s_v, a.red) >= 0.5)) fl |= MLQMC_FLAG_WRONG_PAIR;
    }
    if (threadIdx.x == 0) {
      A.lam[i] = sigma;
      if (A.rq_iters) A.rq_iters[i] = rq;
      if (A.lin_iters) A.lin_iters[i] = lin;
      A.flags[i] = fl;
    }
    if (A.u_out) {  // interior layout, node (i, j) at (j - 1) m + i - 1
      LDS_FOR_NODES(NT, N, k) {
        const int ii = k & (N - 1), jj = k >> Mh::lg;
        A.u_out[i * Mh::D + (jj - 1) * m + ii - 1] = (double)s_v[k];
      }
    }
    have_prev = (fl == 0);
    __syncthreads();
  }
}

// Every array in LDS (meshes up to 1/32).  The five vectors' padding is
// zeroed once; the solvers write interior positions only.  T = float keeps
// vectors, weights and V-cycle in FP32 (mixed precision); the Rayleigh
// quotients then use FP64 weights recomputed from the edge table.
// With kR (Problem 2) the weight block also holds the reaction arrays; with
// FP32 storage an FP64 copy of it serves the Rayleigh quotients.
// Minimum waves per SIMD (the second launch bound), measured per mesh and
// precision: four where the registers allow (more waves beat the spills
// they cause), two for the FP64 1/32 kernels, three for the reaction's 1/8
// and 1/16 kernels (in FP64 5-8 % faster on 1/8 and 1/16 levels and 1.7x on
// a direct 1/16 level than leaving the choice to the compiler, which took
// 180-256 registers and one or two waves; four spilled more and ran 30 %
// slower), one for its 1/32 kernels (110 KB of LDS each).
template <int N, int NT, bool kR>
constexpr int lds_blocks_per_cu(int tsize) {
  return kR ? (N <= 16 ? 3 : 1) : ((N >= 32 && tsize == 8) ? 2 : 4);
}
template <int N, int NT, typename T, bool kR = false>
__global__ __launch_bounds__(NT, (lds_blocks_per_cu<N, NT, kR>(sizeof(T)))) void k_rqi(RqiArgs A) {
  using Mh = lds::Mesh<N>;
  constexpr int P = Mh::P;
  __shared__ T s_w[lds::wblock<kR>() * P];
  __shared__ T s_vec[5 * P];
  __shared__ T s_mg[lds::mg_scratch<N, kR>() + 1];
  __shared__ double s_red[6 * (NT / 64)];
  __shared__ double s_y[kMaxStagedS];
  __shared__ double s_w64[(kR && sizeof(T) < 8) ? 5 * P : 1];
  lds::PcgArrays<T> a;
  a.wx = s_w;
  a.wy = s_w + P;
  a.v = s_vec;
  a.t = s_vec + P;
  a.r = s_vec + 2 * P;
  a.z = s_vec + 3 * P;
  a.p = s_vec + 4 * P;
  a.q = a.z;
  a.mg = s_mg;
  a.red = s_red;
  a.xtmp = nullptr;
  lds::zero<NT>(s_vec, 5 * P);
  __syncthreads();
  if constexpr (sizeof(T) == 8) {
    rqi_chain<N, NT, kR>(A, a, s_y, lds::WeightsFromArrays<N>{s_w, s_w + P});
  } else if constexpr (kR) {
    rqi_chain<N, NT, kR>(A, a, s_y, lds::WeightsFromArrays<N>{s_w64, s_w64 + P}, s_w64);
  } else {
    rqi_chain<N, NT>(A, a, s_y, lds::WeightsFromTable<N>{A.phi, s_y, A.S, A.a0});
  }
}

// Meshes whose vectors exceed LDS (1/64): the top-level weights (with the
// reaction arrays for Problem 2), the five PCG vectors and the smoother's
// second array live in the workgroup's slice of a global scratch buffer
// (L2/MALL resident while it runs); the levels below stay in LDS.
template <int N, bool kR = false>
constexpr int64_t global_doubles() {
  return (int64_t)lds::wblock<kR>() * lds::Mesh<N>::P + 6 * (int64_t)lds::Mesh<N>::P;
}
template <int N, int NT, bool kR = false>
__global__ __launch_bounds__(NT) void k_rqi_global(RqiArgs A) {
  using Mh = lds::Mesh<N>;
  constexpr int P = Mh::P;
  __shared__ double s_mg[lds::mg_scratch<N, kR>() + 1];
  __shared__ double s_red[6 * (NT / 64)];
  __shared__ double s_y[kMaxStagedS];
  double* g = A.scratch + (int64_t)blockIdx.x * global_doubles<N, kR>();
  double* vec = g + lds::wblock<kR>() * P;
  lds::PcgArrays<double> a;
  a.wx = g;
  a.wy = g + P;
  a.v = vec;
  a.t = vec + P;
  a.r = vec + 2 * P;
  a.z = vec + 3 * P;
  a.p = vec + 4 * P;
  a.q = a.z;
  a.xtmp = vec + 5 * P;
  a.mg = s_mg;
  a.red = s_red;
  lds::zero<NT>(vec, 6 * P);
  __syncthreads();
  rqi_chain<N, NT, kR>(A, a, s_y, lds::WeightsFromArrays<N>{g, g + P});
}

// Two-grid update of sample i from its coarse pair: arrays in `a` (zero
// padding), the staged point in s_y (w64: the FP64 weight block of FP32
// storage with the reaction term).
template <int N, int NT, bool kR, typename T>
__device__ void tg_sample(const TgSmallArgs& A, const lds::PcgArrays<T>& a, double* s_y,
                          double* w64, int64_t i) {
  using Mh = lds::Mesh<N>;
  constexpr int P = Mh::P;
  T* const s_v = a.v;
  stage_weights<N, NT, kR>(A.Y, A.ldY, i, A.s, A.phi, A.rphi, A.a0, a, s_y, w64);
  const int mH = A.nH - 1, ratio = N / A.nH;
  const double* uH = A.uH + i * (int64_t)(mH * mH);
  LDS_FOR_NODES(NT, N, k) {
    const int ii = k & (N - 1), jj = k >> Mh::lg;
    s_v[k] = (T)interp_coarse(uH, A.nH, ratio, ii, jj);
  }
  __syncthreads();
  auto run = [&](const auto& wf) {
    using WF = std::decay_t<decltype(wf)>;
    double vMv, vAv;
    lds::rayleigh_parts<NT, N, T, WF, kR>(a, s_v, wf, vMv, vAv);
    lds::scale_vec<NT, N>(s_v, 1.0 / sqrt(vMv));
    const double rho = vAv / vMv;
    const double mu = A.lamH[i];
    bool c, b;
    const int its =
        lds::jd_pcg<NT, N, true, kR>(a, mu, rho, A.lin_rtol, A.max_lin, &c, &b, A.lam_rtol);
    LDS_FOR_NODES(NT, N, k) s_v[k] += a.t[k];
    __syncthreads();
    lds::rayleigh_parts<NT, N, T, WF, kR>(a, s_v, wf, vMv, vAv);
    const double lam = vAv / vMv;
    if (A.g) {
      double sm, mn;
      lds::sum_and_mnorm<NT, N>(a, s_v, sm, mn);
      if (threadIdx.x == 0) A.g[i] = fabs(sm) / ((double)N * N * sqrt(mn));
    }
    if (threadIdx.x == 0) {
      A.lam[i] = lam;
      if (A.lin_iters) A.lin_iters[i] += its;
      uint8_t fl = 0;
      if (!c) fl |= MLQMC_FLAG_LIN_NOCONV;
      if (b) fl |= MLQMC_FLAG_BREAKDOWN;
      if (!isfinite(lam)) fl |= MLQMC_FLAG_NONFINITE;
      A.flags[i] |= fl;
    }
  };
  if constexpr (sizeof(T) == 8)
    run(lds::WeightsFromArrays<N>{(const double*)a.wx, (const double*)a.wx + P});
  else if constexpr (kR)
    run(lds::WeightsFromArrays<N>{w64, w64 + P});
  else
    run(lds::WeightsFromTable<N>{A.phi, s_y, A.s, A.a0});
}

template <int N, int NT, typename T, bool kR = false>
__global__ __launch_bounds__(NT, (lds_blocks_per_cu<N, NT, kR>(sizeof(T)))) void k_tg_small(
    TgSmallArgs A) {
  using Mh = lds::Mesh<N>;
  constexpr int P = Mh::P;
  __shared__ T s_w[lds::wblock<kR>() * P];
  __shared__ T s_vec[5 * P];
  __shared__ T s_mg[lds::mg_scratch<N, kR>() + 1];
  __shared__ double s_red[6 * (NT / 64)];
  __shared__ double s_y[kMaxStagedS];
  __shared__ double s_w64[(kR && sizeof(T) < 8) ? 5 * P : 1];
  lds::PcgArrays<T> a;
  a.wx = s_w;
  a.wy = s_w + P;
  a.v = s_vec;
  a.t = s_vec + P;
  a.r = s_vec + 2 * P;
  a.z = s_vec + 3 * P;
  a.p = s_vec + 4 * P;
  a.q = a.z;
  a.mg = s_mg;
  a.red = s_red;
  a.xtmp = nullptr;
  lds::zero<NT>(s_vec, 5 * P);
  tg_sample<N, NT, kR>(A, a, s_y, s_w64, (int64_t)blockIdx.x);
}

// The V-cycle below the batched levels: one workgroup per sample reads its
// padded arrays of the batched layout ((N + 2) N per vector, same indexing)
// into LDS, runs the cycle (three Chebyshev sweeps per smoothing step),
// writes the interior of X back.
template <int N, int NT, typename T, bool kR = false>
__global__ __launch_bounds__(NT) void k_bottom(const T* __restrict__ w, const T* __restrict__ rhs,
                                               T* __restrict__ X,
                                               const uint8_t* __restrict__ active) {
  using Mh = lds::Mesh<N>;
  constexpr int P = Mh::P, PG = (N + 2) * N, WB = lds::wblock<kR>();
  const int64_t b = blockIdx.x;
  if (active && !active[b]) return;
  __shared__ T s_w[WB * P];
  __shared__ T s_b[P], s_x[P];
  __shared__ T s_mg[lds::mg_scratch<N, kR>() + 1];
  // the global block holds WB arrays of PG entries; LDS keeps the first P of each
  const T* wb = w + b * WB * PG;
  const T* rb = rhs + b * PG;
  for (int e = threadIdx.x; e < P; e += NT) {
#pragma unroll
    for (int a = 0; a < WB; ++a) s_w[a * P + e] = wb[a * PG + e];
    s_b[e] = rb[e];
    s_x[e] = T(0);
  }
  __syncthreads();
  lds::coarsen_all<NT, N, T, kR>(s_w, s_w + P, s_mg);
  lds::vcycle<NT, N, true, T, 3, kR>(s_w, s_w + P, s_b, s_x, s_mg);
  LDS_FOR_NODES(NT, N, k) X[b * PG + k] = s_x[k];
}

template <int N>
hipError_t rqi_n(const RqiArgs& a, hipStream_t st) {
  const int64_t chains = (a.n + a.chain_len - 1) / a.chain_len;
  if (chains <= 0) return hipSuccess;
  if constexpr (N <= 32) {
    constexpr int NT = threads_for<N>();
    if (a.rphi && a.mixed) {  // Problem 2
      hipLaunchKernelGGL((k_rqi<N, NT, float, true>), dim3((unsigned)chains), dim3(NT), 0, st,
                         a);
    } else if (a.rphi) {
      hipLaunchKernelGGL((k_rqi<N, NT, double, true>), dim3((unsigned)chains), dim3(NT), 0, st,
                         a);
    } else if (a.mixed) {
      hipLaunchKernelGGL((k_rqi<N, NT, float>), dim3((unsigned)chains), dim3(NT), 0, st, a);
    } else {
      hipLaunchKernelGGL((k_rqi<N, NT, double>), dim3((unsigned)chains), dim3(NT), 0, st, a);
    }
  } else {
    // Problem 2's eigensolves (direct and coarse meshes) stay at 1/32 or coarser
    if (a.rphi) return hipErrorInvalidValue;
    // the caller provides chains x rqi_scratch_doubles(N) doubles of scratch
    if (!a.scratch || a.scratch_doubles < chains * global_doubles<N>())
      return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_rqi_global<N, 512>), dim3((unsigned)chains), dim3(512), 0, st, a);
  }
  return hipGetLastError();
}

template <int N>
hipError_t tg_small_n(const TgSmallArgs& a, hipStream_t st) {
  constexpr int NT = threads_for<N>();
  if (a.n <= 0) return hipSuccess;
  constexpr int NTR = threads_for_reaction<N>();
  if (a.rphi && a.mixed) {  // Problem 2
    hipLaunchKernelGGL((k_tg_small<N, NTR, float, true>), dim3((unsigned)a.n), dim3(NTR), 0, st,
                       a);
  } else if (a.rphi) {
    hipLaunchKernelGGL((k_tg_small<N, NTR, double, true>), dim3((unsigned)a.n), dim3(NTR), 0, st,
                       a);
  } else if (a.mixed) {
    hipLaunchKernelGGL((k_tg_small<N, NT, float>), dim3((unsigned)a.n), dim3(NT), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_tg_small<N, NT, double>), dim3((unsigned)a.n), dim3(NT), 0, st, a);
  }
  return hipGetLastError();
}

template <int N, typename T>
hipError_t bottom_n(int64_t B, const T* w, const T* rhs, T* X, const uint8_t* active,
                    int reaction, hipStream_t st) {
  constexpr int NT = threads_for<N>();
  if (B <= 0) return hipSuccess;
  if (reaction)
    hipLaunchKernelGGL((k_bottom<N, NT, T, true>), dim3((unsigned)B), dim3(NT), 0, st, w, rhs, X,
                       active);
  else
    hipLaunchKernelGGL((k_bottom<N, NT, T, false>), dim3((unsigned)B), dim3(NT), 0, st, w, rhs, X,
                       active);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rqi(int N, const RqiArgs& a, hipStream_t st) {
  if (a.S + (a.rphi ? 1 : 0) > kMaxStagedS) return hipErrorInvalidValue;
  switch (N) {
    case 4: return rqi_n<4>(a, st);
    case 8: return rqi_n<8>(a, st);
    case 16: return rqi_n<16>(a, st);
    case 32: return rqi_n<32>(a, st);
    case 64: return rqi_n<64>(a, st);
    default: return hipErrorInvalidValue;
  }
}

int64_t rqi_scratch_doubles(int N) { return N == 64 ? global_doubles<64>() : 0; }

template <int N>
hipError_t rqi_occupancy(int* per, int mixed, int reaction) {
  constexpr int NT = threads_for<N>();
  if (reaction) {
    if (mixed)
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_rqi<N, NT, float, true>, NT, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_rqi<N, NT, double, true>, NT, 0);
  }
  if (mixed) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_rqi<N, NT, float>, NT, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_rqi<N, NT, double>, NT, 0);
}

// Workgroups of the eigensolve on mesh N that the current device holds at
// once (compute units x resident workgroups per unit); 0 if unknown.  reaction
// selects the Problem 2 instantiation (more LDS per workgroup).
int rqi_chains_in_flight(int N, int mixed, int reaction) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e = hipErrorInvalidValue;
  switch (N) {
    case 4: e = rqi_occupancy<4>(&per, mixed, reaction); break;
    case 8: e = rqi_occupancy<8>(&per, mixed, reaction); break;
    case 16: e = rqi_occupancy<16>(&per, mixed, reaction); break;
    case 32: e = rqi_occupancy<32>(&per, mixed, reaction); break;
    case 64:
      if (!reaction)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_rqi_global<64, 512>, 512, 0);
      break;
    default: break;
  }
  if (e != hipSuccess || per <= 0) return 0;
  return cus * per;
}

hipError_t launch_tg_small(int N, const TgSmallArgs& a, hipStream_t st) {
  if (a.s + (a.rphi ? 1 : 0) > kMaxStagedS) return hipErrorInvalidValue;
  switch (N) {
    case 4: return tg_small_n<4>(a, st);
    case 8: return tg_small_n<8>(a, st);
    case 16: return tg_small_n<16>(a, st);
    case 32: return tg_small_n<32>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_bottom_vcycle(int NB, int64_t B, const T* w, const T* rhs, T* X,
                                const uint8_t* active, int reaction, hipStream_t st) {
  switch (NB) {
    case 4: return bottom_n<4, T>(B, w, rhs, X, active, reaction, st);
    case 8: return bottom_n<8, T>(B, w, rhs, X, active, reaction, st);
    case 16: return bottom_n<16, T>(B, w, rhs, X, active, reaction, st);
    case 32: return bottom_n<32, T>(B, w, rhs, X, active, reaction, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_bottom_vcycle<double>(int, int64_t, const double*, const double*,
                                                 double*, const uint8_t*, int, hipStream_t);
template hipError_t launch_bottom_vcycle<float>(int, int64_t, const float*, const float*, float*,
                                                const uint8_t*, int, hipStream_t);

}  // namespace mlqmc
