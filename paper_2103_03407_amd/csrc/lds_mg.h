// Per-workgroup solvers for one sample on meshes h = 1/N (N <= 32 in LDS;
// the top level of N = 64 in global scratch):
//
// * a geometric V-cycle for the SPD stiffness matrix A(a) (damped Jacobi,
//   2 pre- and 2 post-sweeps, rediscretised coarse levels whose edge weights
//   are means of the fine ones, exact solve on the one-node mesh 1/2);
// * a projected preconditioned CG for the correction equation
//       P (A - mu M) P^T t = -(A v - rho M v),  P = I - M v v^T,  v^T M t = 0,
//   with v^T M v = 1 and rho = v^T A v.  Its solution gives v + t parallel to
//   (A - mu M)^{-1} M v, the shifted-inverse-iteration step of the RQ iteration
//   (section 2.4, mu = rho) and of the two-grid update (Algorithm 1 step 2,
//   mu = lambda_{H,S}).  On the M-orthogonal complement of v the projected
//   operator is symmetric positive definite while mu is below the second
//   eigenvalue of the pencil restricted there, so CG applies, and the
//   nearly-singular direction of (A - mu M) never enters the iteration.
//   The preconditioner is P^T K^{-1} P with K^{-1} one V-cycle of A.
//
// Padded layout of a level n (the batched kernels use the same indexing):
// node (i, j), 1 <= i, j <= n-1, at k = j n + i in an array of
// P(n) = (n+1) n + 1 entries; row 0, row n, column 0 and the last entry are
// zero and are never written, and the right neighbour of column n-1 aliases
// column 0 of the next row, so every stencil is branch-free.  Edge weights:
// WX[k] is the edge arriving at node k from the west, WY[k] from the south
// (so the east and north edges of node k are WX[k + 1] and WY[k + n]), two
// arrays of P(n) entries.  Loops run over the positions n .. n n - 1 and skip
// column 0.  With the reaction term of Problem 2 (template flag kR) the
// weight block of a level is [WX | WY | RX | RY | RD]: RX, RY hold the mean
// reaction coefficient of the same edges as WX, WY and RD[k] that of the
// diagonal edge arriving at node k from the south-west (RD[k + n + 1] is the
// edge to the north-east); the operator adds
//   (R x)_k = h^2/12 sum over the six edges e of k of r_e (x_k + x_other end)
// (the element mass matrices weighted by b).
// T is the storage and arithmetic type of the vectors, weights and
// V-cycle (double, or float in mixed precision); every dot product and every
// Rayleigh quotient is accumulated in double, the quotients from FP64 weights.
#pragma once

#include "common.h"

namespace mlqmc {
namespace lds {

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

template <int n>
struct Mesh {
  static_assert(n >= 2 && (n & (n - 1)) == 0, "meshes are 1/n with n a power of two");
  static constexpr int m = n - 1;
  static constexpr int D = m * m;            // interior nodes
  static constexpr int P = (n + 1) * n + 1;  // padded length of a vector
  static constexpr int EW = 2 * P;           // [WX | WY]
  static constexpr int lg = ilog2(n);
};

// Loop over the interior positions owned by this thread: k = n + t, n + t +
// NT, ... < n n, skipping column 0.
#define LDS_FOR_NODES(NT, n, k)                                  \
  for (int k = (n) + (int)threadIdx.x; k < (n) * (n); k += (NT)) \
    if ((k & ((n) - 1)) != 0)

// Synchronisation between the steps of a V-cycle level: the workgroup, or
// (kW) only the one wave that runs the coarsest levels by itself.  A wave's
// LDS accesses complete in order, so there the fences only keep the compiler
// from moving them across.
template <bool kW>
MLQMC_DEV void level_sync() {
  if constexpr (kW) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// weight arrays per level: [WX | WY], or [WX | WY | RX | RY | RD] with reaction
template <bool kR>
constexpr int wblock() {
  return kR ? 5 : 2;
}

// (A x)_k (plus (R x)_k with kR) with the diagonal in d, in the weights'
// type T (x may be stored narrower: FP32 vectors with FP64 weights)
template <int n, typename T, bool kR = false, typename X>
MLQMC_DEV T pA(const X* x, const T* wx, const T* wy, int k, T& d) {
  const T ww = wx[k], we = wx[k + 1], ws = wy[k], wn = wy[k + n];
  d = ww + we + ws + wn;
  const T xc = (T)x[k];
  T ax = ww * (xc - (T)x[k - 1]) + we * (xc - (T)x[k + 1]) + ws * (xc - (T)x[k - n]) +
         wn * (xc - (T)x[k + n]);
  if constexpr (kR) {
    constexpr int P = (n + 1) * n + 1;
    const T* rx = wx + 2 * P;
    const T* ry = wx + 3 * P;
    const T* rd = wx + 4 * P;
    const T hm = (T)(1.0 / (12.0 * n * n));
    const T r1 = rx[k], r2 = rx[k + 1], r3 = ry[k], r4 = ry[k + n], r5 = rd[k],
            r6 = rd[k + n + 1];
    ax += hm * (r1 * (xc + (T)x[k - 1]) + r2 * (xc + (T)x[k + 1]) + r3 * (xc + (T)x[k - n]) +
                r4 * (xc + (T)x[k + n]) + r5 * (xc + (T)x[k - n - 1]) +
                r6 * (xc + (T)x[k + n + 1]));
    d += hm * (r1 + r2 + r3 + r4 + r5 + r6);
  }
  return ax;
}
template <int n, typename T, bool kR = false>
MLQMC_DEV T pdiag(const T* wx, const T* wy, int k) {
  T d = wx[k] + wx[k + 1] + wy[k] + wy[k + n];
  if constexpr (kR) {
    constexpr int P = (n + 1) * n + 1;
    const T* rx = wx + 2 * P;
    const T* ry = wx + 3 * P;
    const T* rd = wx + 4 * P;
    d += (T)(1.0 / (12.0 * n * n)) *
         (rx[k] + rx[k + 1] + ry[k] + ry[k + n] + rd[k] + rd[k + n + 1]);
  }
  return d;
}
// (M x)_k without the h^2/12 factor
template <int n, typename T>
MLQMC_DEV T pM12(const T* x, int k) {
  return T(6) * x[k] + x[k - 1] + x[k + 1] + x[k - n] + x[k + n] + x[k + n + 1] + x[k - n - 1];
}

// the same in FP64 whatever T: with FP32 entries, (M x)_k rounded to FP32
// would put a relative error of order 1e-8 into x^T M x and so into the
// Rayleigh quotient
template <int n, typename T>
MLQMC_DEV double pM12d(const T* x, int k) {
  return 6.0 * (double)x[k] + (double)x[k - 1] + (double)x[k + 1] + (double)x[k - n] +
         (double)x[k + n] + (double)x[k + n + 1] + (double)x[k - n - 1];
}

// Coarse levels finer than 1/32 (only below a 1/128 top level, in global
// memory) sweep between two arrays instead of staging in registers, so they
// carry a third vector
constexpr int level_vectors(int c) { return c > 32 ? 3 : 2; }

// Entries of the V-cycle levels strictly below mesh n: per level nc, the
// weights (2 P, or 5 P with reaction) and B, X (2 P; 3 P with the second
// sweep array).
template <int n, bool kR = false>
constexpr int mg_scratch() {
  int s = 0;
  for (int c = n / 2; c >= 2; c /= 2)
    s += (wblock<kR>() + level_vectors(c)) * ((c + 1) * c + 1);
  return s;
}

// zero `count` entries
template <int NT, typename T>
MLQMC_DEV void zero(T* x, int count) {
  for (int e = threadIdx.x; e < count; e += NT) x[e] = T(0);
}

// Weights of every level below n, each the mean of the two collinear fine
// edges it covers (horizontal, vertical and, with reaction, diagonal); the B
// and X arrays of every level are zeroed.
template <int NT, int n, typename T, bool kR = false>
MLQMC_DEV void coarsen_all(const T* wx, const T* wy, T* nxt) {
  if constexpr (n > 2) {
    constexpr int nc = n / 2, Pc = Mesh<nc>::P, P = Mesh<n>::P;
    T* wxc = nxt;
    T* wyc = wxc + Pc;
    for (int e = threadIdx.x; e < Pc; e += NT) {
      const int J = e / nc, I = e % nc;
      const int Ie = (I == 0) ? nc : I, Je = (I == 0) ? J - 1 : J;
      const bool okx = Je >= 1 && Je <= nc - 1, oky = J >= 1 && J <= nc && I >= 1;
      const int fx0 = 2 * Je * n + 2 * Ie - 1, fy0 = (2 * J - 1) * n + 2 * I;
      wxc[e] = okx ? T(0.5) * (wx[fx0] + wx[fx0 + 1]) : T(0);
      wyc[e] = oky ? T(0.5) * (wy[fy0] + wy[fy0 + n]) : T(0);
      if constexpr (kR) {
        const T* rx = wx + 2 * P;
        const T* ry = wx + 3 * P;
        const T* rd = wx + 4 * P;
        wxc[2 * Pc + e] = okx ? T(0.5) * (rx[fx0] + rx[fx0 + 1]) : T(0);
        wxc[3 * Pc + e] = oky ? T(0.5) * (ry[fy0] + ry[fy0 + n]) : T(0);
        // diagonal edge of coarse square (Ic, Jc), stored at its north-east
        // end (column 0 of row Jc + 2 when Ic = nc - 1); it covers the
        // diagonals of fine squares (2Ic, 2Jc) and (2Ic + 1, 2Jc + 1)
        const int Ic = (I == 0) ? nc - 1 : I - 1, Jc = (I == 0) ? J - 2 : J - 1;
        T v = T(0);
        if (Ic >= 0 && Ic <= nc - 1 && Jc >= 0 && Jc <= nc - 1) {
          const int f1 = (2 * Jc + 1) * n + 2 * Ic + 1, f2 = (2 * Jc + 2) * n + 2 * Ic + 2;
          v = T(0.5) * (rd[f1] + rd[f2]);
        }
        wxc[4 * Pc + e] = v;
      }
    }
    T* rest = wxc + wblock<kR>() * Pc;  // B, X (and X2) of this level, then the next
    zero<NT>(rest, level_vectors(nc) * Pc);
    __syncthreads();
    coarsen_all<NT, nc, T, kR>(wxc, wyc, rest + level_vectors(nc) * Pc);
  }
}

// X = omega * B / diag  (first sweep from a zero start)
template <int NT, int n, typename T, bool kR = false, bool kW = false>
MLQMC_DEV void jacobi_first(const T* wx, const T* wy, const T* B, T* X, double om) {
  LDS_FOR_NODES(NT, n, k) X[k] = T(om) * B[k] / pdiag<n, T, kR>(wx, wy, k);
  level_sync<kW>();
}

// X <- X + omega (B - A X) / diag, new values staged in registers
template <int NT, int n, typename T, bool kR = false, bool kW = false>
MLQMC_DEV void jacobi_sweep(const T* wx, const T* wy, const T* B, T* X, double om) {
  constexpr int PT = (n * n - n + NT - 1) / NT;
  T nv[PT];
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    const int k = n + (int)threadIdx.x + q * NT;
    if (k < n * n && (k & (n - 1)) != 0) {
      T d;
      const T ax = pA<n, T, kR>(X, wx, wy, k, d);
      nv[q] = X[k] + T(om) * (B[k] - ax) / d;
    }
  }
  level_sync<kW>();
#pragma unroll
  for (int q = 0; q < PT; ++q) {
    const int k = n + (int)threadIdx.x + q * NT;
    if (k < n * n && (k & (n - 1)) != 0) X[k] = nv[q];
  }
  level_sync<kW>();
}

// Xout = Xin + omega (B - A Xin) / diag (two distinct arrays; for top levels
// too large for register staging)
template <int NT, int n, typename T, bool kR = false>
MLQMC_DEV void jacobi_to(const T* wx, const T* wy, const T* B, const T* Xin, T* Xout,
                         double om) {
  LDS_FOR_NODES(NT, n, k) {
    T d;
    const T ax = pA<n, T, kR>(Xin, wx, wy, k, d);
    Xout[k] = Xin[k] + T(om) * (B[k] - ax) / d;
  }
  __syncthreads();
}

// Bc = P^T (B - A X): the residual at the seven fine nodes each coarse node's
// hat function covers (weight 1 at the node, 1/2 at E, W, N, S, NE, SW, all
// interior), formed on the fly, so no residual array is stored.
template <int NT, int n, typename T, bool kR = false, bool kW = false>
MLQMC_DEV void restrict_residual(const T* wx, const T* wy, const T* B, const T* X, T* Bc) {
  constexpr int nc = n / 2;
  auto res = [&](int k) {
    T d;
    return B[k] - pA<n, T, kR>(X, wx, wy, k, d);
  };
  LDS_FOR_NODES(NT, nc, kc) {
    const int I = kc & (nc - 1), J = kc >> Mesh<nc>::lg;
    const int f = 2 * J * n + 2 * I;
    Bc[kc] = res(f) + T(0.5) * (res(f - 1) + res(f + 1) + res(f - n) + res(f + n) +
                                res(f + n + 1) + res(f - n - 1));
  }
  level_sync<kW>();
}

// X += P Xc (2:1 P1 interpolation: the mean of the coarse values at
// (i>>1, j>>1) and ((i+1)>>1, (j+1)>>1))
template <int NT, int n, typename T, bool kW = false>
MLQMC_DEV void prolong_add(const T* Xc, T* X) {
  constexpr int nc = n / 2;
  LDS_FOR_NODES(NT, n, k) {
    const int i = k & (n - 1), j = k >> Mesh<n>::lg;
    X[k] += T(0.5) * (Xc[(j >> 1) * nc + (i >> 1)] + Xc[((j + 1) >> 1) * nc + ((i + 1) >> 1)]);
  }
  level_sync<kW>();
}

// One V-cycle X = K^{-1} B on mesh n; `nxt` holds the coarser levels (weights
// built by coarsen_all).  kStage: register-staged sweeps (false: the sweeps
// alternate between X and Xtmp, for top levels in global scratch).  kSw: 2 or
// 3 Jacobi sweeps per smoothing step with the Chebyshev weights of that
// degree (3 needs kStage).  The levels of 1/8 and coarser (49 nodes or
// fewer) run in the first wave alone (kW), with no workgroup barrier inside
// them; the other waves wait at one barrier for their result.
template <int NT, int n, bool kStage = true, typename T, int kSw = 2, bool kR = false,
          bool kW = false>
MLQMC_DEV void vcycle(const T* wx, const T* wy, const T* B, T* X, T* nxt, T* Xtmp = nullptr) {
  static_assert(kSw == 2 || (kSw == 3 && kStage), "3 sweeps need register staging");
  static_assert(!kW || NT == 64, "a wave-local level runs on 64 threads");
  if constexpr (n == 2) {
    if (threadIdx.x == 0) X[3] = B[3] / pdiag<2, T, kR>(wx, wy, 3);
    level_sync<kW>();
  } else {
    constexpr int nc = n / 2, Pc = Mesh<nc>::P;
    const T* wxc = nxt;
    const T* wyc = wxc + Pc;
    T* Bc = nxt + wblock<kR>() * Pc;
    T* Xc = Bc + Pc;
    T* X2c = level_vectors(nc) == 3 ? Xc + Pc : nullptr;
    T* nxtc = Xc + (level_vectors(nc) - 1) * Pc;
    if constexpr (kSw == 3) {
      jacobi_first<NT, n, T, kR, kW>(wx, wy, B, X, kCheb3[0]);
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kCheb3[1]);
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kCheb3[2]);
    } else if constexpr (kStage) {
      jacobi_first<NT, n, T, kR, kW>(wx, wy, B, X, kOmega1);
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kOmega2);
    } else {
      jacobi_first<NT, n, T, kR>(wx, wy, B, Xtmp, kOmega1);
      jacobi_to<NT, n, T, kR>(wx, wy, B, Xtmp, X, kOmega2);
    }
    restrict_residual<NT, n, T, kR, kW>(wx, wy, B, X, Bc);
    if constexpr (!kW && NT > 64 && nc <= 8) {
      if (threadIdx.x < 64) vcycle<64, nc, true, T, kSw, kR, true>(wxc, wyc, Bc, Xc, nxtc, X2c);
      __syncthreads();
    } else {
      vcycle<NT, nc, (nc <= 32), T, kSw, kR, kW>(wxc, wyc, Bc, Xc, nxtc, X2c);
    }
    prolong_add<NT, n, T, kW>(Xc, X);
    if constexpr (kSw == 3) {
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kCheb3[0]);
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kCheb3[1]);
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kCheb3[2]);
    } else if constexpr (kStage) {
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kOmega1);
      jacobi_sweep<NT, n, T, kR, kW>(wx, wy, B, X, kOmega2);
    } else {
      jacobi_to<NT, n, T, kR>(wx, wy, B, X, Xtmp, kOmega1);
      jacobi_to<NT, n, T, kR>(wx, wy, B, Xtmp, X, kOmega2);
    }
  }
}

// Arrays of one projected-PCG solve on mesh N, P(N) doubles each except the
// weights [WX | WY] and the multigrid scratch.  q may share z's storage (z is
// dead between forming p and the next V-cycle); xtmp is only used when the
// top level sweeps without register staging.
template <typename T>
struct PcgArrays {
  T *wx, *wy, *v, *t, *r, *z, *p, *q, *mg, *xtmp;
  double* red;
};

// The four FP64 edge weights of node k, from the arrays (double storage) or
// recomputed from the padded edge table (float storage): w = a0 + sum_j y_j Phi[j]
struct Wd {
  double ww, we, ws, wn;
};
template <int n>
struct WeightsFromArrays {
  const double *wx, *wy;
  MLQMC_DEV Wd operator()(int k) const { return Wd{wx[k], wx[k + 1], wy[k], wy[k + n]}; }
};
template <int n>
struct WeightsFromTable {
  const double* phi;  // rows of [WX | WY], (n + 2) n entries each
  const double* ys;
  int S;
  double a0;
  MLQMC_DEV Wd operator()(int k) const {
    constexpr int PG = (n + 2) * n;
    double a[4] = {a0, a0, a0, a0};
    const int e[4] = {k, k + 1, PG + k, PG + k + n};
    for (int j = 0; j < S; ++j) {
      const double y = ys[j];
      const double* row = phi + (int64_t)j * 2 * PG;
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] += y * row[e[q]];
    }
    return Wd{a[0], a[1], a[2], a[3]};
  }
};

// ||x||_M^2 and x^T A x in one pass in FP64 with FP64 weights from wf (all
// threads get both).  With the reaction term wf is WeightsFromArrays over the
// FP64 block [WX | WY | RX | RY | RD] and the stencil runs on it.
template <int NT, int n, typename T, class WF, bool kR = false>
MLQMC_DEV void rayleigh_parts(const PcgArrays<T>& a, const T* x, const WF& wf, double& xMx,
                              double& xAx) {
  double s[2] = {0.0, 0.0};
  LDS_FOR_NODES(NT, n, k) {
    const double xc = (double)x[k];
    double ax;
    if constexpr (kR) {
      double d;
      ax = pA<n, double, true>(x, wf.wx, wf.wy, k, d);
    } else {
      const Wd w = wf(k);
      ax = w.ww * (xc - (double)x[k - 1]) + w.we * (xc - (double)x[k + 1]) +
           w.ws * (xc - (double)x[k - n]) + w.wn * (xc - (double)x[k + n]);
    }
    s[0] += xc * pM12d<n>(x, k);
    s[1] += xc * ax;
  }
  block_sums<NT, 2>(s, a.red);
  xMx = s[0] * mass_scale(n);
  xAx = s[1];
}

// sum of the nodal values and x^T M x, both in FP64: the integral of the P1
// function with these nodal values is h^2 times the sum (each hat function
// integrates to h^2 on this mesh)
template <int NT, int n, typename T>
MLQMC_DEV void sum_and_mnorm(const PcgArrays<T>& a, const T* x, double& sum, double& xMx) {
  double s[2] = {0.0, 0.0};
  LDS_FOR_NODES(NT, n, k) {
    const double xc = (double)x[k];
    s[0] += xc;
    s[1] += xc * pM12d<n>(x, k);
  }
  block_sums<NT, 2>(s, a.red);
  sum = s[0];
  xMx = s[1] * mass_scale(n);
}

template <int NT, int n, typename T>
MLQMC_DEV void scale_vec(T* x, double f) {
  LDS_FOR_NODES(NT, n, k) x[k] = (T)((double)x[k] * f);
  __syncthreads();
}

template <int NT, int n, bool kR = false, typename T>
MLQMC_DEV void precondition(const PcgArrays<T>& a, const T* r, T* z) {
  if constexpr (n > 32)
    vcycle<NT, n, false, T, 2, kR>(a.wx, a.wy, r, z, a.mg, a.xtmp);
  else
    vcycle<NT, n, true, T, 2, kR>(a.wx, a.wy, r, z, a.mg);
}

// Projected PCG for  P (A - mu M) P^T t = -(A v - rho M v), t = 0 initially.
// Requires v^T M v = 1 and rho = v^T A v.  Returns the iteration count;
// sets *conv (stop test met) and *brk (non-positive curvature).
// Stops when sqrt(r.z / r0.z0) <= rtol or, with kTrack, when the estimated
// error of the Rayleigh quotient of v + t is <= lam_tol times it: the
// quotient is tracked as mu + f/m, f = w^T (A - mu M) w, m = w^T M w,
// w = v + t, from the step's dot products, and the error estimated from the
// tails of f (energy, factor c^2) and m (first order, factor c, scaled by
// |lambda - mu|), c the observed residual contraction.
template <int NT, int n, bool kTrack = false, bool kR = false, typename T>
MLQMC_DEV int jd_pcg(const PcgArrays<T>& a, double mu, double rho, double rtol, int maxit,
                     bool* conv, bool* brk, double lam_tol = 0.0) {
  constexpr int K = kTrack ? 6 : 3;
  const T hm = (T)mass_scale(n), muT = (T)mu;
  T* const v = a.v;
  T* const t = a.t;
  T* const r = a.r;
  T* const z = a.z;
  T* const p = a.p;
  T* const q = a.q;
  LDS_FOR_NODES(NT, n, k) {
    T d;
    const T av = pA<n, T, kR>(v, a.wx, a.wy, k, d);
    r[k] = -(av - (T)rho * hm * pM12<n>(v, k));
    t[k] = T(0);
  }
  __syncthreads();
  precondition<NT, n, kR>(a, r, z);
  // rz = r.(P^T z) = r.z - (r.v)(Mv.z);  p = P^T z
  double s3[3] = {0.0, 0.0, 0.0};
  LDS_FOR_NODES(NT, n, k) {
    s3[0] += (double)r[k] * (double)z[k];
    s3[1] += (double)(hm * pM12<n>(v, k)) * (double)z[k];
    s3[2] += (double)r[k] * (double)v[k];
  }
  block_sums<NT, 3>(s3, a.red);
  double rz = s3[0] - s3[2] * s3[1];
  const double rz0 = rz;
  LDS_FOR_NODES(NT, n, k) p[k] = z[k] - (T)s3[1] * v[k];
  __syncthreads();
  *conv = false;
  *brk = false;
  if (!(rz0 > 0.0)) {  // zero right-hand side: t = 0 solves it exactly
    *conv = true;
    return 0;
  }
  int it = 0;
  double f = rho - mu, mm = 1.0, dmp = 0.0, rzp = 0.0;
  while (it < maxit) {
    ++it;
    // q = (A - mu M) p;  pq = p.(P q) = p.q - (p.Mv)(v.q); with kTrack also
    // p.M p, t.M p, t.q for the Rayleigh-quotient tracking
    double s[K];
#pragma unroll
    for (int e = 0; e < K; ++e) s[e] = 0.0;
    LDS_FOR_NODES(NT, n, k) {
      T d;
      const T ap = pA<n, T, kR>(p, a.wx, a.wy, k, d);
      const T mp = hm * pM12<n>(p, k);
      const T qv = ap - muT * mp;
      const double pk = (double)p[k], qd = (double)qv;
      s[0] += pk * qd;
      s[1] += (double)v[k] * qd;
      s[2] += pk * (double)(hm * pM12<n>(v, k));
      if constexpr (kTrack) {
        s[3] += pk * (double)mp;
        s[4] += (double)t[k] * (double)mp;
        s[5] += (double)t[k] * qd;
      }
      q[k] = qv;  // may overwrite z, which is dead here
    }
    block_sums<NT, K>(s, a.red);
    const double pq = s[0] - s[2] * s[1];
    if (!(pq > 0.0)) {
      *brk = true;
      break;
    }
    const double alpha = rz / pq, c = s[1];
    bool lam_done = false;
    if constexpr (kTrack) {
      const double f1 = f + 2.0 * alpha * (s[1] + s[5]) + alpha * alpha * s[0];
      const double dm = 2.0 * alpha * (s[2] + s[4]) + alpha * alpha * s[3];
      const double m1 = mm + dm;
      double cr = rzp > 0.0 ? sqrt(rz / rzp) : 0.5;
      cr = fmin(fmax(cr, 0.05), 0.9);
      const double dmg = fmax(fabs(dm), cr * fabs(dmp));
      const double est = (fabs(f1 - f) * cr * cr / (1.0 - cr * cr) +
                          fabs(f1 / m1) * dmg * cr / (1.0 - cr)) / m1;
      lam_done = est <= lam_tol * fabs(mu + f1 / m1);
      f = f1;
      mm = m1;
      dmp = dm;
    }
    const T aT = (T)alpha, cT = (T)c;
    LDS_FOR_NODES(NT, n, k) {
      t[k] += aT * p[k];
      r[k] -= aT * (q[k] - cT * hm * pM12<n>(v, k));
    }
    __syncthreads();
    if (lam_done) {
      *conv = true;
      break;
    }
    precondition<NT, n, kR>(a, r, z);
    double u[3] = {0.0, 0.0, 0.0};
    LDS_FOR_NODES(NT, n, k) {
      const double zk = (double)z[k];
      u[0] += (double)r[k] * zk;
      u[1] += (double)(hm * pM12<n>(v, k)) * zk;
      u[2] += (double)r[k] * (double)v[k];
    }
    block_sums<NT, 3>(u, a.red);
    const double rzn = u[0] - u[2] * u[1];
    if (sqrt(fabs(rzn / rz0)) <= rtol) {
      *conv = true;
      break;
    }
    const double beta = rzn / rz;
    rzp = rz;
    rz = rzn;
    const T u1 = (T)u[1], bT = (T)beta;
    LDS_FOR_NODES(NT, n, k) p[k] = z[k] - u1 * v[k] + bT * p[k];
    __syncthreads();
  }
  return it;
}

// Padded edge weights of mesh n from a padded edge table of the batched
// path (rows of NSEG segments of (n + 2) n entries: [WX | WY], or the
// reaction's [RX | RY | RD]): w_e = a0 + sum_{j<S} y_j Phi[j][e], the
// segments written contiguously with stride P.  Entries that no stencil
// reads are finite and otherwise unused.
template <int NT, int n, typename T, int NSEG = 2>
MLQMC_DEV void weights_from_table(const double* __restrict__ phi, const double* ys, int S,
                                  double a0, T* w) {
  constexpr int P = Mesh<n>::P, PG = (n + 2) * n;
  for (int e = threadIdx.x; e < NSEG * P; e += NT) {
    const int seg = e / P, idx = e - seg * P;
    const double* src = phi + seg * PG + idx;
    double acc = a0;
    for (int j = 0; j < S; ++j) acc += ys[j] * src[(int64_t)j * NSEG * PG];
    w[e] = (T)acc;
  }
  __syncthreads();
}

}  // namespace lds
}  // namespace mlqmc
