// LDS-resident solvers for one sample per workgroup on meshes h = 1/N, N <= 32.
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
#pragma once

#include "common.h"

namespace mlqmc {
namespace lds {

template <int n>
struct Mesh {
  static constexpr int m = n - 1;
  static constexpr int D = m * m;        // interior nodes
  static constexpr int EX = (n - 1) * n; // horizontal edges
  static constexpr int EY = n * (n - 1); // vertical edges
  static constexpr int EW = EX + EY;
};

// LDS doubles used by the V-cycle levels strictly below mesh n:
// per level nc: weights (EW) + B, X, R (3 D).
template <int n>
constexpr int mg_scratch() {
  int s = 0;
  for (int c = n / 2; c >= 2; c /= 2) s += 2 * (c - 1) * c + 3 * (c - 1) * (c - 1);
  return s;
}

template <int NT, int n>
MLQMC_DEV void coarsen_all(const double* wx, const double* wy, double* nxt) {
  if constexpr (n > 2) {
    constexpr int nc = n / 2, mc = nc - 1;
    double* wxc = nxt;
    double* wyc = wxc + (nc - 1) * nc;
    for (int e = threadIdx.x; e < (nc - 1) * nc; e += NT) {
      const int J = e / nc + 1, I = e % nc;
      wxc[e] = coarsen_wx(wx, n, I, J);
    }
    for (int e = threadIdx.x; e < nc * (nc - 1); e += NT) {
      const int J = e / mc, I = e % mc + 1;
      wyc[e] = coarsen_wy(wy, n, I, J);
    }
    __syncthreads();
    constexpr int Dc = mc * mc;
    coarsen_all<NT, nc>(wxc, wyc, wyc + nc * (nc - 1) + 3 * Dc);
  }
}

// X = omega * B / diag  (first sweep from a zero start)
template <int NT, int n>
MLQMC_DEV void jacobi_first(const double* wx, const double* wy, const double* B, double* X) {
  constexpr int m = n - 1, D = m * m;
  for (int id = threadIdx.x; id < D; id += NT) {
    const int i = id % m + 1, j = id / m + 1;
    X[id] = kOmega * B[id] / stencil_diag(wx, wy, n, i, j);
  }
  __syncthreads();
}

// X <- X + omega (B - A X) / diag, new values staged in registers
template <int NT, int n>
MLQMC_DEV void jacobi_sweep(const double* wx, const double* wy, const double* B, double* X) {
  constexpr int m = n - 1, D = m * m, PT = (D + NT - 1) / NT;
  double nv[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int id = threadIdx.x + k * NT;
    if (id < D) {
      const int i = id % m + 1, j = id / m + 1;
      double d;
      const double ax = stencil_A(X, wx, wy, n, i, j, id, d);
      nv[k] = X[id] + kOmega * (B[id] - ax) / d;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int id = threadIdx.x + k * NT;
    if (id < D) X[id] = nv[k];
  }
  __syncthreads();
}

// One V-cycle X = K^{-1} B on mesh n; R is a residual scratch of D doubles,
// `nxt` the scratch of the coarser levels (weights already built there).
template <int NT, int n>
MLQMC_DEV void vcycle(const double* wx, const double* wy, const double* B, double* X,
                      double* R, double* nxt) {
  constexpr int m = n - 1, D = m * m;
  if constexpr (n == 2) {
    if (threadIdx.x == 0) X[0] = B[0] / stencil_diag(wx, wy, 2, 1, 1);
    __syncthreads();
  } else {
    constexpr int nc = n / 2, mc = nc - 1, Dc = mc * mc;
    const double* wxc = nxt;
    const double* wyc = wxc + (nc - 1) * nc;
    double* Bc = nxt + 2 * (nc - 1) * nc;
    double* Xc = Bc + Dc;
    double* Rc = Xc + Dc;
    jacobi_first<NT, n>(wx, wy, B, X);
    jacobi_sweep<NT, n>(wx, wy, B, X);
    for (int id = threadIdx.x; id < D; id += NT) {
      const int i = id % m + 1, j = id / m + 1;
      double d;
      R[id] = B[id] - stencil_A(X, wx, wy, n, i, j, id, d);
    }
    __syncthreads();
    for (int id = threadIdx.x; id < Dc; id += NT) {
      const int I = id % mc + 1, J = id / mc + 1;
      Bc[id] = restrict_at(R, n, I, J);
    }
    __syncthreads();
    vcycle<NT, nc>(wxc, wyc, Bc, Xc, Rc, Rc + Dc);
    for (int id = threadIdx.x; id < D; id += NT) {
      const int i = id % m + 1, j = id / m + 1;
      X[id] += prolong2_at(Xc, nc, i, j);
    }
    __syncthreads();
    jacobi_sweep<NT, n>(wx, wy, B, X);
    jacobi_sweep<NT, n>(wx, wy, B, X);
  }
}

// Xout = Xin + omega (B - A Xin) / diag (two distinct arrays)
template <int NT, int n>
MLQMC_DEV void jacobi_to(const double* wx, const double* wy, const double* B, const double* Xin,
                         double* Xout) {
  constexpr int m = n - 1, D = m * m;
  for (int id = threadIdx.x; id < D; id += NT) {
    const int i = id % m + 1, j = id / m + 1;
    double d;
    const double ax = stencil_A(Xin, wx, wy, n, i, j, id, d);
    Xout[id] = Xin[id] + kOmega * (B[id] - ax) / d;
  }
  __syncthreads();
}

// The same V-cycle for a top level whose arrays are too large for register
// staging (mesh 1/64 and finer): the sweeps alternate between X and R, the
// levels below run vcycle().
template <int NT, int n>
MLQMC_DEV void vcycle_pingpong(const double* wx, const double* wy, const double* B, double* X,
                               double* R, double* nxt) {
  constexpr int m = n - 1, D = m * m;
  constexpr int nc = n / 2, mc = nc - 1, Dc = mc * mc;
  const double* wxc = nxt;
  const double* wyc = wxc + (nc - 1) * nc;
  double* Bc = nxt + 2 * (nc - 1) * nc;
  double* Xc = Bc + Dc;
  double* Rc = Xc + Dc;
  jacobi_first<NT, n>(wx, wy, B, R);
  jacobi_to<NT, n>(wx, wy, B, R, X);
  for (int id = threadIdx.x; id < D; id += NT) {
    const int i = id % m + 1, j = id / m + 1;
    double d;
    R[id] = B[id] - stencil_A(X, wx, wy, n, i, j, id, d);
  }
  __syncthreads();
  for (int id = threadIdx.x; id < Dc; id += NT) {
    const int I = id % mc + 1, J = id / mc + 1;
    Bc[id] = restrict_at(R, n, I, J);
  }
  __syncthreads();
  vcycle<NT, nc>(wxc, wyc, Bc, Xc, Rc, Rc + Dc);
  for (int id = threadIdx.x; id < D; id += NT) {
    const int i = id % m + 1, j = id / m + 1;
    X[id] += prolong2_at(Xc, nc, i, j);
  }
  __syncthreads();
  jacobi_to<NT, n>(wx, wy, B, X, R);
  jacobi_to<NT, n>(wx, wy, B, R, X);
}

template <int NT, int n>
MLQMC_DEV void vcycle_top(const double* wx, const double* wy, const double* B, double* X,
                          double* R, double* nxt) {
  if constexpr (n > 32)
    vcycle_pingpong<NT, n>(wx, wy, B, X, R, nxt);
  else
    vcycle<NT, n>(wx, wy, B, X, R, nxt);
}

// Arrays of one projected-PCG solve on mesh N (all LDS, D doubles each except
// the weights and the multigrid scratch).
struct PcgArrays {
  double *wx, *wy, *v, *t, *r, *z, *p, *q, *mg, *red;
};

// ||v||_M^2 and v^T A v in one pass (all threads get both)
template <int NT, int n>
MLQMC_DEV void rayleigh_parts(const PcgArrays& a, const double* x, double& xMx, double& xAx) {
  constexpr int m = n - 1, D = m * m;
  double s[2] = {0.0, 0.0};
  for (int id = threadIdx.x; id < D; id += NT) {
    const int i = id % m + 1, j = id / m + 1;
    double d;
    const double ax = stencil_A(x, a.wx, a.wy, n, i, j, id, d);
    s[0] += x[id] * stencil_M12(x, n, i, j, id);
    s[1] += x[id] * ax;
  }
  block_sums<NT, 2>(s, a.red);
  xMx = s[0] * mass_scale(n);
  xAx = s[1];
}

template <int NT, int n>
MLQMC_DEV void scale_vec(double* x, double f) {
  constexpr int D = (n - 1) * (n - 1);
  for (int id = threadIdx.x; id < D; id += NT) x[id] *= f;
  __syncthreads();
}

// Projected PCG for  P (A - mu M) P^T t = -(A v - rho M v), t = 0 initially.
// Requires v^T M v = 1 and rho = v^T A v.  Returns the iteration count;
// sets *conv (stop test met) and *brk (non-positive curvature).
// Stops when sqrt(r.z / r0.z0) <= rtol or, with lam_tol > 0, when the
// estimated error of the Rayleigh quotient of v + t is <= lam_tol times it:
// the quotient is tracked as mu + f/m, f = w^T (A - mu M) w, m = w^T M w,
// w = v + t, from the step's dot products, and the error estimated from the
// tails of f (energy, factor c^2) and m (first order, factor c, scaled by
// |lambda - mu|), c the observed residual contraction.
template <int NT, int n, bool kTrack = false>
MLQMC_DEV int jd_pcg(const PcgArrays& a, double mu, double rho, double rtol, int maxit,
                     bool* conv, bool* brk, double lam_tol = 0.0) {
  constexpr int K = kTrack ? 6 : 3;
  constexpr int m = n - 1, D = m * m;
  const double hm = mass_scale(n);
  double* const v = a.v;
  double* const t = a.t;
  double* const r = a.r;
  double* const z = a.z;
  double* const p = a.p;
  double* const q = a.q;
  for (int id = threadIdx.x; id < D; id += NT) {
    const int i = id % m + 1, j = id / m + 1;
    double d;
    const double av = stencil_A(v, a.wx, a.wy, n, i, j, id, d);
    r[id] = -(av - rho * hm * stencil_M12(v, n, i, j, id));
    t[id] = 0.0;
  }
  __syncthreads();
  vcycle_top<NT, n>(a.wx, a.wy, r, z, q, a.mg);
  // rz = r.(P^T z) = r.z - (r.v)(Mv.z);  p = P^T z
  double s3[3] = {0.0, 0.0, 0.0};
  for (int id = threadIdx.x; id < D; id += NT) {
    const int i = id % m + 1, j = id / m + 1;
    s3[0] += r[id] * z[id];
    s3[1] += hm * stencil_M12(v, n, i, j, id) * z[id];
    s3[2] += r[id] * v[id];
  }
  block_sums<NT, 3>(s3, a.red);
  double rz = s3[0] - s3[2] * s3[1];
  const double rz0 = rz;
  for (int id = threadIdx.x; id < D; id += NT) p[id] = z[id] - s3[1] * v[id];
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
    // q = (A - mu M) p;  pq = p.(P q) = p.q - (p.Mv)(v.q); with lam_tol also
    // p.M p, t.M p, t.q for the Rayleigh-quotient tracking
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int id = threadIdx.x; id < D; id += NT) {
      const int i = id % m + 1, j = id / m + 1;
      double d;
      const double ap = stencil_A(p, a.wx, a.wy, n, i, j, id, d);
      const double mp = hm * stencil_M12(p, n, i, j, id);
      const double qv = ap - mu * mp;
      q[id] = qv;
      s[0] += p[id] * qv;
      s[1] += v[id] * qv;
      s[2] += p[id] * hm * stencil_M12(v, n, i, j, id);
      if constexpr (kTrack) {
        s[3] += p[id] * mp;
        s[4] += t[id] * mp;
        s[5] += t[id] * qv;
      }
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
    for (int id = threadIdx.x; id < D; id += NT) {
      const int i = id % m + 1, j = id / m + 1;
      t[id] += alpha * p[id];
      r[id] -= alpha * (q[id] - c * hm * stencil_M12(v, n, i, j, id));
    }
    __syncthreads();
    if (lam_done) {
      *conv = true;
      break;
    }
    vcycle_top<NT, n>(a.wx, a.wy, r, z, q, a.mg);
    double u[3] = {0.0, 0.0, 0.0};
    for (int id = threadIdx.x; id < D; id += NT) {
      const int i = id % m + 1, j = id / m + 1;
      u[0] += r[id] * z[id];
      u[1] += hm * stencil_M12(v, n, i, j, id) * z[id];
      u[2] += r[id] * v[id];
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
    for (int id = threadIdx.x; id < D; id += NT) p[id] = z[id] - u[1] * v[id] + beta * p[id];
    __syncthreads();
  }
  return it;
}

// Edge weights of mesh n from an edge table: w_e = a0 + sum_{j<S} y_j Phi[j][e].
template <int NT, int n>
MLQMC_DEV void weights_from_table(const double* __restrict__ phi, const double* ys, int S,
                                  double a0, double* wx) {
  constexpr int EW = Mesh<n>::EW;
  for (int e = threadIdx.x; e < EW; e += NT) {
    double acc = a0;
    for (int j = 0; j < S; ++j) acc += ys[j] * phi[(int64_t)j * EW + e];
    wx[e] = acc;  // wy follows wx contiguously
  }
  __syncthreads();
}

}  // namespace lds
}  // namespace mlqmc
