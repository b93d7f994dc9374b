// Device helpers shared by the kernels: fixed-order wavefront/workgroup
// reductions and the P1 stencils on the uniform "/" triangulation.
//
// Storage of one sample on mesh h = 1/n (m = n-1 interior nodes per side):
//   x  [m*m]         interior node (i,j), 1 <= i,j <= m, at (j-1)*m + (i-1)
//   wx [(n-1)*n]     horizontal edge (i,j)-(i+1,j), 1 <= j <= m, 0 <= i <= m, at (j-1)*n + i
//   wy [n*(n-1)]     vertical edge (i,j)-(i,j+1), 0 <= j <= m, 1 <= i <= m,  at j*m + (i-1)
// The edge weight is the stiffness coupling: on right-isosceles P1 elements the
// hypotenuse couplings vanish and each leg of an element with coefficient a_K
// contributes a_K/2, so (A x)_p = sum over the four grid edges pq of w_pq (x_p - x_q)
// with x = 0 on the boundary.  The consistent mass matrix is the 7-point stencil
// h^2/12 [6 at p; 1 at E, W, N, S, NE, SW].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLQMC_DEV __device__ __forceinline__

namespace mlqmc {

// Weights of the two Jacobi sweeps of each multigrid smoothing step: the
// degree-2 Chebyshev smoother for the interval [0.4, 2] of D^{-1} A (the
// sweeps' weights are the reciprocals of the two Chebyshev nodes
// 1.2 +- 0.8 cos(pi/4)), which damps that interval by 2/7 per smoothing step
// against 0.36 for two sweeps of weight 0.8, and stays below 1 in modulus on
// all of (0, 2].  Pre- and post-smoothing use the same pair, so the V-cycle
// stays symmetric (both sweeps are polynomials in D^{-1} A and commute).
constexpr double kOmega1 = 0.5663522991524661;
constexpr double kOmega2 = 1.5765048437046771;
// The degree-3 Chebyshev smoother for the same interval (nodes
// 1.2 + 0.8 cos((2i - 1) pi / 6)), which damps it by 1/9 per smoothing step;
// used by the V-cycle levels below the batched ones, where one more sweep in
// LDS costs little next to the PCG iteration it saves.
constexpr double kCheb3[3] = {0.5283121635129678, 0.8333333333333334, 1.9716878364870327};

// Butterfly sum over the 64 lanes; every lane ends with the same value
// (each stage adds the same two operands in both partner lanes).
MLQMC_DEV double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

MLQMC_DEV float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroup sums of K values, returned to every thread.  `red` is LDS scratch
// of K * (NT/64) doubles.  Fixed order: lanes, then waves in index order.
template <int NT, int K>
MLQMC_DEV void block_sums(double (&v)[K], double* red) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) red[k * NW + wid] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[k * NW + w];
    v[k] = s;
  }
  __syncthreads();
}

// ---- stencils; `n` may be a compile-time or run-time mesh size ----

template <typename T>
MLQMC_DEV T stencil_A(const T* __restrict__ x, const T* __restrict__ wx,
                      const T* __restrict__ wy, int n, int i, int j, int id, T& diag) {
  const int m = n - 1;
  const T xc = x[id];
  const T xw = (i > 1) ? x[id - 1] : T(0);
  const T xe = (i < m) ? x[id + 1] : T(0);
  const T xs = (j > 1) ? x[id - m] : T(0);
  const T xn = (j < m) ? x[id + m] : T(0);
  const T ww = wx[(j - 1) * n + (i - 1)];
  const T we = wx[(j - 1) * n + i];
  const T ws = wy[(j - 1) * m + (i - 1)];
  const T wn = wy[j * m + (i - 1)];
  diag = ww + we + ws + wn;
  return ww * (xc - xw) + we * (xc - xe) + ws * (xc - xs) + wn * (xc - xn);
}

template <typename T>
MLQMC_DEV T stencil_diag(const T* __restrict__ wx, const T* __restrict__ wy, int n, int i,
                         int j) {
  const int m = n - 1;
  return wx[(j - 1) * n + (i - 1)] + wx[(j - 1) * n + i] + wy[(j - 1) * m + (i - 1)] +
         wy[j * m + (i - 1)];
}

// (M x)_p without the h^2/12 factor: 6 x_p + E + W + N + S + NE + SW.
template <typename T>
MLQMC_DEV T stencil_M12(const T* __restrict__ x, int n, int i, int j, int id) {
  const int m = n - 1;
  T s = T(6) * x[id];
  if (i > 1) s += x[id - 1];
  if (i < m) s += x[id + 1];
  if (j > 1) s += x[id - m];
  if (j < m) s += x[id + m];
  if (i < m && j < m) s += x[id + m + 1];
  if (i > 1 && j > 1) s += x[id - m - 1];
  return s;
}

// h^2 / 12 for h = 1/n
MLQMC_DEV double mass_scale(int n) { return 1.0 / (12.0 * double(n) * double(n)); }

// P1 interpolation of a coarse field at fine node (i,j), ratio r = nh/nH:
// barycentric evaluation on the coarse "/" triangle containing the node.
template <typename T>
MLQMC_DEV T interp_coarse(const T* __restrict__ uH, int nH, int r, int i, int j) {
  const int mH = nH - 1;
  const int I = i / r, J = j / r;
  const int li = i - I * r, lj = j - J * r;
  auto U = [&](int a, int b) -> T {
    return (a >= 1 && a <= mH && b >= 1 && b <= mH) ? uH[(b - 1) * mH + (a - 1)] : T(0);
  };
  const T xi = T(li) / T(r), eta = T(lj) / T(r);
  const T u00 = U(I, J);
  if (lj <= li) {  // lower triangle (I,J),(I+1,J),(I+1,J+1)
    const T u10 = U(I + 1, J), u11 = U(I + 1, J + 1);
    return u00 + xi * (u10 - u00) + eta * (u11 - u10);
  } else {         // upper triangle (I,J),(I+1,J+1),(I,J+1)
    const T u01 = U(I, J + 1), u11 = U(I + 1, J + 1);
    return u00 + eta * (u01 - u00) + xi * (u11 - u01);
  }
}

// Weighted restriction (transpose of the 2:1 P1 prolongation) at coarse node
// (I,J) from a fine field rf on mesh n = 2 nc: fine node (2I,2J) with weight 1,
// its E, W, N, S, NE, SW neighbours with weight 1/2 (all interior).
template <typename T>
MLQMC_DEV T restrict_at(const T* __restrict__ rf, int n, int I, int J) {
  const int m = n - 1;
  const int id = (2 * J - 1) * m + (2 * I - 1);
  return rf[id] + T(0.5) * (rf[id - 1] + rf[id + 1] + rf[id - m] + rf[id + m] +
                            rf[id + m + 1] + rf[id - m - 1]);
}

// 2:1 prolongation value at fine node (i,j) from coarse field xc (mesh nc = n/2).
template <typename T>
MLQMC_DEV T prolong2_at(const T* __restrict__ xc, int nc, int i, int j) {
  const int mc = nc - 1;
  auto U = [&](int a, int b) -> T {
    return (a >= 1 && a <= mc && b >= 1 && b <= mc) ? xc[(b - 1) * mc + (a - 1)] : T(0);
  };
  const int I = i >> 1, J = j >> 1;
  if (!(i & 1) && !(j & 1)) return U(I, J);
  if ((i & 1) && !(j & 1)) return T(0.5) * (U(I, J) + U(I + 1, J));
  if (!(i & 1) && (j & 1)) return T(0.5) * (U(I, J) + U(I, J + 1));
  return T(0.5) * (U(I, J) + U(I + 1, J + 1));
}

// Coarse edge weights: the mean of the two collinear fine edges.
template <typename T>
MLQMC_DEV T coarsen_wx(const T* __restrict__ wx, int n, int I, int J) {
  return T(0.5) * (wx[(2 * J - 1) * n + 2 * I] + wx[(2 * J - 1) * n + 2 * I + 1]);
}
template <typename T>
MLQMC_DEV T coarsen_wy(const T* __restrict__ wy, int n, int I, int J) {
  const int m = n - 1;
  return T(0.5) * (wy[(2 * J) * m + (2 * I - 1)] + wy[(2 * J + 1) * m + (2 * I - 1)]);
}

}  // namespace mlqmc
