// Batched fine-mesh kernels of the two-grid update (Algorithm 1 steps 2-4) for
// meshes too large for LDS (h <= 1/64).
//
// Padded layout (mesh h = 1/n, n a power of two): node (i, j), 0 <= i < n,
// 0 <= j <= n+1, at k = j*n + i, (n+2) n positions per sample.  Column 0 and
// rows 0, n and n+1 hold the homogeneous Dirichlet values (zeros); the right
// boundary node (n, j) aliases the left boundary node (0, j+1), also zero (row
// n+1 holds the alias of (n, n), the north-east neighbour of the last interior
// node).  Hence every stencil below is branch-free:
//   E/W = k+-1, N/S = k+-n, NE = k+n+1, SW = k-n-1.
// Edge weights use the same indexing: WX[k] is the horizontal edge ending at
// node k from the west ((i-1,j)-(i,j), so the east edge of k is WX[k+1]), and
// WY[k] the vertical edge ending at k from the south ((i,j-1)-(i,j), north edge
// WY[k+n]).  A sample's weights are [WX | WY], 2 (n+2) n values.  Entries that
// are not edges of an interior node are never read.  Weights use the same
// (n+2) n positions per half.
// With the reaction term of Problem 2 (kR) a sample's block is
// [WX | WY | RX | RY | RD], 5 (n+2) n values: RX, RY the means of b over the two
// elements of each horizontal and vertical edge, indexed as WX, WY, and RD
// those of each "/" diagonal, stored at its north-east end (RD[k] is the
// south-west and RD[k+n+1] the north-east diagonal of node k).  The operator
// is then A + R with (R x)_k = h^2/12 sum over the six edges e at k of
// r_e (x_k + x_e) (element mass matrices weighted by b).
//
// Work mapping: a launch covers B samples x nblk blocks (column blocks x row
// strips of one sample).  Hardware block L runs on XCD L mod 8; sample b is
// mapped to XCD b mod 8 and its blocks to consecutive slots of that XCD, so
// the halo rows a block shares with its neighbours stay in one L2.
//
// Storage type T (double, or float in mixed precision) holds the projected-PCG
// vectors and the smoother's weights; dot products accumulate in FP64, and the
// right-hand side and the Rayleigh quotient are formed in FP64 from FP64 weights
// and the FP64 prolongated vector (lds_mg.h describes the projected solve).
// Samples whose solve has finished are skipped (active[b] == 0).
#include <algorithm>
#include <cstdlib>

#include "../../include/mlqmc.h"
#include "common.h"
#include "kernels.h"

namespace mlqmc {
namespace {

template <typename T>
__device__ __forceinline__ T diagW(const T* wx, const T* wy, int k, int n) {
  return wx[k] + wx[k + 1] + wy[k] + wy[k + n];
}

// (A x)_k and the diagonal
template <typename T>
__device__ __forceinline__ T applyA(const T* x, const T* wx, const T* wy, int k, int n, T& d) {
  const T c = x[k];
  const T ww = wx[k], we = wx[k + 1], ws = wy[k], wn = wy[k + n];
  d = ww + we + ws + wn;
  return ww * (c - x[k - 1]) + we * (c - x[k + 1]) + ws * (c - x[k - n]) + wn * (c - x[k + n]);
}

// 6 x_k + E + W + N + S + NE + SW  (the mass stencil without h^2/12)
template <typename T>
__device__ __forceinline__ T applyM12(const T* x, int k, int n) {
  return T(6) * x[k] + x[k - 1] + x[k + 1] + x[k - n] + x[k + n] + x[k + n + 1] + x[k - n - 1];
}

// 2:1 P1 prolongation at fine (i, j) from a padded coarse field (nc = n/2):
// the mean of the coarse values at ((i>>1), (j>>1)) and ((i+1)>>1, (j+1)>>1)
// (equal points at coarse nodes; the two ends of the horizontal, vertical or
// "/" coarse edge otherwise).
template <typename T>
__device__ __forceinline__ T prolong2(const T* xc, int nc, int i, int j) {
  return T(0.5) * (xc[(j >> 1) * nc + (i >> 1)] + xc[((j + 1) >> 1) * nc + ((i + 1) >> 1)]);
}

// ---------------------------------------------------------------- row marching
//
// Stencil kernels march a block of NTC threads (one per column of a column
// block [c0, c0 + NTC)) up a strip of rows [j0, j1).  The stencil's source
// field is computed once per position into a 4-row LDS ring (with one halo
// column on each side), so every neighbour comes from LDS and every input is
// read from global memory once per strip; one barrier per row.

struct MGeo {
  int n, lg, P;
  int cb;      // column blocks per row (n / NTC)
  int R;       // rows per strip
  int nblk;    // column blocks x strips per sample
  int64_t B;
};

// Strips per sample: as few as keep about `target` workgroups in flight
// (one strip per sample for large batches, so no halo row is read twice);
// with several strips, odd strips march downwards so two neighbours read
// their shared halo rows at the same time and the second read hits in L2.
// The target is a per-mesh tuning value set before each batch.
constexpr int64_t kDefaultTargetBlocks = 65536;
// Jacobi sweeps per smoothing step in the fused V-cycle kernels of the
// batched levels (the kernels take 2 or 3; the weights follow from the
// count).  Three saved under 0.1 PCG iterations per sample on 1/128 and 1/256
// while every pre/post launch got longer (mixed-precision levels took 5-9 %
// longer), so two.
constexpr int kFineSweeps = 2;
thread_local int64_t t_target_blocks = kDefaultTargetBlocks;
inline int strips_for(int rows, int64_t units) {
  const int64_t tb = t_target_blocks;
  int s = (int)((tb + units - 1) / std::max<int64_t>(units, 1));
  s = std::max(1, std::min(s, (rows + 7) / 8));
  return s;
}

template <int NTC>
inline MGeo mgeo(int n, int64_t B) {
  MGeo g;
  g.n = n;
  g.lg = 0;
  while ((1 << g.lg) < n) ++g.lg;
  g.P = (n + 2) * n;
  g.cb = n / NTC;
  const int strips = strips_for(n - 1, B * g.cb);
  g.R = (n - 1 + strips - 1) / strips;
  g.nblk = g.cb * ((n - 1 + g.R - 1) / g.R);
  g.B = B;
  return g;
}

template <int NTC>
__device__ __forceinline__ bool map_march(const MGeo& g, int64_t& b, int& c0, int& j0, int& j1,
                                          int& blk, int& dir) {
  const int64_t L = blockIdx.x;
  const int xcd = (int)(L & 7);
  const int64_t q = L >> 3;
  b = ((q / g.nblk) << 3) + xcd;
  blk = (int)(q % g.nblk);
  if (b >= g.B) return false;
  c0 = (blk % g.cb) * NTC;
  const int strip = blk / g.cb;
  j0 = 1 + strip * g.R;
  j1 = min(j0 + g.R, g.n);
  dir = (strip & 1) ? -1 : 1;
  return true;
}

// March a block of NTC threads (columns c0 .. c0+NTC-1) through the rows
// [j0, j1) of a strip, upwards (dir = 1) or downwards, with a ring of 4 rows
// in LDS holding the stencil's source field (with one halo column each side)
// and one barrier per row.  Every global input is requested one row step
// before use: fetch(k) loads the raw sources of ring position k, value(f)
// turns them into the ring entry (0 outside the interior); fetch_row(k) loads
// the stencil row's own inputs; body(j, k, rs, rc, rn, ci, row inputs, ring
// sources of (j, c)) with south, centre and north ring rows.
template <typename T, int NTC, class Fetch, class Value, class FetchRow, class Body>
__device__ __forceinline__ void march_pf(T (*ring)[NTC + 2], const MGeo& g, int c0, int j0,
                                         int j1, int dir, Fetch fetch, Value value,
                                         FetchRow fetch_row, Body body) {
  using F = decltype(fetch(0));
  using R = decltype(fetch_row(0));
  const int n = g.n, tx = threadIdx.x, c = c0 + tx, ci = tx + 1;
  const bool hl = (tx == 0), hr = (tx == NTC - 1);
  const int ch = hl ? c0 - 1 : c0 + NTC;
  const bool hok = (hl && c0 >= 2) || (hr && c0 + NTC <= n - 1);
  struct Src {
    F f, h;
    bool ok, hk;
  };
  auto fsrc = [&](int j, Src& s) {
    const bool rowok = (j >= 1 && j <= n - 1);
    s.ok = rowok && c >= 1;
    s.hk = rowok && hok;
    if (s.ok) s.f = fetch(j * n + c);
    if (s.hk) s.h = fetch(j * n + ch);
  };
  auto store = [&](int j, const Src& s) {
    T* row = ring[j & 3];
    row[ci] = s.ok ? value(s.f) : T(0);
    if (hl) row[0] = s.hk ? value(s.h) : T(0);
    if (hr) row[NTC + 1] = s.hk ? value(s.h) : T(0);
  };
  auto frow = [&](int j, R& r) {
    if (c >= 1 && j >= j0 && j < j1) r = fetch_row(j * n + c);
  };
  const int jf = dir > 0 ? j0 : j1 - 1;
  const int count = j1 - j0;
  Src s, sn;
  fsrc(jf - dir, s);
  store(jf - dir, s);
  fsrc(jf, s);
  store(jf, s);
  F cur = s.f;  // ring sources of the row the next stencil step handles
  fsrc(jf + dir, sn);
  R rw;
  frow(jf, rw);
  for (int i = 0; i < count; ++i) {
    const int j = jf + i * dir;
    store(j + dir, sn);
    const F nxt = sn.f;
    const R rc = rw;
    if (i + 1 < count) {
      fsrc(j + 2 * dir, sn);
      frow(j + dir, rw);
    }
    __syncthreads();
    if (c >= 1) body(j, j * n + c, ring[(j - 1) & 3], ring[j & 3], ring[(j + 1) & 3], ci, rc, cur);
    cur = nxt;
  }
}

// weight arrays per sample block: [WX | WY], or with the reaction [WX | WY | RX | RY | RD]
template <bool kR>
constexpr int wblk() {
  return kR ? 5 : 2;
}

// The coefficients of node k: the four edge weights of A and, with the
// reaction, h^2/12 times the means of b on the six edges at k (west, east,
// south, north, south-west, north-east).
template <typename W, bool kR = false>
struct Wts {
  W ww, we, ws, wn;
  W rw, re, rs, rn, rsw, rne;
};
template <typename W, bool kR = false>
__device__ __forceinline__ Wts<W, kR> load_wts(const W* wx, const W* wy, int k, int n, int P = 0,
                                               W hm = W(0)) {
  Wts<W, kR> o;
  o.ww = wx[k];
  o.we = wx[k + 1];
  o.ws = wy[k];
  o.wn = wy[k + n];
  if constexpr (kR) {
    const W* rx = wx + 2 * P;
    const W* ry = wx + 3 * P;
    const W* rd = wx + 4 * P;
    o.rw = hm * rx[k];
    o.re = hm * rx[k + 1];
    o.rs = hm * ry[k];
    o.rn = hm * ry[k + n];
    o.rsw = hm * rd[k];
    o.rne = hm * rd[k + n + 1];
  }
  return o;
}
// The same widened to FP64 from weights stored in W, with the reaction scale
// applied in FP64 (rounding the scale to FP32 would shift every reaction
// term by one and the same relative amount, and the eigenvalue with it).
template <typename W, bool kR = false>
__device__ __forceinline__ Wts<double, kR> load_wts_fp64(const W* wx, const W* wy, int k, int n,
                                                         int P, double hm) {
  Wts<double, kR> o;
  o.ww = (double)wx[k];
  o.we = (double)wx[k + 1];
  o.ws = (double)wy[k];
  o.wn = (double)wy[k + n];
  if constexpr (kR) {
    const W* rx = wx + 2 * P;
    const W* ry = wx + 3 * P;
    const W* rd = wx + 4 * P;
    o.rw = hm * (double)rx[k];
    o.re = hm * (double)rx[k + 1];
    o.rs = hm * (double)ry[k];
    o.rn = hm * (double)ry[k + n];
    o.rsw = hm * (double)rd[k];
    o.rne = hm * (double)rd[k + n + 1];
  }
  return o;
}
// ((A [+ R]) x)_k from a ring of x rows (south, centre, north; column ci)
template <typename T, typename W, bool kR = false>
__device__ __forceinline__ T ring_Aw(const T* rs, const T* rc, const T* rn, int ci,
                                     const Wts<W, kR>& w) {
  const T c = rc[ci];
  T a = (T)w.ww * (c - rc[ci - 1]) + (T)w.we * (c - rc[ci + 1]) + (T)w.ws * (c - rs[ci]) +
        (T)w.wn * (c - rn[ci]);
  if constexpr (kR)
    a += (T)w.rw * (c + rc[ci - 1]) + (T)w.re * (c + rc[ci + 1]) + (T)w.rs * (c + rs[ci]) +
         (T)w.rn * (c + rn[ci]) + (T)w.rsw * (c + rs[ci - 1]) + (T)w.rne * (c + rn[ci + 1]);
  return a;
}

template <int NTC, int K>
__device__ __forceinline__ void write_partials_m(double (&s)[K], double* part, int64_t b,
                                                 int blk, int nblk) {
  __shared__ double red[K * (NTC / 64)];
  block_sums<NTC, K>(s, red);
  if (threadIdx.x == 0) {
    const int64_t base = (b * nblk + blk) * K;
#pragma unroll
    for (int k = 0; k < K; ++k) part[base + k] = s[k];
  }
}

template <typename T>
__device__ __forceinline__ T ring_M12(const T* rs, const T* rc, const T* rn, int ci) {
  return T(6) * rc[ci] + rc[ci - 1] + rc[ci + 1] + rs[ci] + rn[ci] + rn[ci + 1] + rs[ci - 1];
}

// ---------------------------------------------------------------- setup

// zero the Dirichlet rows/column of `cnt` padded arrays of B samples (mesh n)
struct ZeroArgs {
  void* p[10];
  int cnt;
  int elem;  // bytes per element
};
// grid: x = (blocks per sample) x samples, y = arrays
__global__ __launch_bounds__(256) void k_zero_boundary(int n, int64_t B, int per_blocks,
                                                       ZeroArgs za) {
  const int64_t b = blockIdx.x / per_blocks;
  const int xb = (int)(blockIdx.x - b * per_blocks);
  const int a = blockIdx.y;
  if (b >= B || a >= za.cnt) return;
  const int P = (n + 2) * n;
  // positions: row 0 (n), rows n and n+1 (2n), column 0 of rows 1..n-1 (n-1)
  for (int t = xb * 256 + threadIdx.x; t < 4 * n - 1; t += per_blocks * 256) {
    const int k = t < n ? t : (t < 3 * n ? n * n + (t - n) : (t - 3 * n + 1) * n);
    if (za.elem == 8)
      static_cast<double*>(za.p[a])[b * P + k] = 0.0;
    else
      static_cast<float*>(za.p[a])[b * P + k] = 0.f;
  }
}

// The prolongated coarse eigenvector v = P u_H, evaluated where it is needed
// instead of being stored: node k of mesh n (padded layout) of sample b.
// Padding positions (column 0, rows 0 and n) come out as 0.
struct Coarse {
  const double* uH;  // [B x (nH - 1)^2] interior layout
  int nH, lr;        // coarse mesh, log2(n / nH)
  double inv_r;      // 2^-lr
};
// In two parts, so that a row-marching kernel can request the loads a row
// step before it needs the value: coarse_src loads the three vertices of the
// coarse triangle holding the node (u00, u11 and the third, (I+1, J) below
// the diagonal or (I, J+1) above it) and keeps the node's offsets in the
// coarse square; coarse_val interpolates, barycentric on that triangle (the
// arithmetic of interp_coarse, with the power-of-two ratio 2^lr: 1/r is
// exact).
struct CoarseSrc {
  double u00, u11, ux;
  int li, lj;
};
__device__ __forceinline__ CoarseSrc coarse_src(const Coarse& cv, const MGeo& g, int64_t b,
                                                int k) {
  const int mH = cv.nH - 1, i = k & (g.n - 1), j = k >> g.lg, r = 1 << cv.lr;
  const double* uH = cv.uH + b * (int64_t)(mH * mH);
  const int I = i >> cv.lr, J = j >> cv.lr;
  CoarseSrc s;
  s.li = i & (r - 1);
  s.lj = j & (r - 1);
  auto U = [&](int a, int c) -> double {
    return (a >= 1 && a <= mH && c >= 1 && c <= mH) ? uH[(c - 1) * mH + (a - 1)] : 0.0;
  };
  const bool lower = s.lj <= s.li;
  s.u00 = U(I, J);
  s.u11 = U(I + 1, J + 1);
  s.ux = U(lower ? I + 1 : I, lower ? J : J + 1);
  return s;
}
__device__ __forceinline__ double coarse_val(const Coarse& cv, const CoarseSrc& s) {
  const double xi = s.li * cv.inv_r, eta = s.lj * cv.inv_r;
  if (s.lj <= s.li) return s.u00 + xi * (s.ux - s.u00) + eta * (s.u11 - s.ux);
  return s.u00 + eta * (s.ux - s.u00) + xi * (s.u11 - s.ux);
}

// interior-layout prolongation for the component entry point
__global__ __launch_bounds__(256) void k_prolong_interior(int xblk, int nH, int nh, int64_t B,
                                                          const double* __restrict__ uH,
                                                          double* __restrict__ uh) {
  const int mH = nH - 1, mh = nh - 1, Dh = mh * mh;
  const int64_t b = blockIdx.x / xblk;  // grid x = xblk blocks per sample x samples
  const int id = (int)(blockIdx.x - b * xblk) * 256 + threadIdx.x;
  if (id >= Dh || b >= B) return;
  const int j = id / mh + 1, i = id - (j - 1) * mh + 1;
  uh[b * Dh + id] = interp_coarse(uH + b * (int64_t)(mH * mH), nH, nh / nH, i, j);
}

// padded weights of mesh n/2 from those of mesh n: each coarse edge weight is
// the mean of the two collinear fine edges it covers (horizontal, vertical
// and, with the reaction, the "/" diagonal of a coarse square, which covers the
// diagonals of fine squares (2I, 2J) and (2I+1, 2J+1))
template <typename T, bool kR>
__global__ __launch_bounds__(256) void k_coarsen(int xblk, int n, int64_t B, const T* __restrict__ w,
                                                 T* __restrict__ wc) {
  const int nc = n / 2;
  const int P = (n + 2) * n, Pc = (nc + 2) * nc;
  const int64_t b = blockIdx.x / xblk;  // grid x = xblk blocks per sample x samples
  const int e = (int)(blockIdx.x - b * xblk) * 256 + threadIdx.x;
  if (e >= wblk<kR>() * Pc || b >= B) return;
  const int seg = e / Pc, f = e - seg * Pc;  // [WX | WY | RX | RY | RD]
  const T* src = w + b * wblk<kR>() * P + (int64_t)seg * P;
  const int J = f / nc, I = f % nc;
  T val = T(0);
  if (seg == 0 || seg == 2) {  // edge (I-1,J)-(I,J), stored at J*nc + I (I = 0: (nc, J-1))
    const int Ie = (I == 0) ? nc : I, Je = (I == 0) ? J - 1 : J;
    if (Je >= 1 && Je <= nc - 1)
      val = T(0.5) * (src[2 * Je * n + 2 * Ie - 1] + src[2 * Je * n + 2 * Ie]);
  } else if (seg == 1 || seg == 3) {  // edge (I,J-1)-(I,J), stored at J*nc + I
    if (J >= 1 && J <= nc && I >= 1)
      val = T(0.5) * (src[(2 * J - 1) * n + 2 * I] + src[2 * J * n + 2 * I]);
  } else {  // diagonal of coarse square (Ic, Jc) at its north-east end (Jc+1)*nc + Ic+1
    const int Ic = (I == 0) ? nc - 1 : I - 1, Jc = (I == 0) ? J - 2 : J - 1;
    if (Ic >= 0 && Ic <= nc - 1 && Jc >= 0 && Jc <= nc - 1)
      val = T(0.5) * (src[(2 * Jc + 1) * n + 2 * Ic + 1] + src[(2 * Jc + 2) * n + 2 * Ic + 2]);
  }
  wc[b * wblk<kR>() * Pc + e] = val;
}

// partials: v.M12 v, v.A v  (raw FP64 v; the weights in their storage
// precision W, the arithmetic in FP64)
template <typename W, int NTC, bool kR>
__global__ __launch_bounds__(NTC) void k_setup_dots(MGeo g, Coarse cv,
                                                    const W* __restrict__ w,
                                                    double* __restrict__ part) {
  __shared__ double ring[4][NTC + 2];
  int64_t b;
  int c0, j0, j1, blk, dir;
  if (!map_march<NTC>(g, b, c0, j0, j1, blk, dir)) return;
  const W* wx = w + b * wblk<kR>() * g.P;
  const W* wy = wx + g.P;
  const double hm = mass_scale(g.n);
  double s[2] = {0.0, 0.0};
  march_pf<double, NTC>(
      ring, g, c0, j0, j1, dir, [&](int k) { return coarse_src(cv, g, b, k); },
      [&](const CoarseSrc& f) { return coarse_val(cv, f); },
      [&](int k) { return load_wts_fp64<W, kR>(wx, wy, k, g.n, g.P, hm); },
      [&](int, int, const double* rs, const double* rc, const double* rn, int ci,
          const Wts<double, kR>& wt, const CoarseSrc&) {
        const double av = ring_Aw(rs, rc, rn, ci, wt);
        s[0] += rc[ci] * ring_M12(rs, rc, rn, ci);
        s[1] += rc[ci] * av;
      });
  write_partials_m<NTC, 2>(s, part, b, blk, g.nblk);
}

// r = -(A v_n - rho M v_n) (FP64 arithmetic on the weights of storage type
// T), vn = v_n, mvn = M v_n (t starts at 0 without being stored: the PCG
// kernels read t only from its third step on)
template <typename T, int NTC, bool kR>
__global__ __launch_bounds__(NTC) void k_setup_rhs(MGeo g, Coarse cv,
                                                   const T* __restrict__ w, FineState S,
                                                   T* __restrict__ r, T* __restrict__ vn,
                                                   T* __restrict__ mvn) {
  __shared__ double ring[4][NTC + 2];
  int64_t b;
  int c0, j0, j1, blk, dir;
  if (!map_march<NTC>(g, b, c0, j0, j1, blk, dir)) return;
  const T* wx = w + b * wblk<kR>() * g.P;
  const T* wy = wx + g.P;
  const double vs = S.vs[b], rho = S.rho[b], hm = mass_scale(g.n);
  march_pf<double, NTC>(
      ring, g, c0, j0, j1, dir, [&](int k) { return coarse_src(cv, g, b, k); },
      [&](const CoarseSrc& f) { return coarse_val(cv, f); },
      [&](int k) { return load_wts_fp64<T, kR>(wx, wy, k, g.n, g.P, hm); },
      [&](int, int k, const double* rs, const double* rc, const double* rn, int ci,
          const Wts<double, kR>& wt, const CoarseSrc&) {
                       const double av = ring_Aw(rs, rc, rn, ci, wt);
                       const double mv = hm * ring_M12(rs, rc, rn, ci);
                       const double rv = -vs * (av - rho * mv);
                       const T rT = (T)rv;
                       const int64_t o = b * g.P + k;
                       __builtin_nontemporal_store(rT, &r[o]);
                       __builtin_nontemporal_store((T)(vs * rc[ci]), &vn[o]);
                       __builtin_nontemporal_store((T)(vs * mv), &mvn[o]);
                     });
}

// ---------------------------------------------------------------- PCG

// p = z - c2 vn + beta p_in (first: beta = 0), q = (A - mu M) p;
// partials p.q, vn.q, p.M vn
template <typename T, int NTC, bool kR>
__global__ __launch_bounds__(NTC) void k_pupdate_apply(MGeo g, const T* __restrict__ z,
                                                       const T* __restrict__ vn,
                                                       const T* __restrict__ pin,
                                                       const T* __restrict__ w,
                                                       T* __restrict__ t, FineState S,
                                                       int first, T* __restrict__ pout,
                                                       T* __restrict__ q,
                                                       double* __restrict__ part) {
  // M vn is recomputed from a ring of vn rows (vn is read anyway) instead of
  // being read; in FP32 storage it then differs from the stored M vn the
  // other kernels read by rounding only
  __shared__ T ring[4][NTC + 2];
  __shared__ T ringv[4][NTC + 2];
  int64_t b;
  int c0, j0, j1, blk, dir;
  if (!map_march<NTC>(g, b, c0, j0, j1, blk, dir) || !S.active[b]) return;
  const T* zz = z + b * g.P;
  const T* vb = vn + b * g.P;
  const T* pb = pin + b * g.P;
  const T* wx = w + b * wblk<kR>() * g.P;
  const T* wy = wx + g.P;
  T* tb = t + b * g.P;
  const T c2 = (T)S.c2[b], beta = first ? T(0) : (T)S.beta[b], mu = (T)S.mu[b];
  const T alpha = first ? T(0) : (T)S.alpha[b];  // the previous step, not yet applied to t
  // t holds t_{k-1} from step 2 on (step k writes t_k = t_{k-1} + alpha p_{k-1});
  // t_0 = 0 is never stored, so steps 0 and 1 do not read it
  const bool tread = !first && S.its[b] >= 2;
  const T hm = (T)mass_scale(g.n);
  const int n = g.n, tx = threadIdx.x, c = c0 + tx, ci = tx + 1;
  // the two threads at the block's edges also load one halo column
  const bool hl = (tx == 0), hr = (tx == NTC - 1);
  const int ch = hl ? c0 - 1 : c0 + NTC;
  const bool hok = (hl && c0 >= 2) || (hr && c0 + NTC <= n - 1);
  // Inputs are requested one row step before they are used: the sources of
  // the ring row p = z - c2 vn + beta p_prev (z, vn, p_prev at the column and
  // the halo column) one row ahead of the rings, the stencil row's weights
  // and t one row ahead of the stencil; vn and p_prev of a row are kept from
  // its ring fill for its stencil step.
  struct Src {
    T z, v, p, zh, vh, ph;
  };
  struct Row {
    Wts<T, kR> w;
    T tt;
  };
  auto fetch_src = [&](int j, Src& f) {
    const bool rowok = (j >= 1 && j <= n - 1);
    f.z = f.v = f.p = f.zh = f.vh = f.ph = T(0);
    if (rowok && c >= 1) {
      const int k = j * n + c;
      f.z = zz[k];
      f.v = vb[k];
      if (!first) f.p = pb[k];
    }
    if (rowok && hok) {
      const int k = j * n + ch;
      f.zh = zz[k];
      f.vh = vb[k];
      if (!first) f.ph = pb[k];
    }
  };
  auto store = [&](int j, const Src& f) {
    T* row = ring[j & 3];
    row[ci] = f.z - c2 * f.v + beta * f.p;
    if (hl) row[0] = f.zh - c2 * f.vh + beta * f.ph;
    if (hr) row[NTC + 1] = f.zh - c2 * f.vh + beta * f.ph;
    T* rv = ringv[j & 3];
    rv[ci] = f.v;
    if (hl) rv[0] = f.vh;
    if (hr) rv[NTC + 1] = f.vh;
  };
  auto fetch_row = [&](int j, Row& r) {
    if (c >= 1 && j >= j0 && j < j1) {
      const int k = j * n + c;
      r.w = load_wts<T, kR>(wx, wy, k, n, g.P, hm);
      r.tt = tread ? tb[k] : T(0);
    }
  };
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int jf = dir > 0 ? j0 : j1 - 1;
  const int count = j1 - j0;
  Src f, fn;
  fetch_src(jf - dir, f);
  store(jf - dir, f);
  fetch_src(jf, f);
  store(jf, f);
  T sv = f.v, sp = f.p;  // vn and p_prev of the row the next stencil step handles
  fetch_src(jf + dir, fn);
  Row rw;
  fetch_row(jf, rw);
  for (int i = 0; i < count; ++i) {
    const int j = jf + i * dir;
    store(j + dir, fn);
    const T nv = fn.v, np = fn.p;
    const Row rc = rw;
    if (i + 1 < count) {
      fetch_src(j + 2 * dir, fn);
      fetch_row(j + dir, rw);
    }
    __syncthreads();
    if (c >= 1) {
      const T* xs = ring[(j - 1) & 3];
      const T* xc = ring[j & 3];
      const T* xn = ring[(j + 1) & 3];
      const T pc = xc[ci];
      const T ap = ring_Aw<T, T, kR>(xs, xc, xn, ci, rc.w);
      const T m12 = T(6) * pc + xc[ci - 1] + xc[ci + 1] + xs[ci] + xn[ci] + xn[ci + 1] +
                    xs[ci - 1];
      const T qv = ap - mu * hm * m12;
      const int64_t o = b * g.P + j * n + c;
      __builtin_nontemporal_store(pc, &pout[o]);
      if (q) q[o] = qv;
      // t_k = t_{k-1} + alpha_{k-1} p_{k-1}, the iterate this step starts from
      T tn = rc.tt;
      if (!first) {
        tn += alpha * sp;
        __builtin_nontemporal_store(tn, &t[o]);
      }
      const double tk = (double)tn;
      s[0] += (double)pc * (double)qv;
      s[1] += (double)sv * (double)qv;
      {
        const T* vs = ringv[(j - 1) & 3];
        const T* vc = ringv[j & 3];
        const T* vnr = ringv[(j + 1) & 3];
        const T mv = hm * (T(6) * vc[ci] + vc[ci - 1] + vc[ci + 1] + vs[ci] + vnr[ci] +
                           vnr[ci + 1] + vs[ci - 1]);
        s[2] += (double)pc * (double)mv;
      }
      s[3] += (double)pc * (double)m12;
      s[4] += tk * (double)m12;
      s[5] += tk * (double)qv;
    }
    sv = nv;
    sp = np;
  }
  write_partials_m<NTC, 6>(s, part, b, blk, g.nblk);
}

// ---------------------------------------------------------------- V-cycle

// ---------------------------------------------------------------- fused V-cycle levels
//
// One block of NTC threads covers full rows (thread t: columns t + q NTC,
// q < CPT = n / NTC) and runs a row pipeline over a strip with LDS rings of
// full rows (n + 1 entries; columns 0 and n are the zero boundary).

struct VGeo {
  int n, lg, P;
  int strips;   // strips per sample
  int Rs;       // rows (PRE: coarse rows) per strip
  int64_t B;
};

template <int NTC, int CPT>
__device__ __forceinline__ bool map_strip(const VGeo& g, int64_t& b, int& s) {
  const int64_t L = blockIdx.x;
  const int xcd = (int)(L & 7);
  const int64_t q = L >> 3;
  b = ((q / g.strips) << 3) + xcd;
  s = (int)(q % g.strips);
  return b < g.B;
}

// stencil of A at column c of the centre ring row
template <typename T>
__device__ __forceinline__ T rowA(const T* rs, const T* rc, const T* rn, int c, const T* wx,
                                  const T* wy, int k, int n, T& d) {
  const T x = rc[c];
  const T ww = wx[k], we = wx[k + 1], ws = wy[k], wn = wy[k + n];
  d = ww + we + ws + wn;
  return ww * (x - rc[c - 1]) + we * (x - rc[c + 1]) + ws * (x - rs[c]) + wn * (x - rn[c]);
}

// Weight of sweep m (0-based) of an NS-sweep smoothing step: the Chebyshev
// weights of that degree.
template <int NS>
__device__ __forceinline__ constexpr double sweep_omega(int m) {
  if constexpr (NS == 3) return kCheb3[m];
  return m == 0 ? kOmega1 : kOmega2;
}

// Row inputs of a node in the fused V-cycle kernels: in[0] the right-hand
// side, in[1..4] the edge weights (west, east, south, north) and, with the
// reaction, in[5..10] h^2/12 times the edge means of b (west, east, south,
// north, south-west, north-east).
template <bool kR>
constexpr int row_inputs() {
  return kR ? 11 : 5;
}
template <typename T, bool kR>
__device__ __forceinline__ void fetch_row_inputs(T* dst, const T* rb, const T* wx, const T* wy,
                                                 int k, int n, int P, T hm) {
  dst[0] = rb[k];
  dst[1] = wx[k];
  dst[2] = wx[k + 1];
  dst[3] = wy[k];
  dst[4] = wy[k + n];
  if constexpr (kR) {
    const T* rx = wx + 2 * P;
    const T* ry = wx + 3 * P;
    const T* rd = wx + 4 * P;
    dst[5] = hm * rx[k];
    dst[6] = hm * rx[k + 1];
    dst[7] = hm * ry[k];
    dst[8] = hm * ry[k + n];
    dst[9] = hm * rd[k];
    dst[10] = hm * rd[k + n + 1];
  }
}
// The same for the row after the one whose inputs are prev (which may be
// dst itself), in the marching direction dir: the vertical edge the two rows
// share (WY, and RY with the reaction) comes from prev instead of a second
// read, which would come one row step later, after the rows of every
// workgroup in flight on the XCD have passed through its L2.
template <typename T, bool kR>
__device__ __forceinline__ void fetch_row_inputs_next(T* dst, const T* prev, int dir,
                                                      const T* rb, const T* wx, const T* wy,
                                                      int k, int n, int P, T hm) {
  const T shared = dir > 0 ? prev[4] : prev[3];
  T rshared = T(0);
  if constexpr (kR) rshared = dir > 0 ? prev[8] : prev[7];
  dst[0] = rb[k];
  dst[1] = wx[k];
  dst[2] = wx[k + 1];
  if (dir > 0) {
    dst[3] = shared;
    dst[4] = wy[k + n];
  } else {
    dst[3] = wy[k];
    dst[4] = shared;
  }
  if constexpr (kR) {
    const T* rx = wx + 2 * P;
    const T* ry = wx + 3 * P;
    const T* rd = wx + 4 * P;
    dst[5] = hm * rx[k];
    dst[6] = hm * rx[k + 1];
    if (dir > 0) {
      dst[7] = rshared;
      dst[8] = hm * ry[k + n];
    } else {
      dst[7] = hm * ry[k];
      dst[8] = rshared;
    }
    dst[9] = hm * rd[k];
    dst[10] = hm * rd[k + n + 1];
  }
}
// the diagonal of A [+ R] at a node from its row inputs
template <typename T, bool kR>
__device__ __forceinline__ T row_diag(const T* in) {
  T d = in[1] + in[2] + in[3] + in[4];
  if constexpr (kR) d += in[5] + in[6] + in[7] + in[8] + in[9] + in[10];
  return d;
}
// ((A [+ R]) x) at column c of the centre row zc (rows zs, zn south and north)
template <typename T, bool kR>
__device__ __forceinline__ T row_op(const T* in, const T* zs, const T* zc, const T* zn, int c) {
  const T x = zc[c];
  T ax = in[1] * (x - zc[c - 1]) + in[2] * (x - zc[c + 1]) + in[3] * (x - zs[c]) +
         in[4] * (x - zn[c]);
  if constexpr (kR)
    ax += in[5] * (x + zc[c - 1]) + in[6] * (x + zc[c + 1]) + in[7] * (x + zs[c]) +
          in[8] * (x + zn[c]) + in[9] * (x + zs[c - 1]) + in[10] * (x + zn[c + 1]);
  return ax;
}

// Pre-smoothing and restriction of one level, NS Jacobi sweeps from zero:
//   X_1 = omega_1 rhs / D;  X_m = X_{m-1} + omega_m (rhs - A X_{m-1}) / D;
//   X = X_NS;  rhs_c = P^T (rhs - A X)
// Strip s owns coarse rows [J0, J1) and fine rows [2 J0 - 1, 2 J1 - 1) (the last
// strip also row n-1).  Sweep m is computed on the owned rows widened by
// NS - m rows on each side (the halo its successor reads), marching one row
// behind sweep m - 1.
// With kUpd (the finest level inside the PCG loop) the right-hand side is
// first brought up to date, r' = r - alpha (q - c M vn), and r' written to
// rout on the rows the strip owns (a second buffer: neighbouring strips still
// read r on their halo rows).  q = (A - mu M) p is recomputed here from the
// direction p (a ring of p rows two rows ahead of the first sweep) with the
// same operations as the apply kernel, so q is never stored.
template <typename T, int NTC, int CPT, bool kUpd, int NS, bool kR>
__global__ __launch_bounds__(NTC) void k_pre(VGeo g, const T* __restrict__ w,
                                             const T* __restrict__ rhs, T* __restrict__ X,
                                             T* __restrict__ rhs_c,
                                             const uint8_t* __restrict__ active,
                                             const T* __restrict__ pd, const T* __restrict__ mvn,
                                             FineState S, T* __restrict__ rout) {
  constexpr int NR = NTC * CPT + 1;
  constexpr int PR = kUpd ? 4 : 1, PN = kUpd ? NR : 1;
  __shared__ T s_sw[NS][4][NR], s_res[4][NR], s_p[PR][PN];
  int64_t b;
  int s;
  if (!map_strip<NTC, CPT>(g, b, s) || !active[b]) return;
  const int n = g.n, nc = n / 2, t = threadIdx.x;
  const int J0 = 1 + s * g.Rs, J1 = min(J0 + g.Rs, nc);
  const int lo = 2 * J0 - 1, hi = 2 * J1 - 1;
  const int own_hi = (J1 == nc) ? hi + 1 : hi;  // owned fine rows [lo, own_hi)
  const int dir = (s & 1) ? -1 : 1;             // odd strips march downwards
  const T* rb = rhs + b * g.P;
  const T* wx = w + b * wblk<kR>() * g.P;
  const T* wy = wx + g.P;
  T* xb = X + b * g.P;
  T* cb = rhs_c + b * (int64_t)((nc + 2) * nc);
  constexpr int NI = row_inputs<kR>();
  T alpha = T(0), cc = T(0), mu = T(0);
  const T hm = (T)mass_scale(n);
  if constexpr (kUpd) {
    alpha = (T)S.alpha[b];
    cc = (T)S.c[b];
    mu = (T)S.mu[b];
  }
  if (t == 0)
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int m = 0; m < NS; ++m) s_sw[m][r][n] = T(0);
      s_res[r][n] = T(0);
      if constexpr (kUpd) s_p[r][n] = T(0);
    }
  // register window of the row inputs (rhs, the edge weights) of the rows
  // at the NS sweep stages and the residual stage: each is loaded once, one
  // row ahead of the first sweep (nx; with kUpd also M vn), and carried
  // through the stages (in[0] -> in[NS])
  T nx[CPT][NI + 1], in[NS + 1][CPT][NI];
  // with kUpd: p of the row the ring takes next, loaded one iteration early
  T pn[CPT];
  auto fetch_p = [&](int j) {
    const bool ok = (j >= 1 && j <= n - 1);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = t + q * NTC;
      pn[q] = (ok && c >= 1) ? pd[b * g.P + j * n + c] : T(0);
    }
  };
  auto store_p = [&](int j) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) s_p[j & 3][t + q * NTC] = pn[q];
  };
  auto fetch = [&](int j) {
    if (!(j >= 1 && j <= n - 1)) return;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = t + q * NTC, k = j * n + c;
      if (c >= 1) {
        fetch_row_inputs<T, kR>(nx[q], rb, wx, wy, k, n, g.P, hm);
        if constexpr (kUpd) nx[q][NI] = mvn[b * g.P + k];
      }
    }
  };
  const int jfirst = dir > 0 ? lo - NS : hi + NS;
  const int last = hi - lo + 2 * NS;
  fetch(jfirst);
  if constexpr (kUpd) {  // the p ring holds rows j - 1 .. j + 1 when row j is updated
    for (int d = -1; d <= 1; ++d) {
      fetch_p(jfirst + d * dir);
      store_p(jfirst + d * dir);
    }
    fetch_p(jfirst + 2 * dir);
    __syncthreads();
  }
  for (int i = 0; i <= last; ++i) {
    const int j = jfirst + i * dir;
    // first sweep (from zero) at row j
    {
      T* row = s_sw[0][j & 3];
      const bool ok = (j >= 1 && j <= n - 1);
      T mvj[CPT];
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
#pragma unroll
        for (int m = NS; m > 0; --m)
#pragma unroll
          for (int e = 0; e < NI; ++e) in[m][q][e] = in[m - 1][q][e];
#pragma unroll
        for (int e = 0; e < NI; ++e) in[0][q][e] = nx[q][e];
        if constexpr (kUpd) mvj[q] = nx[q][NI];
      }
      if (i < last) fetch(j + dir);
      if constexpr (kUpd) {
        // slot of row j + 2 dir is free (row j - 2 dir is done with); read
        // from the next iteration on, after this one's barriers
        store_p(j + 2 * dir);
        if (i < last) fetch_p(j + 3 * dir);
      }
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int c = t + q * NTC, k = j * n + c;
        T v = T(0);
        if (ok && c >= 1) {
          if constexpr (kUpd) {
            const T* xs = s_p[(j - 1) & 3];
            const T* xc = s_p[j & 3];
            const T* xn = s_p[(j + 1) & 3];
            const T* inq = in[0][q];
            const T pc = xc[c];
            const T ap = row_op<T, kR>(inq, xs, xc, xn, c);
            const T m12 = T(6) * pc + xc[c - 1] + xc[c + 1] + xs[c] + xn[c] + xn[c + 1] +
                          xs[c - 1];
            const T qv = ap - mu * hm * m12;
            in[0][q][0] = inq[0] - alpha * (qv - cc * mvj[q]);
            if (j >= lo && j < own_hi)
              __builtin_nontemporal_store(in[0][q][0], &rout[b * g.P + k]);
          }
          v = T(sweep_omega<NS>(0)) * in[0][q][0] / row_diag<T, kR>(in[0][q]);
        }
        row[c] = v;
      }
    }
    __syncthreads();
    // sweeps 2..NS, sweep m one row behind sweep m - 1
#pragma unroll
    for (int m = 1; m < NS; ++m) {
      const int jz = j - m * dir;
      const int wide = NS - m;  // halo rows this sweep still feeds
      if (jz >= lo - wide && jz <= hi + wide) {
        T* row = s_sw[m][jz & 3];
        const bool ok = (jz >= 1 && jz <= n - 1);
        const T* zs = s_sw[m - 1][(jz - 1) & 3];
        const T* zc = s_sw[m - 1][jz & 3];
        const T* zn = s_sw[m - 1][(jz + 1) & 3];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          const int c = t + q * NTC, k = jz * n + c;
          T v = T(0);
          if (ok && c >= 1) {
            const T* inm = in[m][q];
            const T x = zc[c];
            const T ax = row_op<T, kR>(inm, zs, zc, zn, c);
            v = x + T(sweep_omega<NS>(m)) * (inm[0] - ax) / row_diag<T, kR>(inm);
            if (m == NS - 1 && jz >= lo && jz < own_hi) __builtin_nontemporal_store(v, &xb[k]);
          }
          row[c] = v;
        }
      }
      __syncthreads();
    }
    // residual NS rows behind the first sweep
    const int jr = j - NS * dir;
    if (jr >= lo && jr <= hi) {
      T* row = s_res[jr & 3];
      const T* xs = s_sw[NS - 1][(jr - 1) & 3];
      const T* xc = s_sw[NS - 1][jr & 3];
      const T* xn = s_sw[NS - 1][(jr + 1) & 3];
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int c = t + q * NTC;
        T v = T(0);
        if (c >= 1) {
          const T* inr = in[NS][q];
          v = inr[0] - row_op<T, kR>(inr, xs, xc, xn, c);
        }
        row[c] = v;
      }
      __syncthreads();
      // restriction at the coarse row J whose residual rows 2J-1..2J+1 are
      // complete (jr = 2J+1 upwards, 2J-1 downwards)
      if ((jr & 1) && (dir > 0 ? jr >= lo + 2 : jr <= hi - 2)) {
        const int J = dir > 0 ? (jr - 1) >> 1 : (jr + 1) >> 1;
        const T* rs = s_res[(2 * J - 1) & 3];
        const T* rc = s_res[(2 * J) & 3];
        const T* rn = s_res[(2 * J + 1) & 3];
        for (int I = t + 1; I <= nc - 1; I += NTC) {
          const int c = 2 * I;
          cb[J * nc + I] = rc[c] + T(0.5) * (rc[c - 1] + rc[c + 1] + rs[c] + rn[c] + rn[c + 1] +
                                             rs[c - 1]);
        }
      }
    }
  }
}

// The stencil kernels write their full-size outputs (Xout, X, the updated
// residual, p, t, and the set-up's r, vn, M vn) with non-temporal stores: they are read again only a kernel
// or more later, long after they would have left the L2, and kept out of it
// they leave room for the rows the neighbouring strips share (measured 2-8 %
// faster k_post, k_pupdate_apply and k_pre launches).
//
// Post-smoothing of one level: U = Xin + P Xc; NS sweeps; Xout.  On level 0
// (kDots) the last sweep also forms the partials r.z, M vn.z, r.vn.  The
// recursive residual keeps vn^T r at vn^T r_0 = 0 up to the rounding of the
// updates r - alpha (q - c M vn) (vn^T M vn = 1, c = vn^T q); in
// FP64 that drift is ~1e-16 |r_0| against |r| >= 1e-10 |r_0| (the tightest
// residual test), so r.vn is taken as 0 there and vn is not read; FP32
// storage drifts by ~1e-7 |r_0| and keeps the explicit product.  Strip s
// owns fine rows [f0, f1); sweep m runs on them widened by NS - m rows on
// each side.  Xout must differ from Xin (neighbour strips read Xin rows
// across the strip boundary).
template <typename T, int NTC, int CPT, bool kDots, int NS, bool kR>
__global__ __launch_bounds__(NTC) void k_post(VGeo g, const T* __restrict__ w,
                                              const T* __restrict__ rhs,
                                              const T* __restrict__ Xin,
                                              const T* __restrict__ Xc, T* __restrict__ Xout,
                                              const T* __restrict__ vn, const T* __restrict__ mvn,
                                              const uint8_t* __restrict__ active,
                                              double* __restrict__ part) {
  constexpr int NR = NTC * CPT + 1;
  constexpr bool kRv = sizeof(T) < 8;  // r.vn formed explicitly (FP32 storage)
  // s_sw[0]: U; s_sw[m]: after sweep m (the last sweep goes straight out)
  __shared__ T s_sw[NS][4][NR];
  int64_t b;
  int s;
  if (!map_strip<NTC, CPT>(g, b, s) || !active[b]) return;
  const int n = g.n, nc = n / 2, t = threadIdx.x;
  const int f0 = 1 + s * g.Rs, f1 = min(f0 + g.Rs, n);
  const int dir = (s & 1) ? -1 : 1;             // odd strips march downwards
  const T* rb = rhs + b * g.P;
  const T* xi = Xin + b * g.P;
  const T* xc = Xc + b * (int64_t)((nc + 2) * nc);
  const T* wx = w + b * wblk<kR>() * g.P;
  const T* wy = wx + g.P;
  const T* vb = vn + b * g.P;
  constexpr int NI = row_inputs<kR>();
  const T hm = (T)mass_scale(n);
  const T* mb = mvn + b * g.P;
  T* xo = Xout + b * g.P;
  double acc[3] = {0.0, 0.0, 0.0};
  if (t == 0)
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int m = 0; m < NS; ++m) s_sw[m][r][n] = T(0);
  // Every global input is requested one pipeline step before it is used:
  // u-row sources (X_in and the two coarse values of the prolongation) one
  // row ahead, the row inputs of the sweeps (rhs, 4 edge weights) as in[0]
  // one row ahead of the first sweep, then kept through the later sweeps
  // (in[1] -> in[NS]).
  T ux[CPT][3], in[NS + 1][CPT][NI];
  auto fetch_u = [&](int j) {
    const bool ok = (j >= 1 && j <= n - 1);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = t + q * NTC;
      if (ok && c >= 1) {
        ux[q][0] = xi[j * n + c];
        ux[q][1] = xc[(j >> 1) * nc + (c >> 1)];
        ux[q][2] = xc[((j + 1) >> 1) * nc + ((c + 1) >> 1)];
      } else {
        ux[q][0] = ux[q][1] = ux[q][2] = T(0);
      }
    }
  };
  // With one column per thread and no reaction the vertical edge a row
  // shares with the previous one is carried over (in[1] after the shift
  // holds that row's inputs): measured 7 % faster on 1/128, while with 2 or 4
  // columns per thread (1/512, 1/1024) the carry made the kernel 10 % slower,
  // and with the reaction arrays 8 % (FP64) to 27 % (FP32) slower.
  bool have = false;
  auto fetch_in = [&](int j) {
    if (!(j >= max(f0 - NS + 1, 1) && j <= min(f1 + NS - 2, n - 1))) {
      have = false;
      return;
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = t + q * NTC, k = j * n + c;
      if (c >= 1) {
        if (CPT == 1 && !kR && have)
          fetch_row_inputs_next<T, kR>(in[0][q], in[1][q], dir, rb, wx, wy, k, n, g.P, hm);
        else
          fetch_row_inputs<T, kR>(in[0][q], rb, wx, wy, k, n, g.P, hm);
      }
    }
    have = true;
  };
  const int jfirst = dir > 0 ? f0 - NS : f1 + NS - 1;
  const int last = f1 - f0 + 2 * NS - 1;
  fetch_u(jfirst);
  for (int i = 0; i <= last; ++i) {
    const int j = jfirst + i * dir;
    T uc[CPT][3];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
#pragma unroll
      for (int e = 0; e < 3; ++e) uc[q][e] = ux[q][e];
#pragma unroll
      for (int m = NS; m > 0; --m)
#pragma unroll
        for (int e = 0; e < NI; ++e) in[m][q][e] = in[m - 1][q][e];
    }
    if (i < last) {
      fetch_u(j + dir);
      fetch_in(j);
    }
    const int jo = j - NS * dir;
    T dv[CPT][2];
    if constexpr (kDots) {
      if (jo >= f0 && jo < f1) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          const int k = jo * n + t + q * NTC;
          dv[q][0] = mb[k];
          dv[q][1] = kRv ? vb[k] : T(0);
        }
      }
    }
    {
      T* row = s_sw[0][j & 3];
#pragma unroll
      for (int q = 0; q < CPT; ++q)
        row[t + q * NTC] = uc[q][0] + T(0.5) * (uc[q][1] + uc[q][2]);
    }
    __syncthreads();
    // sweeps 1..NS-1 into LDS, sweep m one row behind sweep m - 1
#pragma unroll
    for (int m = 1; m < NS; ++m) {
      const int jm = j - m * dir;
      const int wide = NS - m;
      if (jm >= f0 - wide && jm <= f1 - 1 + wide) {
        T* row = s_sw[m][jm & 3];
        const bool ok = (jm >= 1 && jm <= n - 1);
        const T* us = s_sw[m - 1][(jm - 1) & 3];
        const T* uc0 = s_sw[m - 1][jm & 3];
        const T* un = s_sw[m - 1][(jm + 1) & 3];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          const int c = t + q * NTC;
          T v = T(0);
          if (ok && c >= 1) {
            const T* inm = in[m][q];
            const T x = uc0[c];
            const T ax = row_op<T, kR>(inm, us, uc0, un, c);
            v = x + T(sweep_omega<NS>(m - 1)) * (inm[0] - ax) / row_diag<T, kR>(inm);
          }
          row[c] = v;
        }
      }
      __syncthreads();
    }
    // the last sweep on the owned rows, straight to Xout
    if (jo >= f0 && jo < f1) {
      const T* zs = s_sw[NS - 1][(jo - 1) & 3];
      const T* zc = s_sw[NS - 1][jo & 3];
      const T* zn = s_sw[NS - 1][(jo + 1) & 3];
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int c = t + q * NTC, k = jo * n + c;
        if (c >= 1) {
          const T* inl = in[NS][q];
          const T x = zc[c];
          const T ax = row_op<T, kR>(inl, zs, zc, zn, c);
          const T zz = x + T(sweep_omega<NS>(NS - 1)) * (inl[0] - ax) / row_diag<T, kR>(inl);
          __builtin_nontemporal_store(zz, &xo[k]);
          if constexpr (kDots) {
            acc[0] += (double)inl[0] * (double)zz;
            acc[1] += (double)dv[q][0] * (double)zz;
            if constexpr (kRv) acc[2] += (double)inl[0] * (double)dv[q][1];
          }
        }
      }
    }
  }
  if constexpr (kDots) {
    __shared__ double red[3 * (NTC / 64)];
    block_sums<NTC, 3>(acc, red);
    if (threadIdx.x == 0) {
      const int64_t base = (b * g.strips + s) * 3;
      part[base] = acc[0];
      part[base + 1] = acc[1];
      part[base + 2] = acc[2];
    }
  }
}

// ---------------------------------------------------------------- final

// w = vs v + t (FP64): partials w.A w, w.M12 w in FP64 arithmetic on the
// weights of storage type T, and the sum of w (h^2 times it is the integral
// of the P1 function w)
template <typename T, int NTC, bool kR>
__global__ __launch_bounds__(NTC) void k_final_dots(MGeo g, Coarse cv,
                                                    const T* __restrict__ t,
                                                    const T* __restrict__ p0,
                                                    const T* __restrict__ p1,
                                                    const T* __restrict__ w, FineState S,
                                                    double* __restrict__ part) {
  __shared__ double ring[4][NTC + 2];
  int64_t b;
  int c0, j0, j1, blk, dir;
  if (!map_march<NTC>(g, b, c0, j0, j1, blk, dir)) return;
  const T* tb = t + b * g.P;
  // the sample's last step alpha p is still to be added to t: its direction
  // sits in the buffer that iteration its - 1 wrote
  const int its = S.its[b];
  const T* pl = ((its & 1) ? p1 : p0) + b * g.P;
  const T al = its > 0 ? (T)S.alpha[b] : T(0);
  const bool tread = its >= 2;  // t_{its-1} stored (t_0 = 0 never is)
  const double vs = S.vs[b];
  const T* wx = w + b * wblk<kR>() * g.P;
  const T* wy = wx + g.P;
  const double hm = mass_scale(g.n);
  double s[3] = {0.0, 0.0, 0.0};
  struct Fin {
    CoarseSrc v;
    T t, p;
  };
  march_pf<double, NTC>(
      ring, g, c0, j0, j1, dir,
      [&](int k) { return Fin{coarse_src(cv, g, b, k), tread ? tb[k] : T(0), pl[k]}; },
      [&](const Fin& f) { return vs * coarse_val(cv, f.v) + (double)(T)(f.t + al * f.p); },
      [&](int k) { return load_wts_fp64<T, kR>(wx, wy, k, g.n, g.P, hm); },
      [&](int, int, const double* rs, const double* rc, const double* rn, int ci,
          const Wts<double, kR>& wt, const Fin&) {
        const double aw = ring_Aw(rs, rc, rn, ci, wt);
        s[0] += rc[ci] * aw;
        s[1] += rc[ci] * ring_M12(rs, rc, rn, ci);
        s[2] += rc[ci];
      });
  write_partials_m<NTC, 3>(s, part, b, blk, g.nblk);
}

// one wavefront per sample: sum the sample's block partials in fixed order
__global__ __launch_bounds__(256) void k_scalar(int phase, int n, int64_t B, int nblk,
                                                const double* __restrict__ part, FineState S,
                                                double rtol, int max_it) {
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  int K = 3;
  if (phase == PH_SETUP) K = 2;
  if (phase == PH_ALPHA) K = 6;
  if ((phase == PH_ALPHA || phase == PH_BETA) && !S.active[b]) return;
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
      S.f[b] = S.rho[b] - S.mu[b];  // w_0 = vn, M-normalised
      S.m[b] = 1.0;
      S.dmp[b] = 0.0;
      S.rzp[b] = 0.0;
      S.active[b] = 1;
      S.vact[b] = 1;
      S.its[b] = 0;
      break;
    }
    case PH_FIRST_RZ: {  // s0 = r.z, s1 = Mv.z, s2 = r.v
      const double rz = s[0] - s[2] * s[1];
      S.rz[b] = rz;
      S.rz0[b] = rz;
      S.c2[b] = s[1];
      S.beta[b] = 0.0;
      if (!(rz > 0.0)) S.active[b] = S.vact[b] = 0;  // zero right-hand side: t = 0 is exact
      break;
    }
    case PH_ALPHA: {
      // s0 = p.q, s1 = v.q, s2 = p.Mv, s3 = p.M12 p, s4 = t.M12 p, s5 = t.q
      // (q = (A - mu M) p, t = t_k before this step)
      const double pq = s[0] - s[2] * s[1];
      if (!(pq > 0.0)) {
        S.flags[b] |= MLQMC_FLAG_BREAKDOWN;
        S.active[b] = S.vact[b] = 0;
        S.alpha[b] = 0.0;
        break;
      }
      const double a = S.rz[b] / pq;
      S.alpha[b] = a;
      S.c[b] = s[1];
      // Rayleigh quotient of w_{k+1} = w_k + a p: mu + f/m with
      // f += 2a p^T (A - mu M) w_k + a^2 p^T (A - mu M) p, m += 2a p^T M w_k + a^2 p^T M p
      const double f1 = S.f[b] + 2.0 * a * (s[1] + s[5]) + a * a * s[0];
      const double dm = 2.0 * a * (s[2] + hm * s[4]) + a * a * hm * s[3];
      const double df = f1 - S.f[b];
      const double m1 = S.m[b] + dm;
      S.f[b] = f1;
      S.m[b] = m1;
      // Error left in mu + f/m after this step.  f (the energy) falls by
      // |df| per step with a tail of about |df| c^2 / (1 - c^2); m changes at
      // first order in the error, with a tail of about |dm| c / (1 - c), and
      // enters the quotient scaled by |f/m| = |lambda - mu|.  c is the
      // observed contraction of the preconditioned residual; |dm| is guarded
      // by the previous step's change, since single increments can vanish.
      const double rzp = S.rzp[b];
      double c = rzp > 0.0 ? sqrt(S.rz[b] / rzp) : 0.5;
      c = fmin(fmax(c, 0.05), 0.9);
      const double dmg = fmax(fabs(dm), c * fabs(S.dmp[b]));
      S.dmp[b] = dm;
      const double est =
          (fabs(df) * c * c / (1.0 - c * c) + fabs(f1 / m1) * dmg * c / (1.0 - c)) / m1;
      const double lam = S.mu[b] + f1 / m1;
      if (est <= rtol * fabs(lam)) S.vact[b] = 0;  // converged: this is the last step
      break;
    }
    case PH_BETA: {  // s0 = r.z, s1 = Mv.z, s2 = r.v
      const int it = S.its[b] + 1;
      S.its[b] = it;
      if (!S.vact[b]) {  // the eigenvalue test stopped the sample at its last step
        S.active[b] = 0;
        break;
      }
      const double rzn = s[0] - s[2] * s[1];
      if (sqrt(fabs(rzn / S.rz0[b])) <= rtol) {
        S.active[b] = S.vact[b] = 0;
        break;
      }
      if (it >= max_it) {
        S.flags[b] |= MLQMC_FLAG_LIN_NOCONV;
        S.active[b] = S.vact[b] = 0;
        break;
      }
      S.beta[b] = rzn / S.rz[b];
      S.rzp[b] = S.rz[b];
      S.rz[b] = rzn;
      S.c2[b] = s[1];
      break;
    }
    case PH_FINAL: {  // s0 = w.Aw, s1 = w.M12w, s2 = sum of w
      const double lam = s[0] / (s[1] * hm);
      S.lam[b] = lam;
      if (S.g) S.g[b] = fabs(s[2]) / ((double)n * n * sqrt(s[1] * hm));
      if (S.lin_acc) S.lin_acc[b] += S.its[b];
      if (!isfinite(lam)) S.flags[b] |= MLQMC_FLAG_NONFINITE;
      break;
    }
    case PH_FINAL_TRACKED: {  // mu + f/m of the last step's w (FP64 storage only)
      const double lam = S.mu[b] + S.f[b] / S.m[b];
      S.lam[b] = lam;
      if (S.lin_acc) S.lin_acc[b] += S.its[b];
      if (!isfinite(lam)) S.flags[b] |= MLQMC_FLAG_NONFINITE;
      break;
    }
  }
}

// interior-layout operator apply for the component entry point
__global__ __launch_bounds__(256) void k_apply_plain(int xblk, int n, int64_t B,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ sigma,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ out) {
  const int m = n - 1, D = m * m, EX = (n - 1) * n;
  const int64_t b = blockIdx.x / xblk;  // grid x = xblk blocks per sample x samples
  const int id = (int)(blockIdx.x - b * xblk) * 256 + threadIdx.x;
  if (id >= D || b >= B) return;
  const int j = id / m + 1, i = id - (j - 1) * m + 1;
  const double* xb = x + b * D;
  const double* wx = w + b * (2 * EX);
  double d;
  const double ax = stencil_A(xb, wx, wx + EX, n, i, j, id, d);
  out[b * D + id] = ax - sigma[b] * mass_scale(n) * stencil_M12(xb, n, i, j, id);
}

}  // namespace

hipError_t launch_zero_boundary(int n, int64_t B, void* const* ptrs, int cnt, int elem,
                                hipStream_t st) {
  if (B <= 0 || cnt <= 0) return hipSuccess;
  if (cnt > 10) return hipErrorInvalidValue;
  ZeroArgs za{};
  for (int a = 0; a < cnt; ++a) za.p[a] = ptrs[a];
  za.cnt = cnt;
  za.elem = elem;
  const int per_blocks = (4 * n - 1 + 255) / 256;
  hipLaunchKernelGGL(k_zero_boundary, dim3((unsigned)(per_blocks * B), cnt), dim3(256), 0, st, n,
                     B, per_blocks, za);
  return hipGetLastError();
}

hipError_t launch_prolong_interior(int nH, int nh, int64_t B, const double* uH, double* uh,
                                  hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const int Dh = (nh - 1) * (nh - 1);
  hipLaunchKernelGGL(k_prolong_interior, dim3((unsigned)((Dh + 255) / 256 * B)), dim3(256), 0, st,
                     (Dh + 255) / 256,
                     nH, nh, B, uH, uh);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarsen(int n, int64_t B, const T* w, T* wc, int reaction, hipStream_t st) {
  const int nc = n / 2;
  const int E = (reaction ? 5 : 2) * (nc + 2) * nc;
  const dim3 grid((unsigned)((E + 255) / 256 * B));
  if (reaction)
    hipLaunchKernelGGL((k_coarsen<T, true>), grid, dim3(256), 0, st, (E + 255) / 256, n, B, w, wc);
  else
    hipLaunchKernelGGL((k_coarsen<T, false>), grid, dim3(256), 0, st, (E + 255) / 256, n, B, w,
                       wc);
  return hipGetLastError();
}

// compile-time reaction flag from the runtime one
#define KR_DISPATCH(r, BODY)      \
  do {                            \
    if (r) {                      \
      constexpr bool kR = true;   \
      BODY;                       \
    } else {                      \
      constexpr bool kR = false;  \
      BODY;                       \
    }                             \
  } while (0)

// marching launches: NTC = 64 (n = 64), 128 (n = 128) or 256 (n >= 256)
#define MARCH_DISPATCH(n, BODY)                \
  do {                                         \
    if ((n) <= 64) {                           \
      constexpr int NTC = 64;                  \
      BODY;                                    \
    } else if ((n) == 128) {                   \
      constexpr int NTC = 128;                 \
      BODY;                                    \
    } else {                                   \
      constexpr int NTC = 256;                 \
      BODY;                                    \
    }                                          \
  } while (0)

template <int NTC>
inline dim3 mgrid(const MGeo& g) {
  const int64_t Bp = (g.B + 7) / 8 * 8;
  return dim3((unsigned)(Bp * g.nblk));
}

namespace {
// uH of mesh nH prolongated to mesh n (n / nH a power of two)
Coarse coarse_of(const double* uH, int nH, int n) {
  int lr = 0;
  while ((nH << lr) < n) ++lr;
  return Coarse{uH, nH, lr, 1.0 / (double)(1 << lr)};
}
}  // namespace

template <typename T>
hipError_t launch_setup_dots(int n, int64_t B, const double* uH, int nH, const T* w,
                             double* part, int reaction, hipStream_t st) {
  if (nH < 2 || n % nH) return hipErrorInvalidValue;
  const Coarse cv = coarse_of(uH, nH, n);
  MARCH_DISPATCH(n, KR_DISPATCH(reaction, {
    const MGeo g = mgeo<NTC>(n, B);
    hipLaunchKernelGGL((k_setup_dots<T, NTC, kR>), mgrid<NTC>(g), dim3(NTC), 0, st, g, cv, w,
                       part);
  }));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_setup_rhs(int n, int64_t B, const double* uH, int nH, const T* w,
                            const FineState& S, T* r, T* vn, T* mvn, int reaction,
                            hipStream_t st) {
  if (nH < 2 || n % nH) return hipErrorInvalidValue;
  const Coarse cv = coarse_of(uH, nH, n);
  MARCH_DISPATCH(n, KR_DISPATCH(reaction, {
    const MGeo g = mgeo<NTC>(n, B);
    hipLaunchKernelGGL((k_setup_rhs<T, NTC, kR>), mgrid<NTC>(g), dim3(NTC), 0, st, g, cv, w, S,
                       r, vn, mvn);
  }));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pupdate_apply(int n, int64_t B, const T* z, const T* vn, const T* pin,
                                const T* w, T* t, const FineState& S, int first, T* pout, T* q,
                                double* part, int reaction, hipStream_t st) {
  MARCH_DISPATCH(n, KR_DISPATCH(reaction, {
    const MGeo g = mgeo<NTC>(n, B);
    hipLaunchKernelGGL((k_pupdate_apply<T, NTC, kR>), mgrid<NTC>(g), dim3(NTC), 0, st, g, z, vn,
                       pin, w, t, S, first, pout, q, part);
  }));
  return hipGetLastError();
}

// fused V-cycle launches, (threads, columns per thread) per mesh.  Pre-
// smoothing: one thread per column, (n, 1): its LDS rings of full rows
// (three stages plus the direction's ring with the update) allow one
// workgroup per compute unit on 1/1024, and 16 waves keep more loads in
// flight than 4 (1/1024: 2.99 against 4.18 ms per launch).  Post-smoothing
// holds fewer rings (two workgroups per unit) and keeps four columns per
// thread there (4.19 against 4.39 ms with one).
#define ROW_DISPATCH_PRE(n, BODY)                           \
  do {                                                      \
    if ((n) <= 64) {                                        \
      constexpr int NTC = 64, CPT = 1;                      \
      BODY;                                                 \
    } else if ((n) == 128) {                                \
      constexpr int NTC = 128, CPT = 1;                     \
      BODY;                                                 \
    } else if ((n) == 256) {                                \
      constexpr int NTC = 256, CPT = 1;                     \
      BODY;                                                 \
    } else if ((n) == 512) {                                \
      constexpr int NTC = 512, CPT = 1;                     \
      BODY;                                                 \
    } else {                                                \
      constexpr int NTC = 1024, CPT = 1;                    \
      BODY;                                                 \
    }                                                       \
  } while (0)
#define ROW_DISPATCH_POST(n, BODY)                          \
  do {                                                      \
    if ((n) <= 64) {                                        \
      constexpr int NTC = 64, CPT = 1;                      \
      BODY;                                                 \
    } else if ((n) == 128) {                                \
      constexpr int NTC = 128, CPT = 1;                     \
      BODY;                                                 \
    } else if ((n) == 256) {                                \
      constexpr int NTC = 256, CPT = 1;                     \
      BODY;                                                 \
    } else if ((n) == 512) {                                \
      constexpr int NTC = 256, CPT = 2;                     \
      BODY;                                                 \
    } else {                                                \
      constexpr int NTC = 256, CPT = 4;                     \
      BODY;                                                 \
    }                                                       \
  } while (0)


inline VGeo vgeo_pre(int n, int64_t B) {
  VGeo g;
  g.n = n;
  g.lg = 0;
  while ((1 << g.lg) < n) ++g.lg;
  g.P = (n + 2) * n;
  const int rows = n / 2 - 1;  // coarse rows
  const int st = strips_for(rows, B);
  g.Rs = (rows + st - 1) / st;
  g.strips = (rows + g.Rs - 1) / g.Rs;
  g.B = B;
  return g;
}
inline VGeo vgeo_post(int n, int64_t B) {
  VGeo g = vgeo_pre(n, B);
  const int rows = n - 1;
  const int st = strips_for(rows, B);
  g.Rs = (rows + st - 1) / st;
  g.strips = (rows + g.Rs - 1) / g.Rs;
  return g;
}
inline dim3 sgrid(const VGeo& g) {
  const int64_t Bp = (g.B + 7) / 8 * 8;
  return dim3((unsigned)(Bp * g.strips));
}

template <typename T>
hipError_t launch_pre(int n, int64_t B, const T* w, const T* rhs, T* X, T* rhs_c,
                      const uint8_t* active, const T* p, const T* mvn, const FineState* S,
                      T* rout, int reaction, hipStream_t st) {
  const VGeo g = vgeo_pre(n, B);
  const bool upd = p != nullptr;
  if (upd && (!mvn || !S || !rout || rout == rhs)) return hipErrorInvalidValue;
  const FineState s0 = S ? *S : FineState{};
  ROW_DISPATCH_PRE(n, KR_DISPATCH(reaction, {
    if (NTC * CPT != n) return hipErrorInvalidValue;  // a block covers one full row
    if (upd)
      hipLaunchKernelGGL((k_pre<T, NTC, CPT, true, kFineSweeps, kR>), sgrid(g), dim3(NTC), 0, st,
                         g, w, rhs, X, rhs_c, active, p, mvn, s0, rout);
    else
      hipLaunchKernelGGL((k_pre<T, NTC, CPT, false, kFineSweeps, kR>), sgrid(g), dim3(NTC), 0, st,
                         g, w, rhs, X, rhs_c, active, p, mvn, s0, rout);
  }));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_post(int n, int64_t B, const T* w, const T* rhs, const T* Xin, const T* Xc,
                       T* Xout, const T* vn, const T* mvn, const uint8_t* active, double* part,
                       int reaction, hipStream_t st) {
  const VGeo g = vgeo_post(n, B);
  ROW_DISPATCH_POST(n, KR_DISPATCH(reaction, {
    if (NTC * CPT != n) return hipErrorInvalidValue;  // a block covers one full row
    if (part)
      hipLaunchKernelGGL((k_post<T, NTC, CPT, true, kFineSweeps, kR>), sgrid(g), dim3(NTC), 0, st,
                         g, w, rhs, Xin, Xc, Xout, vn, mvn, active, part);
    else
      hipLaunchKernelGGL((k_post<T, NTC, CPT, false, kFineSweeps, kR>), sgrid(g), dim3(NTC), 0,
                         st, g, w, rhs, Xin, Xc, Xout, vn, mvn, active, part);
  }));
  return hipGetLastError();
}

int post_strips(int n, int64_t B) { return vgeo_post(n, B).strips; }

void set_target_blocks(int64_t v) { t_target_blocks = v > 0 ? v : kDefaultTargetBlocks; }

int march_blocks(int n, int64_t B) {
  int nb = 0;
  MARCH_DISPATCH(n, { nb = mgeo<NTC>(n, B).nblk; });
  return nb;
}

template <typename T>
hipError_t launch_final_dots(int n, int64_t B, const double* uH, int nH, const T* t, const T* p0,
                             const T* p1, const T* w, const FineState& S, double* part,
                             int reaction, hipStream_t st) {
  if (nH < 2 || n % nH) return hipErrorInvalidValue;
  const Coarse cv = coarse_of(uH, nH, n);
  MARCH_DISPATCH(n, KR_DISPATCH(reaction, {
    const MGeo g = mgeo<NTC>(n, B);
    hipLaunchKernelGGL((k_final_dots<T, NTC, kR>), mgrid<NTC>(g), dim3(NTC), 0, st, g, cv, t, p0,
                       p1, w, S, part);
  }));
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
  if (B <= 0) return hipSuccess;
  const int D = (n - 1) * (n - 1);
  hipLaunchKernelGGL(k_apply_plain, dim3((unsigned)((D + 255) / 256 * B)), dim3(256), 0, st,
                     (D + 255) / 256, n, B, w,
                     sigma, x, out);
  return hipGetLastError();
}

#define INST(T)                                                                                 \
  template hipError_t launch_coarsen<T>(int, int64_t, const T*, T*, int, hipStream_t);           \
  template hipError_t launch_setup_dots<T>(int, int64_t, const double*, int, const T*, double*, \
                                           int, hipStream_t);                                   \
  template hipError_t launch_setup_rhs<T>(int, int64_t, const double*, int, const T*,           \
                                          const FineState&, T*, T*, T*, int, hipStream_t);      \
  template hipError_t launch_pupdate_apply<T>(int, int64_t, const T*, const T*, const T*,       \
                                              const T*, T*, const FineState&, int, T*, T*,      \
                                              double*, int, hipStream_t);                       \
  template hipError_t launch_final_dots<T>(int, int64_t, const double*, int, const T*,          \
                                           const T*, const T*, const T*, const FineState&,      \
                                           double*, int, hipStream_t);
INST(double)
INST(float)
#undef INST
#define INST(T)                                                                                 \
  template hipError_t launch_pre<T>(int, int64_t, const T*, const T*, T*, T*, const uint8_t*,   \
                                    const T*, const T*, const FineState*, T*, int, hipStream_t); \
  template hipError_t launch_post<T>(int, int64_t, const T*, const T*, const T*, const T*, T*,  \
                                     const T*, const T*, const uint8_t*, double*, int,          \
                                     hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace mlqmc
