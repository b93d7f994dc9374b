// Lattice points (eq. rqmc / eq. t_kl), coefficient tables and expansion
// (eq. coeff_s at element centroids), and the estimator reductions
// (Algorithm 2, eq. sample_var, eq. ml-var).
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace mlqmc {
namespace {

// y = frac(((k z) mod N) / N + shift) - 1/2.  N is a power of two, so the
// product reduction and the scaling by 1/N are exact; the shift is one
// rounded add and the final -1/2 one rounded subtract.
__device__ __forceinline__ double lattice_coord(int64_t k, int64_t z, int64_t N, double invN,
                                                double shift) {
  const int64_t mk = (k * z) & (N - 1);
  const double t = (double)mk * invN;
  double u = t + shift;
  if (u >= 1.0) u -= 1.0;
  return u - 0.5;
}

// Points k0 + i, i < count, of R shifted rules: Y[(r count + i) ldY + j] for
// j < s, shift r at shifts[r sld + j].  rad_bits = 0: natural order k;
// rad_bits = m > 0 (N = 2^m): the embedded base-2 order, index = the m-bit
// reversal of k, so every prefix of 2^m' points is the 2^m'-point lattice.
__global__ __launch_bounds__(256) void k_lattice(int64_t N, double invN, int s, int R,
                                                 const int64_t* __restrict__ z,
                                                 const double* __restrict__ shifts, int64_t sld,
                                                 int64_t k0, int64_t count, double* __restrict__ Y,
                                                 int64_t ldY, int rad_bits) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)R * count * s;
  if (idx >= total) return;
  const int j = (int)(idx % s);
  const int64_t row = idx / s;  // r * count + i
  const int r = (int)(row / count);
  const int64_t i = row - (int64_t)r * count;
  int64_t k = k0 + i;
  if (rad_bits > 0) k = (int64_t)(__brevll((unsigned long long)k) >> (64 - rad_bits));
  Y[row * ldY + j] = lattice_coord(k, z[j], N, invN, shifts[(int64_t)r * sld + j]);
}

__global__ __launch_bounds__(256) void k_phi_elements(int n, int s, const double* __restrict__ c,
                                                      const int* __restrict__ k1,
                                                      const int* __restrict__ k2,
                                                      double* __restrict__ phi) {
  const int E = 2 * n * n;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (e >= E || j >= s) return;
  const int sq = e >> 1, tri = e & 1;
  const int i = sq % n, jj = sq / n;
  // centroid: lower ((i+2/3)h, (j+1/3)h), upper ((i+1/3)h, (j+2/3)h)
  const double xc = (double)(3 * i + (tri ? 1 : 2)) / (3.0 * n);
  const double yc = (double)(3 * jj + (tri ? 2 : 1)) / (3.0 * n);
  phi[(int64_t)j * E + e] = c[j] * sinpi((double)k1[j] * xc) * sinpi((double)k2[j] * yc);
}

// Problem 2 element table, rows 0 .. s: row 0 the background value (base_in on
// the islands, base_out elsewhere), row j >= 1 term j: c_{j-1} sin(pi k1 x)
// sin(pi k2 y) on its region (region 1: the islands [1/8, 3/8] or [5/8, 7/8] in
// each coordinate; 2: the rest), 0 elsewhere.  Meshes are multiples of 1/8, so
// no centroid lies on an island boundary.
__device__ __forceinline__ bool in_islands(double x, double y) {
  auto band = [](double t) { return (t >= 0.125 && t <= 0.375) || (t >= 0.625 && t <= 0.875); };
  return band(x) && band(y);
}
__global__ __launch_bounds__(256) void k_phi_elements_islands(
    int n, int s, const double* __restrict__ c, const int* __restrict__ k1,
    const int* __restrict__ k2, const int* __restrict__ region, double base_in, double base_out,
    double* __restrict__ phi) {
  const int E = 2 * n * n;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int row = blockIdx.y;
  if (e >= E || row > s) return;
  const int sq = e >> 1, tri = e & 1;
  const int i = sq % n, jj = sq / n;
  const double xc = (double)(3 * i + (tri ? 1 : 2)) / (3.0 * n);
  const double yc = (double)(3 * jj + (tri ? 2 : 1)) / (3.0 * n);
  const bool inside = in_islands(xc, yc);
  double v;
  if (row == 0) {
    v = inside ? base_in : base_out;
  } else {
    const int j = row - 1;
    const bool own = (region[j] == 1) == inside;
    v = own ? c[j] * sinpi((double)k1[j] * xc) * sinpi((double)k2[j] * yc) : 0.0;
  }
  phi[(int64_t)row * E + e] = v;
}

// edge table: horizontal edge (i,j)-(i+1,j) touches lower(i,j) and upper(i,j-1);
// vertical edge (i,j)-(i,j+1) touches upper(i,j) and lower(i-1,j)
__global__ __launch_bounds__(256) void k_phi_edges(int n, int s, const double* __restrict__ pe,
                                                   double* __restrict__ pw) {
  const int E = 2 * n * n, m = n - 1, EX = (n - 1) * n, EW = 2 * EX;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (e >= EW || j >= s) return;
  const double* el = pe + (int64_t)j * E;
  double v;
  if (e < EX) {
    const int jr = e / n + 1, i = e % n;
    v = 0.5 * (el[2 * (jr * n + i)] + el[2 * ((jr - 1) * n + i) + 1]);
  } else {
    const int f = e - EX;
    const int jr = f / m, i = f % m + 1;
    v = 0.5 * (el[2 * (jr * n + i) + 1] + el[2 * (jr * n + i - 1)]);
  }
  pw[(int64_t)j * EW + e] = v;
}

// padded [WX | WY] edge table: WX(j, i) = edge (i-1,j)-(i,j) (lower element of
// square (i-1, j), upper of square (i-1, j-1)) at j*n + i, i in [1, n] (i = n at
// (j+1)*n), j in [1, n-1]; WY(j, i) = edge (i,j-1)-(i,j) (upper of square
// (i, j-1), lower of square (i-1, j-1)) at P + j*n + i, j in [1, n], i in [1, n-1];
// P = (n+2) n.  Other positions are 0.
__global__ __launch_bounds__(256) void k_phi_edges_padded(int n, int s,
                                                          const double* __restrict__ pe,
                                                          double* __restrict__ pw,
                                                          int64_t row_stride) {
  const int E = 2 * n * n, P = (n + 2) * n;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int jt = blockIdx.y;
  if (e >= 2 * P || jt >= s) return;
  const double* el = pe + (int64_t)jt * E;
  double v = 0.0;
  if (e < P) {
    int j = e / n, i = e % n;
    if (i == 0) {
      i = n;
      j -= 1;
    }
    if (j >= 1 && j <= n - 1) v = 0.5 * (el[2 * (j * n + i - 1)] + el[2 * ((j - 1) * n + i - 1) + 1]);
  } else {
    const int f = e - P;
    const int j = f / n, i = f % n;
    if (j >= 1 && j <= n && i >= 1)
      v = 0.5 * (el[2 * ((j - 1) * n + i) + 1] + el[2 * ((j - 1) * n + i - 1)]);
  }
  pw[(int64_t)jt * row_stride + e] = v;
}

// padded diagonal-edge table (the third segment of the reaction table): the
// edge (i,j)-(i+1,j+1) inside square (i, j) touches its two elements; it is
// stored at (j+1)*n + i + 1 (the index of its north-east end, so i = n-1 lands
// in column 0 of row j+2), for 0 <= i, j <= n-1.  Other positions are 0.
__global__ __launch_bounds__(256) void k_phi_diag_padded(int n, int s,
                                                         const double* __restrict__ pe,
                                                         double* __restrict__ pd,
                                                         int64_t row_stride) {
  const int E = 2 * n * n, P = (n + 2) * n;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int jt = blockIdx.y;
  if (e >= P || jt >= s) return;
  const double* el = pe + (int64_t)jt * E;
  // invert e = (j+1) n + i + 1: column 0 of row r is square (n-1, r-2)
  int r = e / n, c = e % n;
  int i, j;
  if (c == 0) {
    i = n - 1;
    j = r - 2;
  } else {
    i = c - 1;
    j = r - 1;
  }
  double v = 0.0;
  if (i >= 0 && i <= n - 1 && j >= 0 && j <= n - 1)
    v = 0.5 * (el[2 * (j * n + i)] + el[2 * (j * n + i) + 1]);
  pd[(int64_t)jt * row_stride + e] = v;
}

// out[b][e] = a0 + sum_j Y[b][j] phi[j][e] (eq. coeff at the quadrature points
// of every sample, as one [B x s] x [s x E] product) on FP64 MFMA
// (v_mfma_f64_16x16x4f64).  A block computes a 128-sample x 128-entry tile
// with 4 waves in 2 x 2, each wave 4 x 4 MFMA tiles of 16 x 16; K runs in
// chunks of 16 through double-buffered LDS, the next chunk's global loads in
// flight while the current one is multiplied.  Tiles are ordered so that the
// blocks sharing one entry tile of phi run together on one XCD (one L2).
// out and out32, each when given, receive the values in FP64 and rounded to FP32.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kXM = 128, kXN = 128, kXK = 16, kXPad = 4;

__global__ __launch_bounds__(256, 2) void k_expand_mfma(int64_t B, int s, int64_t E,
                                                     const double* __restrict__ Y, int64_t ldY,
                                                     const double* __restrict__ phi, double a0,
                                                     double* __restrict__ out,
                                                     float* __restrict__ out32, int nbm,
                                                     int64_t per_xcd, int64_t ntiles,
                                                     int64_t ldo) {
  __shared__ double sY[2][kXK][kXM + kXPad];
  __shared__ double sP[2][kXK][kXN + kXPad];
  const int64_t L = blockIdx.x;
  const int64_t T = (L & 7) * per_xcd + (L >> 3);
  if (T >= ntiles) return;
  const int tm = (int)(T % nbm);
  const int64_t tn = T / nbm;
  const int64_t m0 = (int64_t)tm * kXM, n0 = tn * kXN;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w & 1, wn = w >> 1;
  // global -> register staging: Y rows t/2, 8 terms from (t&1)*8; phi row t/16,
  // 8 entries from (t&15)*8
  const int yr = t >> 1, yj = (t & 1) * 8;
  const int pr = t >> 4, pc = (t & 15) * 8;
  const int64_t yb = m0 + yr;
  const int64_t pe = n0 + pc;  // E is even and pe is even: pairs are in or out together
  double ry[8], rp[8];
  auto load = [&](int j0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int j = j0 + yj + q;
      ry[q] = (yb < B && j < s) ? Y[yb * ldY + j] : 0.0;
    }
    const int j = j0 + pr;
    const double* src = phi + (int64_t)j * E + pe;
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      if (j < s && pe + q < E) {
        const double2 v = *reinterpret_cast<const double2*>(src + q);
        rp[q] = v.x;
        rp[q + 1] = v.y;
      } else {
        rp[q] = rp[q + 1] = 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) sY[buf][yj + q][yr] = ry[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) sP[buf][pr][pc + q] = rp[q];
  };
  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nch = (s + kXK - 1) / kXK;
  load(0);
  store(0);
  __syncthreads();
  const int fr = lane & 15, fk = lane >> 4;
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load((c + 1) * kXK);
#pragma unroll
    for (int kk = 0; kk < kXK; kk += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sY[buf][kk + fk][wm * 64 + i * 16 + fr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sP[buf][kk + fk][wn * 64 + j * 16 + fr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (c + 1 < nch) store(buf ^ 1);
    __syncthreads();
  }
  // D[row][col] of a 16 x 16 tile: lane holds col = lane & 15 and, in its
  // r-th value, row 4 r + (lane >> 4) (A[row][k] sits in lane row + 16 k,
  // B[k][col] in lane col + 16 k)
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t e = n0 + wn * 64 + j * 16 + fr;
      if (e >= E) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t b = m0 + wm * 64 + i * 16 + 4 * r + fk;
        if (b < B) {
          const double v = a0 + acc[i][j][r];
          if (out) out[b * ldo + e] = v;
          if (out32) out32[b * ldo + e] = (float)v;
        }
      }
    }
}

// ---------------------------------------------------------------- separable expansion
//
// For a family whose terms are products sin(pi k1 x1) sin(pi k2 x2) the sum
// over j collects into C(y)[p][q] = sum of y_j c_j over the terms with
// (k1, k2) = (p + 1, q + 1), and at a point with coordinates (x1, x2)
//   sum_j y_j a_j = sum_p sin(pi (p+1) x1) U_p(x2),  U_p(x2) = sum_q C[p][q] sin(pi (q+1) x2).
// Every element centroid lies on the grid of thirds of the mesh, x = m h / 3,
// so with S[p][m] = sin(pi (p+1) m / (3 n)) and U[m][p] the row sums at
// x2 = m h / 3, an edge weight (the mean over its two elements) is
//   WX(i, j) = a0 + (S[.][3i-2] . U[3j-1] + S[.][3i-1] . U[3j+1]) / 2
//     (the upper element of square (i-1, j-1), centroid (i - 2/3, j - 1/3) h,
//      and the lower one of square (i-1, j), (i - 1/3, j + 1/3) h),
//   WY(i, j) = a0 + (S[.][3i-1] . U[3j-2] + S[.][3i+1] . U[3j-1]) / 2
//     (the lower element of square (i-1, j-1), (i - 1/3, j - 2/3) h, and the
//      upper one of square (i, j-1), (i + 1/3, j - 1/3) h):
// 2 kx multiply-adds per weight instead of 2 s (kx = the largest k1).

// S[p][m] = sin(pi (p + 1) m / (3 n)), p < kmax, m < 3 n + 2
__global__ __launch_bounds__(256) void k_sep_sin(int n, int kmax, double* __restrict__ S) {
  const int M = 3 * n + 2;
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)kmax * M) return;
  const int p = (int)(id / M), m = (int)(id - (int64_t)p * M);
  S[id] = sinpi((double)((p + 1) * m) / (3.0 * n));
}

// U[b][m][p] for m in [m0, m0 + 64) of sample b (grid: m tiles x samples):
// C_b from the terms of each (k1, k2) cell in term order, then the row sums,
// with the S values of the tile's rows staged in LDS kSepRowsQC terms q at a
// time.  Rows m = 3 t hold no element centroid and are never used as
// factors: they are stored as zeros (the set-up products multiply them by
// zero interval sums).
constexpr int kSepMaxK = 32, kSepMaxCells = 1024;
constexpr int kSepRowsQC = 32;
__global__ __launch_bounds__(256) void k_sep_rows(int n, int s, int kx, int ky,
                                                  const double* __restrict__ Y, int64_t ldY,
                                                  const double* __restrict__ c,
                                                  const int* __restrict__ cell_start,
                                                  const int* __restrict__ cell_term,
                                                  const double* __restrict__ S,
                                                  double* __restrict__ U) {
  __shared__ double sC[kSepMaxCells];
  __shared__ double sS[kSepRowsQC][64];
  const int64_t b = blockIdx.y;
  const int M = 3 * n + 2;
  const int m0 = blockIdx.x * 64, t = threadIdx.x;
  for (int cell = t; cell < kx * ky; cell += 256) {
    double v = 0.0;
    for (int k = cell_start[cell]; k < cell_start[cell + 1]; ++k) {
      const int j = cell_term[k];
      v += Y[b * ldY + j] * c[j];
    }
    sC[cell] = v;
  }
  // thread t owns the outputs e = t + 256 u (row m0 + e / kx, term e % kx);
  // 64 kx <= 256 kSepMaxK / 4
  constexpr int kPer = kSepMaxK / 4;
  double acc[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) acc[u] = 0.0;
  for (int q0 = 0; q0 < ky; q0 += kSepRowsQC) {
    __syncthreads();
    for (int e = t; e < kSepRowsQC * 64; e += 256) {
      const int qq = e >> 6, r = e & 63, q = q0 + qq, m = m0 + r;
      sS[qq][r] = (q < ky && m < M) ? S[(int64_t)q * M + m] : 0.0;
    }
    __syncthreads();
    const int qn = min(kSepRowsQC, ky - q0);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = t + 256 * u;
      if (e >= 64 * kx) break;
      const int r = e / kx, p = e - r * kx;
      if ((m0 + r) % 3 == 0) continue;
      const double* cp = sC + p * ky + q0;
      double v = acc[u];
      for (int qq = 0; qq < qn; ++qq) v += cp[qq] * sS[qq][r];
      acc[u] = v;
    }
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + 256 * u;
    if (e >= 64 * kx) break;
    const int r = e / kx, p = e - r * kx, m = m0 + r;
    if (m < M) U[(b * M + m) * kx + p] = acc[u];
  }
}

// Padded [WX | WY] of B samples from U on FP64 MFMA (v_mfma_f64_16x16x4f64),
// with no LDS: a wave owns 32 columns of one sample and marches down all
// n + 2 rows in steps of 16 (the row index of the MFMA tiles), forming per node
// two element products of kx terms, each used by two edges:
//   Lo(i, j)  = U_{3j+1} . S_{3i-1}  (lower element of square (i-1, j)),
//   Up'(i, j) = U_{3j-1} . S_{3i+1}  (upper element of square (i, j-1)),
//   WX(i, j) = a0 + (Up'(i-1, j) + Lo(i, j)) / 2,
//   WY(i, j) = a0 + (Lo(i, j-1) + Up'(i, j)) / 2,
// the shifts by one column and one row being lane shuffles of the MFMA
// results (the row above the tile is carried from the previous step; the
// column left of the wave is a short dot product on the vector units).  The
// S fragments of the wave's columns stay in registers for every term (they
// depend on neither the sample nor the row); the two U rows of a step come
// from global memory (L2: the waves of one sample run on one XCD).  Two waves
// per SIMD; no barriers; K is padded to a multiple of 4 only.  NK = ceil(kx / 4).
// Positions that are not edges of interior nodes get a0, as in the table
// product.  Measured alternatives, all slower: the two edge products of each
// weight formed directly (four per node, 1.1 times as long), 64 x 64 tiles
// staged through LDS (1.7 times), 16 columns per wave (three waves per SIMD,
// 1.2 times), and the next step's U rows loaded before this step's stores
// (one wave per SIMD at 32 columns, 1.4 times in mixed precision).
constexpr int kSepMarchMaxNK = kSepMaxK / 4;
template <int NK>
__global__ __launch_bounds__(256) void k_sep_march(int64_t B, int n, int kx, int cw_per,
                                                   int64_t per_xcd,
                                                   const double* __restrict__ U,
                                                   const double* __restrict__ S, double a0,
                                                   double* __restrict__ out,
                                                   float* __restrict__ out32, int64_t ldo) {
  constexpr int C = 2;  // 16-column MFMA tiles per wave
  // XCD-aware: block L runs on XCD L mod 8 and takes logical block
  // (L mod 8) per_xcd + L / 8, so consecutive logical blocks (the column waves
  // of one sample) share an XCD and its L2
  const int64_t L = blockIdx.x;
  const int64_t lb = (L & 7) * per_xcd + (L >> 3);
  const int lane = threadIdx.x & 63;
  const int64_t W = lb * 4 + (threadIdx.x >> 6);
  const int64_t b = W / cw_per;
  if (b >= B) return;
  const int ic = (int)(W - b * cw_per) * 16 * C;
  const int M = 3 * n + 2, P = (n + 2) * n;
  const int fr = lane & 15, fk = lane >> 4;
  const double* Ub = U + b * (int64_t)M * kx;
  // B[k][col] in lane col + 16 k: column i = ic + 16 c + fr, term p = 4 kk + fk.
  // Column 0 holds no WX edge of its own: its Lo takes the S values of column
  // n, and the column left of it is column n - 1, so that its WX is the edge
  // into the right boundary, which the padded layout stores at column 0 of the
  // next row (its WY is a0).
  double sl[C][NK], su[C][NK], sh[NK];
  const int ih = ic == 0 ? n - 1 : ic - 1;  // the halo column of Up'
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    const int p = 4 * kk + fk;
    const bool ok = p < kx;
    const double* Sp = S + (int64_t)p * M;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int i = ic + 16 * c + fr, ia = i == 0 ? n : i;
      sl[c][kk] = ok ? Sp[3 * ia - 1] : 0.0;
      su[c][kk] = ok ? Sp[3 * i + 1] : 0.0;
    }
    sh[kk] = ok ? Sp[3 * ih + 1] : 0.0;
  }
  const int src_col = (lane & 48) | ((fr + 15) & 15);  // column i - 1 of the same 16
  const int src_row = (lane + 48) & 63;                // row 4 r + fk - 1 (fk > 0)
  // A[row][k] in lane row + 16 k: U rows 3 j + 1 (squares j in [0, n)) and
  // 3 j - 1 (squares j - 1) of row j = jt + fr; zero elsewhere
  auto load_u = [&](int jt, double (&ul)[NK], double (&uu)[NK]) {
    const int j = jt + fr;
    const bool okl = j <= n - 1, oku = j >= 1 && j <= n;
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      const int p = 4 * kk + fk;
      const bool ok = p < kx;
      ul[kk] = (ok && okl) ? Ub[(int64_t)(3 * j + 1) * kx + p] : 0.0;
      uu[kk] = (ok && oku) ? Ub[(int64_t)(3 * j - 1) * kx + p] : 0.0;
    }
  };
  double carry[C];  // Lo of the row above the tile, in lanes fk = 0
#pragma unroll
  for (int c = 0; c < C; ++c) carry[c] = 0.0;
  for (int jt = 0; jt < n + 2; jt += 16) {
    double ul[NK], uu[NK];
    load_u(jt, ul, uu);
    v4d lo[C], up[C];
#pragma unroll
    for (int c = 0; c < C; ++c) lo[c] = up[c] = v4d{0.0, 0.0, 0.0, 0.0};
    double hd = 0.0;
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        lo[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ul[kk], sl[c][kk], lo[c], 0, 0, 0);
        up[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(uu[kk], su[c][kk], up[c], 0, 0, 0);
      }
      hd += uu[kk] * sh[kk];
    }
    // Up' of the halo column for row jt + fr: the four term groups summed
    hd += __shfl_xor(hd, 16);
    hd += __shfl_xor(hd, 32);
    // D[row][col]: lane holds col = lane & 15 and, in its r-th value, row 4 r + (lane >> 4)
    double upl[C][4], lou[C][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double h = __shfl(hd, 4 * r + fk);
      double t[C];
#pragma unroll
      for (int c = 0; c < C; ++c) t[c] = __shfl(up[c][r], src_col);
#pragma unroll
      for (int c = 0; c < C; ++c) upl[c][r] = fr == 0 ? (c == 0 ? h : t[c - 1]) : t[c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      double t[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) t[r] = __shfl(lo[c][r], src_row);
#pragma unroll
      for (int r = 0; r < 4; ++r) lou[c][r] = fk > 0 ? t[r] : (r > 0 ? t[r - 1] : carry[c]);
      carry[c] = t[3];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int i = ic + 16 * c + fr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jt + 4 * r + fk;
        if (j > n + 1) continue;
        const double vx = (j >= 1 && j <= n - 1) ? a0 + 0.5 * (upl[c][r] + lo[c][r]) : a0;
        const double vy = (i >= 1 && j >= 1 && j <= n) ? a0 + 0.5 * (lou[c][r] + up[c][r]) : a0;
        const int64_t o = b * ldo + (int64_t)j * n + i;
        // column 0: WX of row j goes to row j + 1 (rows 1 .. n + 1), and row 0 gets a0
        const bool al = i == 0;
        const bool wx = !al || j <= n;
        const int64_t ox = al ? o + n : o;
        if (out) {
          if (wx) out[ox] = vx;
          if (al && j == 0) out[o] = a0;
          out[o + P] = vy;
        }
        if (out32) {
          if (wx) out32[ox] = (float)vx;
          if (al && j == 0) out32[o] = (float)a0;
          out32[o + P] = (float)vy;
        }
      }
    }
  }
}

// ---------------------------------------------------------------- separable set-up products
//
// The set-up of a two-grid update needs v^T M_h v and v^T A_h v for the
// prolongated coarse eigenvector v = P u_H.  On nested meshes both follow from
// coarse quantities.  The P1 mass matrices integrate exactly, so
// v^T M_h v = u_H^T M_H u_H.  The gradient of v is constant on each coarse
// triangle T and the fine elements K tile T, so
//   v^T A_h v = sum_K a_K |K| |grad v|_K^2 = sum_T |grad u_H|_T^2 (h^2 / 2) sum_{K in T} a_K,
// with a_K the coefficient at the centroid of K.  In the separable form
// a_K = a0 + S[.][x_K] . U[y_K] (grid of thirds: the lower element of fine
// square (a, b) has its centroid at x = 3a + 2, y = 3b + 1, the upper one at
// 3a + 1, 3b + 2), so with r = n / nH the sum over T is r^2 a0 plus, over the
// fine rows b = r B + beta of coarse row B, U rows 3b + 1 and 3b + 2 against
// sums of S over the fine squares of that row that lie in T (a = r A + alpha;
// below the coarse diagonal alpha > beta, above alpha < beta, and on it the
// lower element goes to the lower triangle and the upper one to the upper).
// Those interval sums do not depend on the sample: Tp [K x 2 nH], K = 3 r kx,
// row (3 beta + e) kx + p for U row 3 (r B + beta) + e (e = 0 holds no
// centroid: zero), column A for the lower and nH + A for the upper triangle
// of coarse square (A, B).

// Tp (grid: K x 2 nH entries)
__global__ __launch_bounds__(256) void k_sep_tri(int n, int nH, int kx,
                                                 const double* __restrict__ S,
                                                 double* __restrict__ Tp) {
  const int r = n / nH, K = 3 * r * kx, NC = 2 * nH, M = 3 * n + 2;
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)K * NC) return;
  const int k = (int)(id / NC), col = (int)(id - (int64_t)k * NC);
  const int beta = k / (3 * kx), e = (k / kx) % 3, p = k % kx;
  const int A = col % nH, upper = col / nH;
  int lo = 0, hi = 0, off = 0;  // alpha in [lo, hi), x index 3 (r A + alpha) + off
  if (e == 1) {                 // lower fine elements
    off = 2;
    lo = upper ? 0 : beta;
    hi = upper ? beta : r;
  } else if (e == 2) {          // upper fine elements
    off = 1;
    lo = upper ? 0 : beta + 1;
    hi = upper ? beta + 1 : r;
  }
  double acc = 0.0;
  for (int alpha = lo; alpha < hi; ++alpha) acc += S[(int64_t)p * M + 3 * (r * A + alpha) + off];
  Tp[id] = acc;
}

// part[2 b] = sum over fine nodes of v (M12 v), part[2 b + 1] = v^T A_h v, the
// partial sums the set-up kernel k_setup_dots forms on the fine mesh (one
// block per sample).  One workgroup per sample; wave w takes the 16-row strip
// w of the [nH x 2 nH] product U_b Tp on FP64 MFMA (nH <= 64: four strips at
// most), with Tp staged through LDS in chunks of kSepTriKC rows shared by the
// four waves, and weights each entry with |grad u_H|^2 of its triangle.
constexpr int kSepTriMaxCT = 8;  // column tiles: nH <= 64
constexpr int kSepTriKC = 16, kSepTriLd = 16 * kSepTriMaxCT + 16;
__global__ __launch_bounds__(256) void k_sep_setup_dots(int64_t B, int n, int nH, int kx,
                                                        const double* __restrict__ U,
                                                        const double* __restrict__ Tp,
                                                        const double* __restrict__ uH, double a0,
                                                        double* __restrict__ part) {
  __shared__ double sT[kSepTriKC][kSepTriLd];
  __shared__ double red[2 * 4];
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  const int r = n / nH, K = 3 * r * kx, NC = 2 * nH, M = 3 * n + 2, mH = nH - 1;
  const int CT = (NC + 15) / 16, RS = (nH + 15) / 16;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const double* ub = uH + b * (int64_t)mH * mH;
  auto u = [&](int a, int c) -> double {
    return (a >= 1 && a <= mH && c >= 1 && c <= mH) ? ub[(c - 1) * mH + (a - 1)] : 0.0;
  };
  const double r2a0 = (double)r * r * a0;
  double s[2] = {0.0, 0.0};
  v4d acc[kSepTriMaxCT];
#pragma unroll
  for (int c = 0; c < kSepTriMaxCT; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  const int brow = w * 16 + fr;
  const double* ur = U + ((int64_t)b * M + (int64_t)3 * r * brow) * kx;
  for (int k0 = 0; k0 < K; k0 += kSepTriKC) {
    for (int e = t; e < kSepTriKC * 16 * CT; e += 256) {
      const int kk = e / (16 * CT), col = e - kk * 16 * CT, k = k0 + kk;
      sT[kk][col] = (k < K && col < NC) ? Tp[(int64_t)k * NC + col] : 0.0;
    }
    __syncthreads();
    if (w < RS) {
#pragma unroll
      for (int kk = 0; kk < kSepTriKC; kk += 4) {
        // A[row][k] in lane row + 16 k; B[k][col] in lane col + 16 k
        const int k = k0 + kk + fk;
        const double a = (brow < nH && k < K) ? ur[k] : 0.0;
#pragma unroll
        for (int c = 0; c < kSepTriMaxCT; ++c)
          if (c < CT)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sT[kk + fk][16 * c + fr], acc[c], 0,
                                                          0, 0);
      }
    }
    __syncthreads();
  }
  // D[row][col]: lane holds col = lane & 15 and, in its q-th value, row 4 q + (lane >> 4)
  if (w < RS) {
#pragma unroll
    for (int c = 0; c < kSepTriMaxCT; ++c) {
      if (c >= CT) continue;
      const int col = 16 * c + fr;
      if (col >= NC) continue;
      const int A = col % nH, upper = col / nH;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int Bc = w * 16 + 4 * q + fk;
        if (Bc >= nH) continue;
        double dx, dy;
        if (upper) {  // (A, B), (A + 1, B + 1), (A, B + 1)
          dx = u(A + 1, Bc + 1) - u(A, Bc + 1);
          dy = u(A, Bc + 1) - u(A, Bc);
        } else {      // (A, B), (A + 1, B), (A + 1, B + 1)
          dx = u(A + 1, Bc) - u(A, Bc);
          dy = u(A + 1, Bc + 1) - u(A + 1, Bc);
        }
        s[1] += (dx * dx + dy * dy) * (r2a0 + acc[c][q]);
      }
    }
  }
  // u_H^T M12_H u_H over the coarse interior nodes
  for (int k = t; k < mH * mH; k += 256) {
    const int a = k % mH + 1, c = k / mH + 1;
    const double x = u(a, c);
    s[0] += x * (6.0 * x + u(a - 1, c) + u(a + 1, c) + u(a, c - 1) + u(a, c + 1) +
                 u(a + 1, c + 1) + u(a - 1, c - 1));
  }
  block_sums<256, 2>(s, red);
  if (t == 0) {
    // fine-mesh scaling: M_h / M_H = (h / H)^2, and |K| |grad|^2 = (diff)^2 / (2 r^2)
    part[2 * b] = s[0] * r * r;
    part[2 * b + 1] = s[1] / (2.0 * r * r);
  }
}

__global__ __launch_bounds__(256) void k_level_sums(int64_t N, const double* __restrict__ lam,
                                                    const double* __restrict__ lam_prev,
                                                    double* __restrict__ Q) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  const double* a = lam + (int64_t)r * N;
  const double* p = lam_prev ? lam_prev + (int64_t)r * N : nullptr;
  double s[1] = {0.0};
  for (int64_t k = threadIdx.x; k < N; k += 256) s[0] += a[k] - (p ? p[k] : 0.0);
  block_sums<256, 1>(s, red);
  if (threadIdx.x == 0) Q[r] = s[0] / (double)N;
}

// Running sums of an extensible estimate: for shift r = blockIdx.x,
// sums[r] += sum_{i < count} (lam[r ld + off + i] - lam_prev[r ldp + offp + i])
// (the same fixed-order tree as k_level_sums) and Q[r] = sums[r] / N.
__global__ __launch_bounds__(256) void k_level_sums_acc(int64_t count, int64_t N,
                                                        const double* __restrict__ lam,
                                                        int64_t ld, int64_t off,
                                                        const double* __restrict__ lam_prev,
                                                        int64_t ldp, int64_t offp,
                                                        double* __restrict__ sums,
                                                        double* __restrict__ Q) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  double s[1] = {0.0};
  if (count > 0) {
    const double* a = lam + (int64_t)r * ld + off;
    const double* p = lam_prev ? lam_prev + (int64_t)r * ldp + offp : nullptr;
    for (int64_t k = threadIdx.x; k < count; k += 256) s[0] += a[k] - (p ? p[k] : 0.0);
  }
  block_sums<256, 1>(s, red);
  if (threadIdx.x == 0) {
    const double t = sums[r] + s[0];
    sums[r] = t;
    Q[r] = t / (double)N;
  }
}

// Qhat_l, V_l (eq. sample_var) and Q^ML = sum_l Qhat_l; est[1] = sum_l V_l, or
// with shared = 1 (one set of shifts for all levels) the sample variance of
// the per-shift totals sum_l Q_l^(r)
__global__ void k_estimator_final(int L, int R, const double* __restrict__ Q,
                                  double* __restrict__ Qhat, double* __restrict__ V,
                                  double* __restrict__ est, int shared) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double qml = 0.0, vml = 0.0;
  for (int l = 0; l < L; ++l) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += Q[l * R + r];
    const double qh = s / R;
    double v = NAN;
    if (R > 1) {
      double d = 0.0;
      for (int r = 0; r < R; ++r) d += (qh - Q[l * R + r]) * (qh - Q[l * R + r]);
      v = d / ((double)R * (R - 1));
    }
    Qhat[l] = qh;
    V[l] = v;
    qml += qh;
    vml += v;
  }
  if (shared) {
    vml = NAN;
    if (R > 1) {
      double m = 0.0;
      for (int r = 0; r < R; ++r) {
        double t = 0.0;
        for (int l = 0; l < L; ++l) t += Q[l * R + r];
        m += t;
      }
      m /= R;
      double d = 0.0;
      for (int r = 0; r < R; ++r) {
        double t = 0.0;
        for (int l = 0; l < L; ++l) t += Q[l * R + r];
        d += (m - t) * (m - t);
      }
      vml = d / ((double)R * (R - 1));
    }
  }
  est[0] = qml;
  est[1] = vml;
}

}  // namespace

namespace {
int log2_exact(int64_t N) {
  int m = 0;
  while (((int64_t)1 << m) < N) ++m;
  return m;
}
}  // namespace

hipError_t launch_lattice(int64_t N, int s, const int64_t* z_dev, const double* shift_dev,
                          int64_t k0, int64_t count, double* Y, int64_t ldY, hipStream_t st) {
  const int64_t total = count * s;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lattice, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, N,
                     ldexp(1.0, -log2_exact(N)), s, 1, z_dev, shift_dev, (int64_t)s, k0, count, Y,
                     ldY, 0);
  return hipGetLastError();
}

hipError_t launch_lattice_multi(int64_t N, int s, int R, const int64_t* z_dev,
                                const double* shifts_dev, int64_t count, double* Y,
                                int64_t ldY, hipStream_t st) {
  const int64_t total = (int64_t)R * count * s;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lattice, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, N,
                     ldexp(1.0, -log2_exact(N)), s, R, z_dev, shifts_dev, (int64_t)s, (int64_t)0,
                     count, Y, ldY, 0);
  return hipGetLastError();
}

hipError_t launch_lattice_embedded(int64_t N, int s, int R, const int64_t* z_dev,
                                   const double* shifts_dev, int64_t sld, int64_t k0,
                                   int64_t count, double* Y, int64_t ldY, hipStream_t st) {
  const int64_t total = (int64_t)R * count * s;
  if (total <= 0) return hipSuccess;
  const int m = log2_exact(N);
  hipLaunchKernelGGL(k_lattice, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, N,
                     ldexp(1.0, -m), s, R, z_dev, shifts_dev, sld, k0, count, Y, ldY, m);
  return hipGetLastError();
}

hipError_t launch_phi_elements(int n, int s, const double* c, const int* k1, const int* k2,
                               double* phi, hipStream_t st) {
  if (s <= 0) return hipSuccess;
  const int E = 2 * n * n;
  hipLaunchKernelGGL(k_phi_elements, dim3((E + 255) / 256, s), dim3(256), 0, st, n, s, c, k1, k2,
                     phi);
  return hipGetLastError();
}

hipError_t launch_phi_edges(int n, int s, const double* phi_el, double* phi_edge,
                            hipStream_t st) {
  if (s <= 0) return hipSuccess;
  const int EW = 2 * (n - 1) * n;
  hipLaunchKernelGGL(k_phi_edges, dim3((EW + 255) / 256, s), dim3(256), 0, st, n, s, phi_el,
                     phi_edge);
  return hipGetLastError();
}

hipError_t launch_phi_edges_padded(int n, int s, const double* phi_el, double* phi_pad,
                                   hipStream_t st) {
  if (s <= 0) return hipSuccess;
  const int E = 2 * (n + 2) * n;
  hipLaunchKernelGGL(k_phi_edges_padded, dim3((E + 255) / 256, s), dim3(256), 0, st, n, s,
                     phi_el, phi_pad, (int64_t)E);
  return hipGetLastError();
}

hipError_t launch_phi_elements_islands(int n, int rows, const double* c, const int* k1,
                                       const int* k2, const int* region, double base_in,
                                       double base_out, double* phi, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int E = 2 * n * n;
  hipLaunchKernelGGL(k_phi_elements_islands, dim3((E + 255) / 256, rows), dim3(256), 0, st, n,
                     rows - 1, c, k1, k2, region, base_in, base_out, phi);
  return hipGetLastError();
}

hipError_t launch_phi_reaction_padded(int n, int rows, const double* phi_el, double* phi_r,
                                      hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int PG = (n + 2) * n;
  const int64_t stride = 3 * (int64_t)PG;
  hipLaunchKernelGGL(k_phi_edges_padded, dim3((2 * PG + 255) / 256, rows), dim3(256), 0, st, n,
                     rows, phi_el, phi_r, stride);
  hipLaunchKernelGGL(k_phi_diag_padded, dim3((PG + 255) / 256, rows), dim3(256), 0, st, n, rows,
                     phi_el, phi_r + 2 * PG, stride);
  return hipGetLastError();
}

hipError_t launch_expand(int64_t B, int s, int64_t E, const double* Y, int64_t ldY,
                         const double* phi, double a0, double* out, float* out32,
                         hipStream_t st, int64_t ldo) {
  if (B <= 0 || E <= 0) return hipSuccess;
  if (E & 1) return hipErrorInvalidValue;  // rows of phi are read in aligned pairs
  if (ldo == 0) ldo = E;
  if (ldo < E) return hipErrorInvalidValue;
  const int nbm = (int)((B + kXM - 1) / kXM);
  const int64_t nbn = (E + kXN - 1) / kXN;
  const int64_t ntiles = (int64_t)nbm * nbn;
  const int64_t per_xcd = (ntiles + 7) / 8;
  hipLaunchKernelGGL(k_expand_mfma, dim3((unsigned)(per_xcd * 8)), dim3(256), 0, st, B, s, E, Y,
                     ldY, phi, a0, out, out32, nbm, per_xcd, ntiles, ldo);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_prepend_one(int64_t B, int s, const double* __restrict__ Y,
                                                     int64_t ldY, double* __restrict__ Y1) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t w = s + 1;
  if (id >= B * w) return;
  const int64_t b = id / w;
  const int j = (int)(id - b * w);
  Y1[id] = j == 0 ? 1.0 : Y[b * ldY + j - 1];
}

hipError_t launch_prepend_one(int64_t B, int s, const double* Y, int64_t ldY, double* Y1,
                              hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const int64_t tot = B * (s + 1);
  hipLaunchKernelGGL(k_prepend_one, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, B, s,
                     Y, ldY, Y1);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_or_flags(int64_t n, uint8_t* __restrict__ dst,
                                                  const uint8_t* __restrict__ src) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] |= src[i];
}

hipError_t launch_or_flags(int64_t n, uint8_t* dst, const uint8_t* src, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_or_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, dst, src);
  return hipGetLastError();
}

hipError_t launch_sep_sin(int n, int kmax, double* S, hipStream_t st) {
  const int64_t tot = (int64_t)kmax * (3 * n + 2);
  hipLaunchKernelGGL(k_sep_sin, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, kmax, S);
  return hipGetLastError();
}

hipError_t launch_expand_separable(int64_t B, int n, int s, int kx, int ky, const double* Y,
                                   int64_t ldY, const double* c, const int* cell_start,
                                   const int* cell_term, const double* S, double* U, double a0,
                                   double* out, float* out32, int64_t ldo, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (n < 64 || (n & 63) || kx < 1 || ky < 1 || kx > kSepMaxK || kx * ky > kSepMaxCells ||
      ldo < 2 * (int64_t)(n + 2) * n)
    return hipErrorInvalidValue;
  const int M = 3 * n + 2;
  hipLaunchKernelGGL(k_sep_rows, dim3((unsigned)((M + 63) / 64), (unsigned)B), dim3(256), 0, st, n,
                     s, kx, ky, Y, ldY, c, cell_start, cell_term, S, U);
  // four column waves of 32 columns per block; the block count is a multiple of 8
  const int cw_per = n / 32;
  const int64_t blocks = (B * cw_per + 3) / 4, per_xcd = (blocks + 7) / 8;
  const dim3 grid((unsigned)(8 * per_xcd));
#define MLQMC_SEP_MARCH(K)                                                                   \
  case K:                                                                                    \
    hipLaunchKernelGGL(k_sep_march<K>, grid, dim3(256), 0, st, B, n, kx, cw_per, per_xcd, U, \
                       S, a0, out, out32, ldo);                                              \
    break;
  switch ((kx + 3) / 4) {
    MLQMC_SEP_MARCH(1)
    MLQMC_SEP_MARCH(2)
    MLQMC_SEP_MARCH(3)
    MLQMC_SEP_MARCH(4)
    MLQMC_SEP_MARCH(5)
    MLQMC_SEP_MARCH(6)
    MLQMC_SEP_MARCH(7)
    MLQMC_SEP_MARCH(8)
  }
#undef MLQMC_SEP_MARCH
  static_assert(kSepMarchMaxNK == 8, "one case per NK");
  return hipGetLastError();
}

hipError_t launch_sep_tri(int n, int nH, int kx, const double* S, double* Tp, hipStream_t st) {
  if (nH < 2 || n % nH || kx < 1 || kx > kSepMaxK) return hipErrorInvalidValue;
  const int64_t tot = (int64_t)3 * (n / nH) * kx * 2 * nH;
  hipLaunchKernelGGL(k_sep_tri, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nH, kx,
                     S, Tp);
  return hipGetLastError();
}

hipError_t launch_sep_setup_dots(int64_t B, int n, int nH, int kx, const double* U,
                                 const double* Tp, const double* uH, double a0, double* part,
                                 hipStream_t st) {
  if (B <= 0) return hipSuccess;
  if (nH < 2 || nH > 16 * kSepTriMaxCT / 2 || n % nH || kx < 1 || kx > kSepMaxK)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sep_setup_dots, dim3((unsigned)B), dim3(256), 0, st, B, n, nH, kx, U, Tp,
                     uH, a0, part);
  return hipGetLastError();
}

hipError_t launch_level_sums(int64_t N, int R, const double* lam, const double* lam_prev,
                             double* Q, hipStream_t st) {
  hipLaunchKernelGGL(k_level_sums, dim3(R), dim3(256), 0, st, N, lam, lam_prev, Q);
  return hipGetLastError();
}

hipError_t launch_level_sums_acc(int64_t count, int64_t N, int R, const double* lam, int64_t ld,
                                 int64_t off, const double* lam_prev, int64_t ldp, int64_t offp,
                                 double* sums, double* Q, hipStream_t st) {
  hipLaunchKernelGGL(k_level_sums_acc, dim3(R), dim3(256), 0, st, count, N, lam, ld, off,
                     lam_prev, ldp, offp, sums, Q);
  return hipGetLastError();
}

hipError_t launch_estimator_final(int L, int R, const double* Q, double* Qhat, double* V,
                                  double* est, int shared, hipStream_t st) {
  hipLaunchKernelGGL(k_estimator_final, dim3(1), dim3(64), 0, st, L, R, Q, Qhat, V, est, shared);
  return hipGetLastError();
}

}  // namespace mlqmc
