/*
 * mlqmc.h -- C ABI of the MI355X two-grid MLQMC eigen-sample library.
 *
 * Problem (introduction, eq. evp, with b = 0, c = 1, D = (0,1)^2): the smallest
 * eigenvalue of  -div(a(x,y) grad u) = lambda u,  u = 0 on the boundary, for
 *     a(x,y) = a0 + sum_j y_j c_j sin(pi k1_j x1) sin(pi k2_j x2)      (eq. coeff)
 * truncated to s terms (eq. coeff_s), discretised by P1 finite elements on the
 * uniform "/"-diagonal triangulation with h = 1/n (section 2.3), the stiffness
 * coefficient taken at element centroids and the mass matrix exact.
 *
 * Interior nodes (i,j), 1 <= i,j <= n-1, are stored row-major with x fastest:
 * index (j-1)*(n-1) + (i-1).  Elements of square (i,j) are numbered 2*(j*n+i)
 * (lower, vertices (i,j),(i+1,j),(i+1,j+1)) and 2*(j*n+i)+1 (upper, vertices
 * (i,j),(i+1,j+1),(i,j+1)).  Multi-sample arrays are sample-major.
 *
 * Conventions for every call:
 *  - returns mlqmc_status; nothing throws or aborts across the ABI;
 *  - the caller owns every buffer; inputs are only read during the call;
 *  - io_on_device (in mlqmc_opts, or the argument of the component calls)
 *    selects device pointers (1; work is enqueued on the context's stream and
 *    the call returns after that stream has finished it) or host pointers (0);
 *  - on MLQMC_EINVAL nothing is written and mlqmc_last_error() says why;
 *  - a context is bound to one device and one stream and is not reentrant:
 *    use one context per host thread.
 */
#ifndef MLQMC_H
#define MLQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLQMC_OK = 0,
  MLQMC_EINVAL = -1,   /* invalid argument; nothing written */
  MLQMC_ENOMEM = -2,   /* device allocation failed or exceeds opts.device_mem_cap */
  MLQMC_EDEVICE = -3,  /* HIP runtime error (text in mlqmc_last_error) */
  MLQMC_ENOCONV = -4   /* >= 1 sample flagged; every output is still written */
} mlqmc_status;

typedef enum { MLQMC_FP64 = 0, MLQMC_MIXED = 1 } mlqmc_precision;

/* per-sample flag bits */
#define MLQMC_FLAG_RQ_NOCONV   1u  /* Rayleigh-quotient iteration hit max_rq_iter */
#define MLQMC_FLAG_LIN_NOCONV  2u  /* a linear solve hit max_lin_iter */
#define MLQMC_FLAG_BREAKDOWN   4u  /* non-positive curvature in the projected solve */
#define MLQMC_FLAG_NONFINITE   8u  /* NaN/Inf produced */
#define MLQMC_FLAG_WRONG_PAIR 16u  /* converged vector has M-overlap < 1/2 with
                                      sin(pi x1) sin(pi x2): not the first eigenpair */

typedef struct mlqmc_ctx mlqmc_ctx;

/* Coefficient family (eq. coeff): a0 + sum_{j<s} y_j c[j] sin(pi k1[j] x1) sin(pi k2[j] x2).
 * Host arrays of length s_max, copied by mlqmc_create.  Requirements
 * (Assumption A1.3 with |y_j| <= 1/2): a0 - 0.5 * sum_j |c[j]| > 0, k1, k2 >= 1. */
typedef struct {
  int32_t s_max;
  double a0;
  const double* c;
  const int32_t* k1;
  const int32_t* k2;
} mlqmc_coeff;

/* One level of the estimator (Algorithm 2).  n_* are 1/h; powers of two.
 *  n_fine, s_fine   : fine mesh h_l and truncation s_l;
 *  n_coarse, s_coarse: coarse mesh H_l and truncation S_l of the two-grid step
 *                     (Algorithm 1); n_coarse == 0 means a direct eigensolve
 *                     on the fine mesh (lambda_{h_l,s_l}, level 0 of Algorithm 2);
 *  n_prev, s_prev   : mesh and truncation of the level-(l-1) term evaluated at
 *                     the same point with the same coarse pair; 0 = no such term.
 * Limits: 4 <= n_coarse <= 64 and n_coarse < n_fine <= 1024 for two-grid levels;
 * 4 <= n_fine <= 64 for direct levels (the eigensolve runs in LDS up to 1/32; on
 * 1/64 in FP64 with each chain's top level in global scratch). */
typedef struct {
  int32_t n_fine, s_fine;
  int32_t n_coarse, s_coarse;
  int32_t n_prev, s_prev;
} mlqmc_level;

typedef struct {
  int32_t prec;              /* mlqmc_precision */
  double eig_rtol;           /* RQ iteration stops when |sigma_k - sigma_{k-1}| <= eig_rtol*sigma_k;
                                the iteration converges cubically, so the returned
                                sigma_k is accurate far below eig_rtol */
  int32_t max_rq_iter;       /* cap on RQ iterations per coarse eigensolve */
  double lin_rtol;           /* fine two-grid solve: projected PCG stops at sqrt(r.z / r0.z0) <= lin_rtol
                                (0 = the precision's default: FP64 1e-10, mixed 1e-7) ... */
  double lam_rtol;           /* ... or when the estimated error of the Rayleigh quotient of the
                                current iterate is <= lam_rtol * lambda (0 = default: FP64 5e-12,
                                mixed 5e-10, a factor >= 10 inside the stated accuracies 1e-10
                                and 1e-8) */
  double rq_lin_rtol;        /* the same test for the inner solves of the RQ iteration; the
                                iteration converges from inexact inner solves, so a loose
                                value (default 1e-2) costs fewer inner steps in total */
  int32_t max_lin_iter;      /* cap on PCG iterations per linear solve */
  int32_t chain_len;         /* samples per warm-start chain (<=0: library default) */
  int32_t batch;             /* samples per fine-solve batch (<=0: library default, up to
                                96 GB of working arrays, split evenly) */
  int32_t pcg_graph;         /* 1: replay the batched PCG iterations from a captured HIP graph
                                (cached per layout); 0: launch them one by one */
  int32_t io_on_device;      /* 1: device pointers, 0: host pointers */
  int64_t device_mem_cap;    /* bytes; 0 = unlimited (a test hook for MLQMC_ENOMEM) */
  double eig_atol;           /* > 0: the RQ iteration stops when |sigma_k - sigma_{k-1}| <= eig_atol
                                instead (an absolute tolerance, as in section 5, which uses
                                5e-8); 0 (default): eig_rtol */
} mlqmc_opts;

/* Fills *opt with the defaults (FP64, eig_rtol 1e-8, max_rq_iter 12,
 * lin_rtol 0 and lam_rtol 0 (per precision), rq_lin_rtol 1e-2, max_lin_iter 60,
 * pcg_graph 1, io_on_device 0). */
void mlqmc_default_opts(mlqmc_opts* opt);

/* Creates a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  Validates and copies
 * the coefficient family.  MLQMC_EDEVICE if the device does not exist.
 *
 * device = MLQMC_HOST_ONLY makes a host-only context: nothing touches a
 * device, and every call on it checks its arguments as on a device context,
 * returning MLQMC_EINVAL for invalid ones and MLQMC_EDEVICE (nothing written)
 * for valid ones.  It never computes; it exists so that argument checking can
 * be exercised on a machine without a GPU. */
#define MLQMC_HOST_ONLY (-1)
mlqmc_status mlqmc_create(mlqmc_ctx** out, const mlqmc_coeff* coeff, int device,
                          void* hip_stream);
/* Problem 2 of the numerical section (the domain with four interior islands
 * D_f = [1/8,3/8] or [5/8,7/8] in each coordinate): a diffusion coefficient a
 * and a reaction coefficient b, both affine in y with region-wise parts,
 *   a(x, y) = a0(x) + sum_{j<s} y_j ca[j] phi_j(x),
 *   b(x, y) = b0(x) + sum_{j<s} y_j cb[j] phi_j(x),
 *   a0 = a0_in on D_f and a0_out elsewhere (b0 likewise),
 *   phi_j = sin(pi k1[j] x1) sin(pi k2[j] x2) on region[j] (1: D_f, 2: the
 *           rest of D) and 0 on the other region.
 * The operator is the P1 stiffness matrix of a plus the P1 mass matrix
 * weighted by b (the element mass matrices times b at the centroid). */
typedef struct {
  int32_t s_max;
  double a0_in, a0_out, b0_in, b0_out;
  const double* ca;       /* [s_max] host */
  const double* cb;       /* [s_max] host */
  const int32_t* k1;      /* [s_max] host, >= 1 */
  const int32_t* k2;      /* [s_max] host, >= 1 */
  const int32_t* region;  /* [s_max] host, 1 or 2 */
} mlqmc_islands;

/* Creates a context for the Problem 2 family (arguments as mlqmc_create).
 * Requires a >= a0_* - 0.5 sum |ca| > 0 and b >= 0 on each region for all
 * |y_j| <= 1/2 (MLQMC_EINVAL otherwise).  Contexts of this family run their
 * eigensolves (direct and coarse meshes) on 1/8 .. 1/32, every array of a
 * solve in LDS, and take 1/64 .. 1/1024 as the fine or previous mesh of a
 * two-grid level (the batched kernels with the reaction term: weight blocks
 * [WX | WY | RX | RY | RD] from two coefficient products), in either
 * precision; meshes are multiples of 1/8 so that the islands' edges are mesh
 * lines.  The level and estimator calls return MLQMC_EINVAL for other meshes,
 * and mlqmc_coefficient / mlqmc_apply_operator / mlqmc_edge_weights for any
 * call (they cover Problem 1). */
mlqmc_status mlqmc_create_islands(mlqmc_ctx** out, const mlqmc_islands* cf, int device,
                                  void* hip_stream);
/* Frees everything the context allocated.  NULL-safe. */
void mlqmc_destroy(mlqmc_ctx* ctx);
/* Text of the last error on this context (owned by ctx, valid until the next
 * call on it).  Accepts NULL (returns the text of the last failed create). */
const char* mlqmc_last_error(const mlqmc_ctx* ctx);

/* ---- components of the hot path (one call per step, for parity checks) ---- */

/* Randomly shifted rank-1 lattice points (eq. rqmc, eq. t_kl):
 *   Y[i][j] = frac(((k0+i) * z[j] mod N) / N + shift[j]) - 1/2,  i < count, j < s.
 * N a power of two; z[j] in [0, N); shift[j] in [0,1).  z, shift are host
 * arrays; Y is [count x s] (device if io_on_device). */
mlqmc_status mlqmc_lattice_points(mlqmc_ctx* ctx, int64_t N, int32_t s, const int64_t* z,
                                  const double* shift, int64_t k0, int64_t count,
                                  double* Y, int32_t io_on_device);

/* Points of the base-2 embedded lattice rule (embedded rules of section 2.5;
 * the block-by-block enumeration of section 5): point k of N = 2^m points is
 * the lattice point with index rev_m(k), the m-bit reversal of k,
 *   Y[i][j] = frac((rev_m(k0+i) * z[j] mod N) / N + shift[j]) - 1/2,
 * so the first 2^m' points always form the 2^m'-point lattice and each later
 * block fills the gaps between the earlier points.  k0 + count <= N; other
 * arguments and errors as mlqmc_lattice_points. */
mlqmc_status mlqmc_embedded_points(mlqmc_ctx* ctx, int64_t N, int32_t s, const int64_t* z,
                                   const double* shift, int64_t k0, int64_t count,
                                   double* Y, int32_t io_on_device);

/* Coefficient at the element centroids (eq. coeff_s, centroid rule):
 *   aK[b][e] = a0 + sum_{j<s} Y[b][j] c_j sin(pi k1_j xc_e) sin(pi k2_j yc_e)
 * Y is [B x s], aK is [B x 2n^2]. */
mlqmc_status mlqmc_coefficient(mlqmc_ctx* ctx, int32_t n, int32_t s, int64_t B,
                               const double* Y, double* aK, int32_t io_on_device);

/* Matrix-free P1 operator (section 2.3): out[b] = (A_h(y_b) - sigma[b] M_h) x[b],
 * A from the centroid coefficient with s terms, M the consistent mass matrix.
 * Y [B x s], sigma [B], x and out [B x (n-1)^2]. */
mlqmc_status mlqmc_apply_operator(mlqmc_ctx* ctx, int32_t n, int32_t s, int64_t B,
                                  const double* Y, const double* sigma, const double* x,
                                  double* out, int32_t io_on_device);

/* Edge weights of the fine-mesh solves (eq. coeff at the element centroids,
 * the quadrature of section 4.2; on these right-isosceles elements a
 * horizontal or vertical edge couples its two nodes in the stiffness matrix
 * of section 2.3 with the mean of a over the two elements sharing it, and
 * hypotenuses do not couple).  For B points Y [B x s] (row stride s), out
 * [B x 2 (n+2) n] receives the padded [WX | WY] blocks the batched kernels
 * read: WX[j n + i] the edge arriving at node (i, j) from the west
 * (i, j = 1..n-1), column 0 of row j + 1 the edge from node (n-1, j) into the
 * right boundary (j = 1..n-1), WY[j n + i] the edge arriving from the south
 * (i = 1..n-1, j = 1..n), every other entry a0.  Formed as those solves form
 * them for this family and truncation: the separable product (sums over k1
 * and k2 of the sine pairs) when the largest k1 among the s terms, kx, has
 * kx <= 32, 4 kx < s and kx times the largest k2 <= 1024, else the table
 * product.
 * Problem 1 only; n a power of two in [64, 1024]; host or device memory as
 * on_dev.  MLQMC_EINVAL for other arguments (nothing written). */
mlqmc_status mlqmc_edge_weights(mlqmc_ctx* ctx, int32_t n, int32_t s, int64_t B,
                                const double* Y, double* out, int32_t on_dev);

/* P1 interpolation from mesh 1/nH to mesh 1/nh (nh a multiple of nH; section 3):
 * uh[b] = values at the fine interior nodes of the coarse P1 function uH[b]. */
mlqmc_status mlqmc_prolong(mlqmc_ctx* ctx, int32_t nH, int32_t nh, int64_t B, const double* uH,
                           double* uh, int32_t io_on_device);

/* ---- the hot path ---- */

/* Eigen-samples of one level for an explicit point batch Y [n x s_fine]:
 *   direct level:   lam[i] = lambda_{h,s}(y_i) (smallest FE eigenvalue), and
 *                   lam_prev[i] = lambda_{h_prev,s_prev}(y_i) if n_prev > 0;
 *   two-grid level: coarse pair by warm-started RQ iteration on (H,S), then
 *                   lam[i] = lambda^{h,s}(y_i) (Algorithm 1) and, if n_prev > 0,
 *                   lam_prev[i] = the same update on (h_prev, s_prev) from the
 *                   same coarse pair (Algorithm 2).
 * warm_chain = 1: sample i starts its RQ iteration from the eigenvector of
 * sample i-1 of the same chain (the nearby-QMC-point start of section 4.3),
 * chains being runs of opt->chain_len consecutive samples; 0: every sample
 * starts from the eigenvector of the coefficient a = a0.
 * lam_prev, lam_coarse, rq_iters, lin_iters may be NULL.  lam_coarse[i] =
 * lambda_{H,S}(y_i) (NaN on direct levels); rq_iters[i] = RQ iterations of the
 * coarse eigensolve; lin_iters[i] = PCG iterations of the fine solve(s);
 * flags[i] = MLQMC_FLAG_* bits.
 * g, g_prev (NULL or [n]): the linear functional of the eigenfunction the
 * introduction estimates alongside lambda, G(u) = integral over D of u, for
 * the level's eigenvector approximation (the direct eigenvector, or the
 * two-grid w) normalised to ||u||_M = 1 with the sign that makes the
 * integral positive; g_prev the same for the level-(l-1) approximation
 * (written only if n_prev > 0).  With g or g_prev requested the two-grid
 * solves stop on the residual test alone, and each converged eigenvector of
 * the RQ iteration (direct or coarse) is refined by one correction solve to
 * lin_rtol (FP64).  Returns MLQMC_ENOCONV if any flag is set. */
mlqmc_status mlqmc_eig_level(mlqmc_ctx* ctx, const mlqmc_level* lvl, const mlqmc_opts* opt,
                             int64_t n, const double* Y, int32_t warm_chain, double* lam,
                             double* lam_prev, double* lam_coarse, int32_t* rq_iters,
                             int32_t* lin_iters, uint8_t* flags, double* g, double* g_prev);

/* Bytes of device scratch the library holds on every GPU it runs on (one
 * static copy per device, kept until the process ends) for
 * mlqmc_eig_level_noalloc. */
#define MLQMC_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as mlqmc_eig_level, without g / g_prev, that allocates nothing.
 * Every intermediate (coefficient tables of the level's meshes, coarse
 * vectors, counters) lives in the library's static device scratch of
 * MLQMC_NOALLOC_SCRATCH_BYTES on this context's device; its address is taken
 * once per device when a context is created there.
 * Requirements: opt->io_on_device = 1 (Y and every output are device
 * pointers); every mesh of the level (fine, coarse, previous) 1/32 or coarser
 * (the per-sample LDS solvers).  Arguments, outputs, flags and return codes
 * as mlqmc_eig_level.  MLQMC_EINVAL (nothing written) when the call would
 * need more scratch than the maximum: about 8 (n_coarse - 1)^2 bytes per
 * sample on a two-grid level plus the coefficient tables, 8 (2 n^2 +
 * 2 (n + 2) n) bytes per term and mesh (twice that for Problem 2).
 * The scratch is shared by every call on one GPU and keeps the last call's
 * contents (each call rebuilds what it reads): calls that overlap on one GPU
 * (other streams, threads or contexts) race, so the caller serialises them. */
mlqmc_status mlqmc_eig_level_noalloc(mlqmc_ctx* ctx, const mlqmc_level* lvl,
                                     const mlqmc_opts* opt, int64_t n, const double* Y,
                                     int32_t warm_chain, double* lam, double* lam_prev,
                                     double* lam_coarse, int32_t* rq_iters, int32_t* lin_iters,
                                     uint8_t* flags);

/* Two-grid MLQMC estimator (Algorithm 2; eq. tg-mlqmc, eq. sample_var, eq. ml-var).
 * Levels l = 0..n_levels-1 with N[l] points (powers of two), R shifts, z the
 * concatenated generating vectors ([s_fine of level l] each) and shifts the
 * concatenated [R x s_fine] blocks per level, values in [0,1).  All of z, N,
 * shifts and lvls are host arrays.  Outputs (host unless opt->io_on_device):
 *   Q_lr [n_levels x R] = Q_l^(r), Qhat [n_levels], V [n_levels] (NaN if R == 1),
 *   est[0] = Q^ML = sum_l Qhat_l, est[1] = sum_l V_l.
 * g_stats (NULL, or [n_levels x R + 2 n_levels + 2]): the same estimator for
 * E[G(u)] (G as in mlqmc_eig_level; the telescoping sum of the introduction
 * with Y_l = G(u^l) - G(u^{l-1})), laid out as Q_lr, Qhat, V, est. */
mlqmc_status mlqmc_estimate(mlqmc_ctx* ctx, int32_t n_levels, const mlqmc_level* lvls,
                            const int64_t* N, int32_t R, const int64_t* z, const double* shifts,
                            const mlqmc_opts* opt, double* Q_lr, double* Qhat, double* V,
                            double* est, double* g_stats);

/* Nested two-grid MLQMC estimator with shared shifts (end of section 4.3):
 * one embedded rule (z [s_max], s_max = max_l s_fine, entries in [0, 2^31); a
 * rule of N points uses them modulo N) and one set of R shifts ([R x s_max],
 * values in [0,1)) serve every level; level l uses the first N[l] points of
 * the embedded rule (N[l] powers of two, non-increasing) and the first s_fine
 * components.  The level list must be:
 *   level 0   direct (n_coarse = 0, n_prev = 0);
 *   level l>0 two-grid with (n_coarse, s_coarse) = level 0's (n_fine, s_fine)
 *             and (n_prev, s_prev) = level l-1's (n_fine, s_fine);
 * so the coarse pair of every point is its level-0 eigenpair (H_l = h_0) and
 * lambda^{l-1} at level l is the value level l-1 computed at the same point:
 * no coarse eigensolve after level 0 and no recomputed previous term.
 * Outputs as mlqmc_estimate, except est[1] = the sample variance (eq.
 * sample_var) of the per-shift totals sum_l Q_l^(r): with shared shifts the
 * level terms of one shift are dependent and sum_l V_l is no longer the
 * variance of Q^ML.  lam_out (NULL, or [R * sum_l N[l]]) receives lambda^l at
 * every point, level-major, then shift r, then point k.  g_stats as in
 * mlqmc_estimate (with est[1] of the functional again the variance of the
 * per-shift totals).
 * Errors: MLQMC_EINVAL (a level list of another shape, N, z or shifts out of
 * range), MLQMC_ENOMEM, MLQMC_EDEVICE; MLQMC_ENOCONV if a sample is flagged
 * (all outputs still written). */
mlqmc_status mlqmc_estimate_nested(mlqmc_ctx* ctx, int32_t n_levels, const mlqmc_level* lvls,
                                   const int64_t* N, int32_t R, const int64_t* z,
                                   const double* shifts, const mlqmc_opts* opt, double* Q_lr,
                                   double* Qhat, double* V, double* est, double* lam_out,
                                   double* g_stats);

/* Extensible nested estimate (embedded rules of sections 2.5 and 5, shared
 * shifts of section 4.3): the points of the embedded base-2 rule do not depend
 * on its size (point k is the lattice point phi_2(k) z + shift for every rule
 * of more than k points), so an estimate over N_done[l] points per level
 * continues to N[l] by adding the level values of the points
 * [N_done[l], N[l]).  sums [n_levels x R] (in/out, host or device as
 * io_on_device) holds the per-(level, shift) sums of Y_l = lambda^l -
 * lambda^{l-1} over the first N_done[l] points (zeros with N_done = 0); on
 * return it holds them over the first N[l].  Q_lr = sums / N[l] and Qhat, V,
 * est then follow as in mlqmc_estimate_nested, for N[l] points.  g_sums and
 * g_stats (both NULL, or [n_levels x R] and as in mlqmc_estimate) do the same
 * for G.  Calling it with N_done = 0 and zero sums equals
 * mlqmc_estimate_nested (without lam_out); a chain of calls equals one call
 * to rounding (the sums are added in another order).  The values at a point
 * are recomputed where a level needs the previous level's there (level l is
 * evaluated from min(N_done[l], N_done[l+1])).
 * Errors as mlqmc_estimate_nested, and MLQMC_EINVAL for N_done[l] outside
 * [0, N[l]]; on an error other than MLQMC_ENOCONV the sums are unchanged. */
mlqmc_status mlqmc_estimate_nested_extend(mlqmc_ctx* ctx, int32_t n_levels,
                                          const mlqmc_level* lvls, const int64_t* N_done,
                                          const int64_t* N, int32_t R, const int64_t* z,
                                          const double* shifts, const mlqmc_opts* opt,
                                          double* sums, double* Q_lr, double* Qhat, double* V,
                                          double* est, double* g_sums, double* g_stats);

/* ---- tuning ---- */

/* ---- adaptive choice of N_l and L (nested estimator) ----
 *
 * The paper picks the points per level and the number of levels with a greedy
 * adaptive MLQMC algorithm it cites but does not state (section 4.2; the
 * numerical section's set-up).  This library's own rule, from what the paper
 * does state: the mean-square error is variance plus squared bias, so ask
 * sum_l V_l <= eps^2 / 2 (eq. sample_var, eq. ml-var) and bias <= eps / sqrt 2;
 * a sample on level l costs C_l = s_l h_l^-2 + h_l^-gamma (section 4.2, d = 2).
 *  - While the variance is too large, double N_l on the level with the largest
 *    V_l / (N_l C_l) (the first on ties); coarser levels are raised to at
 *    least the new N (nested rules need N_0 >= N_1 >= ...).
 *  - Then, while |Qhat_{L-1}| / (2^alpha - 1) (the remaining bias for level
 *    differences decaying like h_l^alpha, h halving per level) exceeds
 *    eps / sqrt 2, add a level with N_init points.
 * Sums are taken left to right in FP64. */
typedef struct {
  double eps;       /* target root-mean-square error of Q^ML */
  double alpha;     /* decay of E[Y_l] in h_l (2 for the eigenvalue, section 2.3) */
  double gamma;     /* solve-cost exponent (2: the multigrid-preconditioned solves) */
  int64_t N_init;   /* points of a level when it starts (power of two) */
  int64_t N_max;    /* no level grows beyond this (power of two, <= 2^30) */
} mlqmc_adaptive_opts;

enum {
  MLQMC_ADAPT_DONE = 0,    /* both targets met */
  MLQMC_ADAPT_DOUBLE = 1,  /* double N on *level */
  MLQMC_ADAPT_ADD = 2,     /* add level *level (= n_levels) */
  MLQMC_ADAPT_BUDGET = 3,  /* doubling *level would pass N_max: stop, not converged */
  MLQMC_ADAPT_LEVELS = 4   /* the bias needs a level beyond max_levels: stop, not converged */
};

/* One decision of the rule (host arithmetic only; no context or device):
 * from the current n_levels <= max_levels, Qhat, V, N and per-sample cost
 * arrays [n_levels].  Returns an MLQMC_ADAPT_* code and the level it concerns
 * in *level (-1 for DONE), or -1 on invalid arguments. */
int32_t mlqmc_adaptive_decide(int32_t n_levels, int32_t max_levels, const double* Qhat,
                              const double* V, const int64_t* N, const double* cost, double eps,
                              double alpha, int64_t N_max, int32_t* level);

/* The nested estimator (shared shifts, one embedded rule; as
 * mlqmc_estimate_nested, whose level list shape it requires for
 * lvls[0 .. max_levels)) with N_l and L chosen by the rule above: it starts
 * with min(2, max_levels) levels of N_init points and, after every decision,
 * evaluates only the new points (the extensible rule of
 * mlqmc_estimate_nested_extend).  z [s_max] and shifts [R x s_max] with s_max
 * = max s_fine over all max_levels levels.  Host arrays (opt->io_on_device =
 * 0); R >= 2.
 * Outputs: *n_levels = L used; N [max_levels] (first L written); Q_lr
 * [max_levels x R] (first L rows), Qhat, V [max_levels]; est[0] = Q^ML,
 * est[1] = sum_l V_l; *converged = 1 if the rule ended with both targets met;
 * trace [trace_cap x 2] the (action, level) of every decision, *trace_len
 * their count (may exceed trace_cap; only the first trace_cap are stored).
 * Errors as mlqmc_estimate_nested; MLQMC_ENOCONV if a sample was flagged (all
 * outputs still written). */
mlqmc_status mlqmc_estimate_adaptive(mlqmc_ctx* ctx, int32_t max_levels, const mlqmc_level* lvls,
                                     int32_t R, const int64_t* z, const double* shifts,
                                     const mlqmc_adaptive_opts* aopt, const mlqmc_opts* opt,
                                     int32_t* n_levels, int64_t* N, double* Q_lr, double* Qhat,
                                     double* V, double* est, int32_t* converged, int32_t* trace,
                                     int32_t trace_cap, int32_t* trace_len);

/* Sets how many workgroups in flight the batched stencil kernels of the fine
 * solve on mesh 1/n_fine (64..1024, a power of two) aim for in precision
 * `prec`; the number of row strips per sample follows from it and the batch
 * size.  0 restores the default (65536).  The package's autotuner measures
 * the choices on a device and writes a table the Python binding applies.
 * The strip count sets the order in which the solver's dot products are
 * summed, so results agree to rounding, not bit for bit, across settings.
 * Errors: MLQMC_EINVAL (mesh, precision or value out of range). */
mlqmc_status mlqmc_set_tuning(mlqmc_ctx* ctx, int32_t n_fine, int32_t prec,
                              int64_t target_blocks);

/* ---- instrumentation ---- */

/* Kernel classes that can be timed with HIP events around each launch. */
enum {
  MLQMC_K_NONE = 0,
  MLQMC_K_COEFF = 1,     /* coefficient expansion on the fine mesh */
  MLQMC_K_APPLY = 2,     /* fine operator apply inside the projected PCG */
  MLQMC_K_SMOOTH = 3,    /* finest-level coarse correction + post-smoothing + PCG dots */
  MLQMC_K_COARSE = 4,    /* eigensolves (coarse, direct and direct previous-level; the
                            chain kernel) */
  MLQMC_K_PRE = 5,       /* finest-level pre-smoothing + residual restriction */
  MLQMC_K_TG_LDS = 6     /* per-sample two-grid update in LDS (fine meshes up to 1/32);
                            its model bytes are 0 */
};
/* Selects the kernel class whose launches are bracketed by HIP events on the
 * context's stream (MLQMC_K_NONE disables) and clears the totals. */
mlqmc_status mlqmc_set_timing(mlqmc_ctx* ctx, int32_t kernel_class);
/* Number of timed launches, their summed duration in ms, and the summed
 * algorithmic bytes and flops of those launches (the library's per-kernel
 * model: bytes each array is moved once, flops of the arithmetic the kernel
 * must do; flops are counted for the coefficient expansion only, else 0).
 * Any output may be NULL. */
mlqmc_status mlqmc_get_timing(mlqmc_ctx* ctx, int64_t* launches, double* total_ms,
                              double* model_bytes, double* model_flops);

#ifdef __cplusplus
}
#endif

#endif /* MLQMC_H */
