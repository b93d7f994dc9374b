// Launch wrappers of the HIP kernels (host side).  Every wrapper enqueues on
// `st` and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlqmc {

// ---------------- per-sample LDS kernels (meshes 1/4 .. 1/32) ----------------

struct RqiArgs {
  const double* Y;      // points [n x ldY]; the first S columns are used
  int64_t ldY;
  int S;
  const double* phi;    // edge table [>=S][EW] of the mesh
  double a0;
  const double* rphi;   // Problem 2: reaction table [>=S+1][3 (n+2) n]; then phi and
                        // rphi carry the background values as row 0 and a0 is unused
                        // (meshes up to 1/32).  nullptr: Problem 1
  int64_t n;            // samples
  int chain_len;        // samples per warm-start chain (one workgroup per chain)
  int warm;             // 1: start from the previous sample's eigenvector
  double eig_rtol;
  double eig_atol;  // > 0: absolute RQ stopping tolerance instead of eig_rtol
  int max_rq;
  double lin_rtol;
  int max_lin;
  double* lam;          // [n] converged Rayleigh quotient
  double* u_out;        // [n x D] M-normalised eigenvectors, or nullptr
  int* rq_iters;        // [n] or nullptr
  int* lin_iters;       // [n] or nullptr
  uint8_t* flags;       // [n]
  double* g_out;        // [n] G(u) = integral of the M-normalised eigenvector, sign
                        // fixed positive, or nullptr; then each converged vector is
                        // first refined by one correction solve to g_lin_rtol (0: not)
  double g_lin_rtol;
  int refine;           // 1: refine converged vectors (as with g_out) without writing G
  double* scratch;      // meshes above 1/32: per-chain global scratch
  int64_t scratch_doubles;
  int mixed;            // 1: FP32 vectors, weights and V-cycle (meshes up to 1/32)
};
hipError_t launch_rqi(int N, const RqiArgs& a, hipStream_t st);
// doubles of global scratch one chain needs on mesh N (0: all in LDS)
int64_t rqi_scratch_doubles(int N);
// workgroups of the eigensolve on mesh N resident on the current device at once
int rqi_chains_in_flight(int N, int mixed, int reaction);

struct TgSmallArgs {
  const double* Y;      // [n x ldY], first s columns
  int64_t ldY;
  int s;
  const double* phi;    // edge table [>=s][EW] of the fine mesh
  double a0;
  const double* rphi;   // Problem 2 reaction table (as in RqiArgs), or nullptr
  const double* uH;     // [n x DH] coarse eigenvectors
  const double* lamH;   // [n]
  int nH;               // coarse mesh
  int64_t n;
  double lin_rtol;
  double lam_rtol;      // eigenvalue stopping test of the solve (0: residual test only)
  int mixed;            // 1: FP32 vectors, weights and V-cycle
  int max_lin;
  double* lam;          // [n] two-grid value
  double* g;            // [n] G of the two-grid eigenvector (integral, normalised), or nullptr
  int* lin_iters;       // [n] added to, or nullptr
  uint8_t* flags;       // [n] OR-ed
};
// Two-grid update with every array in LDS, one workgroup per sample (N <= 32)
hipError_t launch_tg_small(int N, const TgSmallArgs& a, hipStream_t st);

// One V-cycle X = K^{-1} B per active sample on mesh NB <= 32 from padded global
// arrays (weights [WX | WY], or [WX | WY | RX | RY | RD] with the reaction;
// rhs, X; see k_fine.hip), computed in LDS in the storage type T, three
// Chebyshev-weighted Jacobi sweeps per smoothing step.
template <typename T>
hipError_t launch_bottom_vcycle(int NB, int64_t B, const T* w, const T* rhs, T* X,
                                const uint8_t* active, int reaction, hipStream_t st);

// ---------------- batched fine-mesh kernels (XCD-aware 1-D grid over samples x blocks) ----------------

struct FineState {      // per-sample scalars of the projected PCG, arrays of length B
  double *mu, *vs, *rho, *rz, *rz0, *alpha, *c, *c2, *beta, *lam;
  // Rayleigh quotient of w_k = vn + t_k, tracked from the PCG dots:
  // f = w^T (A - mu M) w, m = w^T M w; dmp = the previous step's change of m,
  // rzp = the previous r.z (for the observed contraction)
  double *f, *m, *dmp, *rzp;
  double* g;            // G(w / ||w||_M) = |integral of w| / ||w||_M at the end, or nullptr
  int* its;
  int* lin_acc;         // per-sample PCG iteration totals, added to at the end (or nullptr)
  uint8_t* active;      // the sample still takes PCG steps
  uint8_t* vact;        // the sample still needs the preconditioner this step
  uint8_t* flags;
};

inline int64_t padded_size(int n) { return (int64_t)(n + 2) * n; }

// zero the Dirichlet positions (rows 0, n, n+1 and column 0) of cnt padded arrays
hipError_t launch_zero_boundary(int n, int64_t B, void* const* ptrs, int cnt, int elem,
                                hipStream_t st);

// interior layout -> interior layout (component entry point)
hipError_t launch_prolong_interior(int nH, int nh, int64_t B, const double* uH, double* uh,
                                   hipStream_t st);
// `reaction` (Problem 2): weight blocks [WX | WY | RX | RY | RD] and the
// operator A + R in every kernel below that takes the flag
template <typename T>
hipError_t launch_coarsen(int n, int64_t B, const T* w, T* wc, int reaction, hipStream_t st);
// The set-up and final kernels take the coarse eigenvectors uH [B x (nH-1)^2]
// and evaluate v = P u_H (P1 interpolation to mesh n) where they need it; they
// read the edge weights in the storage precision T and compute in FP64.
template <typename T>
hipError_t launch_setup_dots(int n, int64_t B, const double* uH, int nH, const T* w,
                             double* part, int reaction, hipStream_t st);
template <typename T>
hipError_t launch_setup_rhs(int n, int64_t B, const double* uH, int nH, const T* w,
                            const FineState& S, T* r, T* vn, T* mvn, int reaction,
                            hipStream_t st);
// the new direction pout = z - c2 vn + beta pin and q = (A - mu M) pout (stored
// only if q != nullptr), with the dot-product partials of the step (M vn is
// formed from vn in the kernel)
template <typename T>
hipError_t launch_pupdate_apply(int n, int64_t B, const T* z, const T* vn, const T* pin,
                                const T* w, T* t, const FineState& S, int first, T* pout, T* q,
                                double* part, int reaction, hipStream_t st);
// fused V-cycle level, pre-smoothing from zero and restriction:
//   X = Chebyshev-weighted Jacobi sweeps on A X = rhs from X = 0;
//   rhs_c = P^T (rhs - A X); with p != nullptr (the current direction) the rhs
//   is first updated, rhs - alpha (q - c mvn) -> rout, q = (A - mu M) p
//   recomputed from p
template <typename T>
hipError_t launch_pre(int n, int64_t B, const T* w, const T* rhs, T* X, T* rhs_c,
                      const uint8_t* active, const T* p, const T* mvn, const FineState* S,
                      T* rout, int reaction, hipStream_t st);
// fused V-cycle level, coarse correction and post-smoothing:
//   Xout = Chebyshev-weighted sweeps from Xin + P Xc; with part != nullptr also
//   the partials rhs.Xout, mvn.Xout, rhs.vn per strip (level 0 of the projected
//   PCG; rhs.vn is 0 with FP64 storage)
template <typename T>
hipError_t launch_post(int n, int64_t B, const T* w, const T* rhs, const T* Xin, const T* Xc,
                       T* Xout, const T* vn, const T* mvn, const uint8_t* active, double* part,
                       int reaction, hipStream_t st);
// strips per sample of launch_post for a batch of B (its partial-sum count per sample)
int post_strips(int n, int64_t B);
// workgroups in flight the batched stencil kernels aim for (<= 0: default);
// the strips per sample follow from it and the batch size
void set_target_blocks(int64_t v);
// blocks per sample of the row-marching kernels for a batch of B (their partial-sum count)
int march_blocks(int n, int64_t B);
template <typename T>
hipError_t launch_final_dots(int n, int64_t B, const double* uH, int nH, const T* t, const T* p0,
                             const T* p1, const T* w, const FineState& S, double* part,
                             int reaction, hipStream_t st);

// scalar phases: one wavefront per sample sums that sample's block partials
enum ScalarPhase {
  PH_SETUP = 0,
  PH_FIRST_RZ = 1,
  PH_ALPHA = 2,
  PH_BETA = 3,
  PH_FINAL = 4,
  PH_FINAL_TRACKED = 5  // the eigenvalue from the tracked quotient (no partial sums)
};
hipError_t launch_scalar(int phase, int n, int64_t B, int nblk, const double* part,
                         const FineState& S, double rtol, int max_it, hipStream_t st);

// plain operator apply out = (A - sigma M) x for the component entry point
hipError_t launch_apply_plain(int n, int64_t B, const double* w, const double* sigma,
                              const double* x, double* out, hipStream_t st);

// ---------------- points, tables, coefficient expansion, estimator ----------------

hipError_t launch_lattice(int64_t N, int s, const int64_t* z_dev, const double* shift_dev,
                          int64_t k0, int64_t count, double* Y, int64_t ldY, hipStream_t st);
// lattice points for R shifts at once: Y[(r*count + i) * ldY + j]
hipError_t launch_lattice_multi(int64_t N, int s, int R, const int64_t* z_dev,
                                const double* shifts_dev, int64_t count, double* Y,
                                int64_t ldY, hipStream_t st);
// the embedded base-2 order (N = 2^m): point k0 + i is lattice point
// rev_m(k0 + i); rows r * count + i, shift r at shifts_dev[r * sld ...]
hipError_t launch_lattice_embedded(int64_t N, int s, int R, const int64_t* z_dev,
                                   const double* shifts_dev, int64_t sld, int64_t k0,
                                   int64_t count, double* Y, int64_t ldY, hipStream_t st);
// element table phi[j][e] = c_j sin(pi k1_j xc_e) sin(pi k2_j yc_e), e < 2n^2
hipError_t launch_phi_elements(int n, int s, const double* c, const int* k1, const int* k2,
                               double* phi, hipStream_t st);
// edge table: the mean of the element table over the two elements of each leg
hipError_t launch_phi_edges(int n, int s, const double* phi_el, double* phi_edge,
                            hipStream_t st);
// the same edge table in the padded [WX | WY] layout of the batched kernels
hipError_t launch_phi_edges_padded(int n, int s, const double* phi_el, double* phi_pad,
                                   hipStream_t st);
// Problem 2 element table, `rows` = s + 1 rows: row 0 the background value by
// region (base_in on the islands), row j the region-masked term j - 1
hipError_t launch_phi_elements_islands(int n, int rows, const double* c, const int* k1,
                                       const int* k2, const int* region, double base_in,
                                       double base_out, double* phi, hipStream_t st);
// reaction edge table, rows of [RX | RY | RD], (n + 2) n entries each: the mean
// of the element table over the two elements of each horizontal, vertical and
// diagonal edge, in the padded layout (RX, RY as WX, WY; RD[k] the diagonal
// edge arriving at node k from the south-west)
hipError_t launch_phi_reaction_padded(int n, int rows, const double* phi_el, double* phi_r,
                                      hipStream_t st);
// out[b * ldo + e] = a0 + sum_{j<s} Y[b][j] phi[j][e], e < E (ldo = 0: E);
// out32 the same rounded to FP32; either may be null
hipError_t launch_expand(int64_t B, int s, int64_t E, const double* Y, int64_t ldY,
                         const double* phi, double a0, double* out, float* out32,
                         hipStream_t st, int64_t ldo = 0);
// The separable expansion of a Problem 1 table (terms c_j sin(pi k1_j x1)
// sin(pi k2_j x2)): S [kmax x (3n+2)] the sines on the grid of thirds
// (launch_sep_sin once per mesh); cells of the kx x ky box of (k1, k2) in CSR
// (cell_start [kx ky + 1], cell_term: the term indices of each cell, in order);
// U scratch [B x (3n+2) x kx].  Writes the padded [WX | WY] of B samples at
// out[b * ldo ...] and / or out32, equal to launch_expand with the padded edge
// table up to rounding.  n a multiple of 64, kx <= 32, kx ky <= 1024.
hipError_t launch_sep_sin(int n, int kmax, double* S, hipStream_t st);
// The set-up products v^T M v and v^T A v of v = P u_H (mesh n from mesh nH)
// from coarse quantities, for the separable expansion: Tp [3 (n/nH) kx x 2 nH]
// the sample-independent interval sums of S (launch_sep_tri once per mesh
// pair), U the row sums the expansion of the same batch left in its scratch.
// Writes part[2 b], part[2 b + 1] as the set-up kernel's partial sums with one
// block per sample (v.M12 v without the mass scale, v.A v).  nH <= 64.
hipError_t launch_sep_tri(int n, int nH, int kx, const double* S, double* Tp, hipStream_t st);
hipError_t launch_sep_setup_dots(int64_t B, int n, int nH, int kx, const double* U,
                                 const double* Tp, const double* uH, double a0, double* part,
                                 hipStream_t st);
// dst[i] |= src[i], i < n
hipError_t launch_or_flags(int64_t n, uint8_t* dst, const uint8_t* src, hipStream_t st);
hipError_t launch_expand_separable(int64_t B, int n, int s, int kx, int ky, const double* Y,
                                   int64_t ldY, const double* c, const int* cell_start,
                                   const int* cell_term, const double* S, double* U, double a0,
                                   double* out, float* out32, int64_t ldo, hipStream_t st);
// Y1[b] = (1, Y[b][0 .. s)): the points with the leading 1 that selects the
// background row of a Problem 2 table
hipError_t launch_prepend_one(int64_t B, int s, const double* Y, int64_t ldY, double* Y1,
                              hipStream_t st);
// Q[l*R + r] = (1/N) sum_k (lam[r*N + k] - lam_prev[r*N + k]) (fixed-order tree);
// lam_prev may be nullptr (lambda^{-1} = 0)
hipError_t launch_level_sums(int64_t N, int R, const double* lam, const double* lam_prev,
                             double* Q, hipStream_t st);
// sums[r] += sum_{i<count} (lam[r*ld + off + i] - lam_prev[r*ldp + offp + i]),
// Q[r] = sums[r] / N, r < R (lam_prev may be nullptr; the same tree as above)
hipError_t launch_level_sums_acc(int64_t count, int64_t N, int R, const double* lam, int64_t ld,
                                 int64_t off, const double* lam_prev, int64_t ldp, int64_t offp,
                                 double* sums, double* Q, hipStream_t st);
// Qhat, V, est from Q [L x R]; shared = 1: est[1] is the variance of the
// per-shift totals (one set of shifts for all levels) instead of sum_l V_l
hipError_t launch_estimator_final(int L, int R, const double* Q, double* Qhat, double* V,
                                  double* est, int shared, hipStream_t st);

}  // namespace mlqmc
