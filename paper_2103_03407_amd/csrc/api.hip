// C ABI of the two-grid MLQMC eigen-sample library: argument validation,
// device buffers, and the orchestration of the kernels for one level
// (coarse eigensolve -> two-grid updates) and for the estimator (Algorithm 2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mlqmc.h"
#include "kernels.h"

using namespace mlqmc;

namespace {

std::string g_create_error;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Coefficient tables of one mesh.  Problem 1: s rows, one per term.
// Problem 2: s + 1 rows, row 0 the background values a0, b0 by region; no
// interior-layout table; the reaction b in rel / rpad.
struct Table {
  int s = 0;
  int64_t bytes = 0;
  double* el = nullptr;    // [s][2n^2]
  double* edge = nullptr;  // [s][2(n-1)n]   interior-layout edge weights (LDS kernels)
  double* pad = nullptr;   // [s][2(n+2)n]   padded [WX | WY] edge weights (batched kernels)
  double* rel = nullptr;   // Problem 2: [s+1][2n^2] reaction at the centroids
  double* rpad = nullptr;  // Problem 2: [s+1][3(n+2)n] padded [RX | RY | RD] edge means
  void release() {
    // a failed free leaves a sticky error that the next HIP call reports
    for (double** q : {&el, &edge, &pad, &rel, &rpad}) {
      if (*q) (void)hipFree(*q);
      *q = nullptr;
    }
    s = 0;
    bytes = 0;
  }
};

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Status {
  mlqmc_status code = MLQMC_OK;
};

}  // namespace

// Device scratch of mlqmc_eig_level_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes this name to a kernel or a copy; it
// uses the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[MLQMC_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of `scratch` on it

// Address of `scratch` on `device`, which must be current: looked up once
// per device and kept.
hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[device] = p;
  *out = p;
  return hipSuccess;
}
}  // namespace

#define CARVE_OR_FAIL(expr)          \
  do {                               \
    mlqmc_status c_ = (expr);        \
    if (c_ != MLQMC_OK) return c_;   \
  } while (0)

struct mlqmc_ctx {
  int device = 0;
  bool host_only = false;  // created with MLQMC_HOST_ONLY: validates, never computes
  hipStream_t stream = nullptr;
  // captured PCG iterations (graph replay): one entry per fine-solve tag,
  // valid while every argument baked into it (the key) is unchanged
  struct PcgGraph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    int pairs = 0;  // replays the batch needed the last time it ran (0: not known)
  };
  std::map<std::string, PcgGraph> graphs;
  hipStream_t cap_stream = nullptr;  // private stream for capturing (default priority)
  // tuning: workgroups in flight for the batched stencil kernels, per
  // (fine mesh, precision); absent = the library default
  std::map<std::pair<int, int>, int64_t> target_blocks;
  // eigensolve workgroups resident on the device at once, per (mesh, precision)
  std::map<std::pair<int, int>, int> chain_slots;
  int64_t target_for(int n, int prec) const {
    auto it = target_blocks.find({n, prec});
    return it == target_blocks.end() ? 0 : it->second;
  }
  int s_max = 0;
  double a0 = 0.0;
  double* d_c = nullptr;
  int* d_k1 = nullptr;
  int* d_k2 = nullptr;
  // Problem 2 (islands): d_c holds the diffusion terms, d_cb the reaction's
  bool islands = false;
  double a_in = 0.0, a_out = 0.0, b_in = 0.0, b_out = 0.0;
  double* d_cb = nullptr;
  int* d_region = nullptr;
  std::map<std::string, DevBuf> bufs;
  std::map<int, Table> tables;
  // Problem 1 family on the host (the separable expansion's term boxes)
  std::vector<int> h_k1, h_k2;
  // separable expansion per (mesh, truncation): the term box kx x ky, its
  // cells in CSR, the sines on the grid of thirds
  struct SepTable {
    int kx = 0, ky = 0;
    int* cell_start = nullptr;
    int* cell_term = nullptr;
    double* S = nullptr;
    // per coarse mesh nH: the interval sums of S behind the coarse-side set-up
    // products (launch_sep_tri)
    std::map<int, double*> tri;
  };
  std::map<std::pair<int, int>, SepTable> seps;
  // No-allocation mode (mlqmc_eig_level_noalloc): named buffers and tables
  // are carved in order from this device's copy of `scratch` and live for one
  // call; nothing is allocated and nothing is cached past the call.
  void* scratch_base = nullptr;
  hipError_t scratch_err = hipSuccess;
  char* arena = nullptr;
  size_t arena_size = 0, arena_used = 0;
  std::map<int, Table> arena_tables;
  int64_t bytes_alloc = 0;
  int64_t mem_cap = 0;

  // The separable table for (n, s), or nullptr when the dense product is
  // taken: the separable form costs 4 kx flops per padded node and sample (two
  // element products of kx terms) against 4 s for the table product, both on
  // the matrix cores, plus the row sums U and their traffic; it is taken for
  // kx <= 32 and 4 kx < s, which leaves the row sums a wide margin.
  mlqmc_status sep_table(int n, int s, SepTable** out) {
    *out = nullptr;
    if (islands || n < 64 || (n % 64) || s < 1 || (int)h_k1.size() < s) return MLQMC_OK;
    int kx = 0, ky = 0;
    for (int j = 0; j < s; ++j) {
      kx = std::max(kx, h_k1[j]);
      ky = std::max(ky, h_k2[j]);
    }
    if (kx > 32 || kx * ky > 1024 || !(4 * kx < s)) return MLQMC_OK;
    SepTable& t = seps[{n, s}];
    if (!t.S) {
      const int kmax = std::max(kx, ky), cells = kx * ky;
      std::vector<int> start(cells + 1, 0), term(s);
      for (int j = 0; j < s; ++j) ++start[(h_k1[j] - 1) * ky + (h_k2[j] - 1) + 1];
      for (int c = 0; c < cells; ++c) start[c + 1] += start[c];
      std::vector<int> fill(start.begin(), start.end() - 1);
      for (int j = 0; j < s; ++j) term[fill[(h_k1[j] - 1) * ky + (h_k2[j] - 1)]++] = j;
      const size_t bs = (size_t)kmax * (3 * n + 2) * sizeof(double);
      const size_t bc = (cells + 1) * sizeof(int), bt = (size_t)s * sizeof(int);
      if (mem_cap > 0 && bytes_alloc + (int64_t)(bs + bc + bt) > mem_cap)
        return fail(MLQMC_ENOMEM, "separable table for n=%d exceeds the device memory cap", n);
      hipError_t e = hipMalloc(&t.S, bs);
      if (e == hipSuccess) e = hipMalloc(&t.cell_start, bc);
      if (e == hipSuccess) e = hipMalloc(&t.cell_term, bt);
      if (e == hipSuccess)
        e = hipMemcpy(t.cell_start, start.data(), bc, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(t.cell_term, term.data(), bt, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = launch_sep_sin(n, kmax, t.S, stream);
      if (e != hipSuccess) {
        for (void* q : {(void*)t.S, (void*)t.cell_start, (void*)t.cell_term})
          if (q) (void)hipFree(q);
        seps.erase({n, s});
        return fail(MLQMC_ENOMEM, "separable table: %s", hipGetErrorString(e));
      }
      bytes_alloc += (int64_t)(bs + bc + bt);
      t.kx = kx;
      t.ky = ky;
    }
    *out = &t;
    return MLQMC_OK;
  }
  // The interval sums of the separable table t for fine mesh n over coarse
  // mesh nH, or nullptr where the coarse-side set-up products do not apply
  // (nH > 64, n not a multiple of nH)
  mlqmc_status sep_tri(SepTable* t, int n, int nH, double** out) {
    *out = nullptr;
    if (!t || nH < 2 || nH > 64 || n % nH) return MLQMC_OK;
    auto it = t->tri.find(nH);
    if (it != t->tri.end()) {
      *out = it->second;
      return MLQMC_OK;
    }
    const size_t bytes = (size_t)3 * (n / nH) * t->kx * 2 * nH * sizeof(double);
    if (mem_cap > 0 && bytes_alloc + (int64_t)bytes > mem_cap)
      return fail(MLQMC_ENOMEM, "set-up table for n=%d exceeds the device memory cap", n);
    double* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) e = launch_sep_tri(n, nH, t->kx, t->S, p, stream);
    if (e != hipSuccess) {
      if (p) (void)hipFree(p);
      return fail(MLQMC_ENOMEM, "set-up table: %s", hipGetErrorString(e));
    }
    bytes_alloc += (int64_t)bytes;
    t->tri[nH] = p;
    *out = p;
    return MLQMC_OK;
  }
  std::string err;
  // timing
  int timing_class = MLQMC_K_NONE;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  int64_t t_launches = 0;
  double t_ms = 0.0;
  double t_bytes = 0.0;
  double t_flops = 0.0;

  mlqmc_status fail(mlqmc_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  mlqmc_status hip_fail(hipError_t e, const char* what) {
    return fail(MLQMC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  }
  // makes the context's device current for a call whose arguments passed
  mlqmc_status bind() {
    if (host_only)
      return fail(MLQMC_EDEVICE, "host-only context: the arguments are valid; no device to run on");
    hipError_t e = hipSetDevice(device);
    return e == hipSuccess ? MLQMC_OK : hip_fail(e, "set device");
  }

  mlqmc_status carve(const char* name, size_t bytes, void** out) {
    const size_t b = round256(bytes ? bytes : 8);
    if (arena_used + b > arena_size)
      return fail(MLQMC_ENOMEM, "no-allocation scratch exhausted by %s (%zu of %zu bytes used)",
                  name, arena_used, arena_size);
    *out = arena + arena_used;
    arena_used += b;
    return MLQMC_OK;
  }

  // streams of the levels that run beside the context's stream (default
  // priority, non-blocking) and the fork / join events, created on first use
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> sync_ev;
  mlqmc_status side_stream(int k, hipStream_t* out) {
    while ((int)side.size() <= k) {
      hipStream_t s = nullptr;
      const hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "side stream");
      side.push_back(s);
    }
    *out = side[k];
    return MLQMC_OK;
  }
  mlqmc_status event(int k, hipEvent_t* out) {
    while ((int)sync_ev.size() <= k) {
      hipEvent_t ev = nullptr;
      const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "event");
      sync_ev.push_back(ev);
    }
    *out = sync_ev[k];
    return MLQMC_OK;
  }

  // growable named device buffer
  mlqmc_status get(const char* name, size_t bytes, void** out) {
    if (arena) return carve(name, bytes, out);
    DevBuf& b = bufs[name];
    if (b.bytes >= bytes && b.p) {
      *out = b.p;
      return MLQMC_OK;
    }
    if (b.p) {
      zeroed.erase(b.p);
      (void)hipFree(b.p);
      bytes_alloc -= (int64_t)b.bytes;
      b.p = nullptr;
      b.bytes = 0;
    }
    if (bytes == 0) bytes = 8;
    if (mem_cap > 0 && bytes_alloc + (int64_t)bytes > mem_cap)
      return fail(MLQMC_ENOMEM, "buffer %s: %zu bytes exceed the device memory cap", name, bytes);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      b.p = nullptr;
      return fail(MLQMC_ENOMEM, "hipMalloc(%zu) for %s: %s", bytes, name, hipGetErrorString(e));
    }
    b.bytes = bytes;
    bytes_alloc += (int64_t)bytes;
    *out = b.p;
    return MLQMC_OK;
  }
  // Padded per-node buffers whose Dirichlet positions are known to be zero:
  // pointer -> (mesh, element size, samples).  Kernels never write those
  // positions, so a buffer is zeroed once per layout, not once per call.
  struct ZeroKey {
    int n, elem;
    int64_t batch;
  };
  std::map<void*, ZeroKey> zeroed;
  bool boundary_is_zero(void* p, int n, int elem, int64_t batch) const {
    auto it = zeroed.find(p);
    return it != zeroed.end() && it->second.n == n && it->second.elem == elem &&
           it->second.batch >= batch;
  }

  template <typename T>
  mlqmc_status getT(const char* name, size_t count, T** out) {
    void* p = nullptr;
    mlqmc_status s = get(name, count * sizeof(T), &p);
    *out = static_cast<T*>(p);
    return s;
  }

  // Tables in the no-allocation scratch: the element and padded edge tables
  // (and the reaction's), rebuilt in every call.
  mlqmc_status arena_table(int n, int s, Table** out) {
    Table& t = arena_tables[n];
    const int rows = islands ? s + 1 : std::max(s, 1);
    if (t.el && t.s >= (islands ? s : rows)) {
      *out = &t;
      return MLQMC_OK;
    }
    void *el = nullptr, *pad = nullptr, *rel = nullptr, *rpad = nullptr;
    CARVE_OR_FAIL(carve("table", (size_t)rows * 2 * n * n * 8, &el));
    CARVE_OR_FAIL(carve("table", (size_t)rows * 2 * padded_size(n) * 8, &pad));
    if (islands) {
      CARVE_OR_FAIL(carve("table", (size_t)rows * 2 * n * n * 8, &rel));
      CARVE_OR_FAIL(carve("table", (size_t)rows * 3 * padded_size(n) * 8, &rpad));
    }
    t.el = (double*)el;
    t.pad = (double*)pad;
    t.rel = (double*)rel;
    t.rpad = (double*)rpad;
    t.edge = nullptr;
    hipError_t e;
    if (islands) {
      t.s = s;
      e = launch_phi_elements_islands(n, rows, d_c, d_k1, d_k2, d_region, a_in, a_out, t.el,
                                      stream);
      if (e == hipSuccess) e = launch_phi_edges_padded(n, rows, t.el, t.pad, stream);
      if (e == hipSuccess)
        e = launch_phi_elements_islands(n, rows, d_cb, d_k1, d_k2, d_region, b_in, b_out, t.rel,
                                        stream);
      if (e == hipSuccess) e = launch_phi_reaction_padded(n, rows, t.rel, t.rpad, stream);
    } else {
      t.s = rows;
      e = launch_phi_elements(n, rows, d_c, d_k1, d_k2, t.el, stream);
      if (e == hipSuccess) e = launch_phi_edges_padded(n, rows, t.el, t.pad, stream);
    }
    if (e != hipSuccess) {
      t = Table{};
      return hip_fail(e, "coefficient tables (scratch)");
    }
    *out = &t;
    return MLQMC_OK;
  }

  // coefficient tables for mesh n with at least s terms
  mlqmc_status table(int n, int s, Table** out) {
    if (arena) return arena_table(n, s, out);
    Table& t = tables[n];
    if (t.s < s || !t.el) {
      bytes_alloc -= t.bytes;
      t.release();
      // Problem 1: one row per term; Problem 2: the background row and s terms
      const int rows = islands ? s + 1 : std::max(s, 1);
      const size_t be = (size_t)rows * 2 * n * n * 8,
                   bw = islands ? 0 : (size_t)rows * 2 * (n - 1) * n * 8,
                   bp = (size_t)rows * 2 * padded_size(n) * 8,
                   br = islands ? (size_t)rows * 3 * padded_size(n) * 8 : 0;
      const size_t total = be + bw + bp + (islands ? be + br : 0);
      if (mem_cap > 0 && bytes_alloc + (int64_t)total > mem_cap)
        return fail(MLQMC_ENOMEM, "coefficient table for n=%d exceeds the device memory cap", n);
      hipError_t e = hipMalloc(&t.el, be);
      if (e == hipSuccess && bw) e = hipMalloc(&t.edge, bw);
      if (e == hipSuccess) e = hipMalloc(&t.pad, bp);
      if (e == hipSuccess && islands) e = hipMalloc(&t.rel, be);
      if (e == hipSuccess && islands) e = hipMalloc(&t.rpad, br);
      if (e != hipSuccess) {
        t.release();
        return fail(MLQMC_ENOMEM, "table allocation: %s", hipGetErrorString(e));
      }
      t.bytes = (int64_t)total;
      bytes_alloc += t.bytes;
      if (islands) {
        t.s = s;
        e = launch_phi_elements_islands(n, rows, d_c, d_k1, d_k2, d_region, a_in, a_out, t.el,
                                        stream);
        if (e == hipSuccess) e = launch_phi_edges_padded(n, rows, t.el, t.pad, stream);
        if (e == hipSuccess)
          e = launch_phi_elements_islands(n, rows, d_cb, d_k1, d_k2, d_region, b_in, b_out, t.rel,
                                          stream);
        if (e == hipSuccess) e = launch_phi_reaction_padded(n, rows, t.rel, t.rpad, stream);
      } else {
        t.s = rows;
        e = launch_phi_elements(n, rows, d_c, d_k1, d_k2, t.el, stream);
        if (e == hipSuccess) e = launch_phi_edges(n, rows, t.el, t.edge, stream);
        if (e == hipSuccess) e = launch_phi_edges_padded(n, rows, t.el, t.pad, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "coefficient tables");
    }
    *out = &t;
    return MLQMC_OK;
  }

  // timing around launches of the selected class
  bool timed(int cls) const { return timing_class != MLQMC_K_NONE && timing_class == cls; }
  void t_begin(int cls) {
    if (!timed(cls)) return;
    if (ev_used == ev_pool.size()) {
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        timing_class = MLQMC_K_NONE;  // instrumentation only: stop timing, keep computing
        return;
      }
      ev_pool.push_back({a, b});
    }
    if (hipEventRecord(ev_pool[ev_used].first, stream) != hipSuccess) timing_class = MLQMC_K_NONE;
  }
  void t_end(int cls, double bytes, double flops = 0.0) {
    if (!timed(cls)) return;
    if (hipEventRecord(ev_pool[ev_used].second, stream) != hipSuccess) {
      timing_class = MLQMC_K_NONE;
      return;
    }
    ++ev_used;
    ++t_launches;
    t_bytes += bytes;
    t_flops += flops;
  }
  void t_collect() {
    for (size_t k = 0; k < ev_used; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev_pool[k].first, ev_pool[k].second) == hipSuccess) t_ms += ms;
    }
    ev_used = 0;
  }
  mlqmc_status sync(const char* what) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, what);
    t_collect();
    return MLQMC_OK;
  }
};

namespace {

#define CK(expr, what)                        \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return ctx->hip_fail(e_, what); \
  } while (0)
#define CS(expr)                      \
  do {                                \
    mlqmc_status s_ = (expr);         \
    if (s_ != MLQMC_OK) return s_;    \
  } while (0)

// copy n elements in from caller memory to a named device buffer (or alias)
template <typename T>
mlqmc_status stage_in(mlqmc_ctx* ctx, const char* name, const T* src, size_t n, int on_dev,
                      const T** out) {
  if (on_dev) {
    *out = src;
    return MLQMC_OK;
  }
  T* d = nullptr;
  CS(ctx->getT(name, n, &d));
  if (n) CK(hipMemcpyAsync(d, src, n * sizeof(T), hipMemcpyHostToDevice, ctx->stream), "copy in");
  *out = d;
  return MLQMC_OK;
}

template <typename T>
mlqmc_status out_buf(mlqmc_ctx* ctx, const char* name, T* dst, size_t n, int on_dev, T** out) {
  if (on_dev) {
    *out = dst;
    return MLQMC_OK;
  }
  return ctx->getT(name, n, out);
}

template <typename T>
mlqmc_status stage_out(mlqmc_ctx* ctx, T* dst, const T* dev, size_t n, int on_dev) {
  if (on_dev || !dst || n == 0) return MLQMC_OK;
  CK(hipMemcpyAsync(dst, dev, n * sizeof(T), hipMemcpyDeviceToHost, ctx->stream), "copy out");
  return MLQMC_OK;
}

// Two-grid solve stopping tests; 0 selects the precision's default.
// lin_rtol bounds the preconditioned residual, sqrt(r.z / r0.z0).  lam_rtol
// bounds the estimated error of the Rayleigh quotient of v + t_k, which the
// PCG tracks from its own dots: the solve stops as soon as the eigenvalue,
// the quantity returned, is settled.  The defaults leave the eigenvalues a
// factor of at least 10 inside the stated accuracies (FP64 1e-10, mixed 1e-8).
double lin_tol(const mlqmc_opts* o) {
  if (o->lin_rtol > 0) return o->lin_rtol;
  return o->prec == MLQMC_MIXED ? 1e-7 : 1e-10;
}
double lam_tol(const mlqmc_opts* o) {
  if (o->lam_rtol < 0) return 0.0;  // internal: the residual test alone
  if (o->lam_rtol > 0) return o->lam_rtol;
  return o->prec == MLQMC_MIXED ? 5e-10 : 5e-12;
}

mlqmc_status check_opts(mlqmc_ctx* ctx, const mlqmc_opts* o) {
  if (!o) return ctx->fail(MLQMC_EINVAL, "opts is NULL");
  if (o->prec != MLQMC_FP64 && o->prec != MLQMC_MIXED)
    return ctx->fail(MLQMC_EINVAL, "unknown precision %d", o->prec);
  if (!(o->eig_rtol > 0) || !(o->eig_atol >= 0) || !(o->lin_rtol >= 0) || !(o->lam_rtol >= 0) ||
      !(o->rq_lin_rtol > 0))
    return ctx->fail(MLQMC_EINVAL,
                     "tolerances must be positive (eig_atol, lin_rtol, lam_rtol: >= 0)");
  if (o->max_rq_iter < 1 || o->max_lin_iter < 1)
    return ctx->fail(MLQMC_EINVAL, "iteration caps must be >= 1");
  if (o->device_mem_cap < 0) return ctx->fail(MLQMC_EINVAL, "device_mem_cap must be >= 0");
  return MLQMC_OK;
}

// Problem 2 meshes: multiples of 1/8 (the islands' edges are mesh lines) up
// to 1/1024 (every array of a solve in LDS up to 1/32; finer two-grid meshes
// on the batched kernels with the reaction term); 0 = not used
bool islands_mesh_ok(int n) { return n == 0 || (n >= 8 && n <= 1024); }

// Problem 2 takes meshes finer than 1/32 only as a two-grid fine or previous
// mesh (the eigensolves stay at 1/32 or coarser)
mlqmc_status check_islands_level(mlqmc_ctx* ctx, const mlqmc_level* l) {
  if (!ctx->islands) return MLQMC_OK;
  if (l->n_coarse == 0 && (l->n_fine > 32 || l->n_prev > 32))
    return ctx->fail(MLQMC_EINVAL, "islands direct levels need meshes up to 1/32");
  if (l->n_coarse > 32)
    return ctx->fail(MLQMC_EINVAL, "islands coarse meshes go up to 1/32");
  return MLQMC_OK;
}

mlqmc_status check_level(mlqmc_ctx* ctx, const mlqmc_level* l) {
  if (!l) return ctx->fail(MLQMC_EINVAL, "level is NULL");
  if (!is_pow2(l->n_fine)) return ctx->fail(MLQMC_EINVAL, "n_fine=%d is not a power of two", l->n_fine);
  if (l->s_fine < 0 || l->s_fine > ctx->s_max)
    return ctx->fail(MLQMC_EINVAL, "s_fine=%d outside [0, s_max=%d]", l->s_fine, ctx->s_max);
  if (l->s_fine > 512) return ctx->fail(MLQMC_EINVAL, "s_fine=%d exceeds 512", l->s_fine);
  if (l->n_coarse == 0) {
    if (l->n_fine < 4 || l->n_fine > 64)
      return ctx->fail(MLQMC_EINVAL, "direct levels need 4 <= n_fine <= 64 (got %d)", l->n_fine);
  } else {
    if (!is_pow2(l->n_coarse) || l->n_coarse < 4 || l->n_coarse > 64)
      return ctx->fail(MLQMC_EINVAL, "n_coarse=%d must be a power of two in [4, 64]", l->n_coarse);
    if (l->n_fine <= l->n_coarse || l->n_fine > 1024)
      return ctx->fail(MLQMC_EINVAL, "need n_coarse < n_fine <= 1024 (got %d, %d)", l->n_coarse,
                       l->n_fine);
    if (l->s_coarse < 0 || l->s_coarse > l->s_fine)
      return ctx->fail(MLQMC_EINVAL, "s_coarse=%d outside [0, s_fine]", l->s_coarse);
  }
  if (l->n_prev != 0) {
    if (!is_pow2(l->n_prev)) return ctx->fail(MLQMC_EINVAL, "n_prev=%d is not a power of two", l->n_prev);
    if (l->s_prev < 0 || l->s_prev > l->s_fine)
      return ctx->fail(MLQMC_EINVAL, "s_prev=%d outside [0, s_fine]", l->s_prev);
    if (l->n_coarse == 0) {
      if (l->n_prev < 4 || l->n_prev > 64)
        return ctx->fail(MLQMC_EINVAL, "direct previous level needs 4 <= n_prev <= 64");
    } else if (l->n_prev < l->n_coarse || l->n_prev > 1024) {
      return ctx->fail(MLQMC_EINVAL, "need n_coarse <= n_prev <= 1024 (got %d)", l->n_prev);
    }
  }
  if (ctx->islands &&
      !(islands_mesh_ok(l->n_fine) && islands_mesh_ok(l->n_coarse) && islands_mesh_ok(l->n_prev)))
    return ctx->fail(MLQMC_EINVAL,
                     "the islands family (Problem 2) needs meshes 1/8 .. 1/1024 (got %d, %d, %d)",
                     l->n_fine, l->n_coarse, l->n_prev);
  return MLQMC_OK;
}

// Samples per warm-start chain of the eigensolve on mesh N: as short as keeps
// every workgroup slot of the device busy (one chain per workgroup).
// The occupancy is cached in the context (a context is used by one host
// thread at a time), per (mesh, precision), for the context's family.
int default_chain(mlqmc_ctx* ctx, int64_t n, int warm, int chain_len, int N, int mixed) {
  if (!warm) return 1;
  if (chain_len > 0) return chain_len;
  auto it = ctx->chain_slots.find({N, mixed});
  if (it == ctx->chain_slots.end()) {
    const int c = rqi_chains_in_flight(N, mixed, ctx->islands ? 1 : 0);
    it = ctx->chain_slots.emplace(std::make_pair(N, mixed), c > 0 ? c : 512).first;
  }
  const int64_t target = it->second;
  const int64_t c = (n + target - 1) / target;
  return (int)std::max<int64_t>(1, c);
}

// Everything a captured PCG iteration bakes into its kernel arguments.
template <typename T, typename V>
std::vector<uint64_t> graph_key(int nh, int64_t Bn, const mlqmc_opts* o, const FineState& S,
                                std::initializer_list<const void*> ptrs, const V& W, const V& X,
                                const V& Xb, const V& Bv, int nblk0, int nblk_post) {
  std::vector<uint64_t> k = {(uint64_t)nh, (uint64_t)Bn, sizeof(T), (uint64_t)nblk0,
                             (uint64_t)nblk_post, (uint64_t)o->max_lin_iter};
  double tl[2] = {lin_tol(o), lam_tol(o)};
  uint64_t bits[2];
  std::memcpy(bits, tl, sizeof bits);
  k.push_back(bits[0]);
  k.push_back(bits[1]);
  for (const void* p : ptrs) k.push_back((uint64_t)(uintptr_t)p);
  const void* sp[] = {S.mu, S.vs, S.rho, S.rz, S.rz0, S.alpha, S.c, S.c2, S.beta, S.lam, S.f,
                      S.m, S.dmp, S.rzp, S.g, S.its, S.lin_acc, S.active, S.vact, S.flags};
  for (const void* p : sp) k.push_back((uint64_t)(uintptr_t)p);
  for (const V* v : {&W, &X, &Xb, &Bv})
    for (auto* p : *v) k.push_back((uint64_t)(uintptr_t)p);
  return k;
}

// The instantiated graph of `body` (launches on the stream it is given) for
// this tag and key: reused while the key matches, captured on the context's
// private stream otherwise.
template <typename F>
mlqmc_status pcg_graph(mlqmc_ctx* ctx, const char* tag, int64_t, F body,
                       const std::vector<uint64_t>& key, hipGraphExec_t* out) {
  mlqmc_ctx::PcgGraph& g = ctx->graphs[tag];
  if (g.exec && g.key == key) {
    *out = g.exec;
    return MLQMC_OK;
  }
  if (g.exec) {
    CK(hipGraphExecDestroy(g.exec), "graph destroy");
    g.exec = nullptr;
  }
  if (!ctx->cap_stream) CK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking),
                           "capture stream");
  CK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  const mlqmc_status st = body(ctx->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
  if (st != MLQMC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  CK(e, "end capture");
  const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  CK(ei, "graph instantiate");
  g.key = key;
  *out = g.exec;
  return MLQMC_OK;
}

// Two-grid update on mesh nh (>= 64) for n samples, batched.  T is the
// storage type of the projected PCG and the V-cycle (double; float in mixed
// precision); the right-hand side and the Rayleigh quotient are FP64.
// Problem 2 (ctx->islands): weight blocks [WX | WY | RX | RY | RD] from the
// two coefficient products of the diffusion and reaction tables (their row 0
// the background values, selected by a leading 1 in the point), and the
// operator A + R in every kernel.
template <typename T>
mlqmc_status fine_batched(mlqmc_ctx* ctx, const mlqmc_opts* o, int nh, int s, const double* Y,
                          int64_t ldY, const double* uH, const double* lamH, int nH, int64_t n,
                          double* lam, double* g, int* lin_iters, uint8_t* flags,
                          const char* tag) {
  constexpr bool kMixed = std::is_same<T, float>::value;
  const int rx = ctx->islands ? 1 : 0;   // reaction term
  const int WB = rx ? 5 : 2;             // weight arrays per sample
  Table* tb = nullptr;
  CS(ctx->table(nh, s, &tb));
  std::vector<int> lv;
  for (int m = nh; m > 32; m /= 2) lv.push_back(m);
  const int nb = 32;
  const size_t nL = lv.size();
  auto D = [](int m) { return (int64_t)(m - 1) * (m - 1); };  // interior nodes (coarse uH)
  auto P = [](int m) { return padded_size(m); };                // padded vector
  auto EW = [WB](int m) { return WB * padded_size(m); };        // padded weight block
  const int64_t sz = (int64_t)sizeof(T);
  int64_t per_sample = sz * EW(nh) + 8 * 2 * P(nh) + sz * (9 * P(nh));
  for (size_t k = 1; k < nL; ++k) per_sample += sz * (EW(lv[k]) + 3 * P(lv[k]));
  per_sample += sz * (EW(nb) + 2 * P(nb));
  if (rx) per_sample += 8 * (s + 1);  // the points with their leading 1
  mlqmc_ctx::SepTable* sep = nullptr;  // the separable expansion, when cheaper
  CS(ctx->sep_table(nh, s, &sep));
  if (sep) per_sample += 8 * (3 * nh + 2) * sep->kx;  // its row sums U
  // default batch: up to 96 GB of working arrays (a third of the 288 GB of
  // HBM), in multiples of the 128-sample tile of the coefficient product when
  // larger, and the samples split evenly over the batches that takes (no
  // small last batch).  On the h = 1/1024 workload 768 samples per batch ran
  // 8 % faster than 384 (fewer batch set-ups and PCG tails, half the strips'
  // halo rows); 1152 no faster.
  int64_t batch = o->batch;
  if (batch <= 0) {
    int64_t cap = std::max<int64_t>(1, (int64_t)96e9 / per_sample);
    if (cap > 128) cap -= cap % 128;
    const int64_t nb = (n + cap - 1) / cap;
    batch = (n + nb - 1) / nb;
    if (batch > 128) batch = std::min(cap, (batch + 127) / 128 * 128);
  }
  batch = std::min<int64_t>(batch, n);
  // partial-sum counts depend on the batch size through the strip choice;
  // the partial buffer is sized for the largest (smallest batch)

  std::string p = tag;
  auto nm = [&](const char* x) { return p + x; };
  // The edge weights are stored once, in the storage precision: the FP64
  // set-up residual and Rayleigh quotients read them there too and compute in
  // FP64.  In mixed precision that puts an FP32 rounding into every weight of
  // the operator whose eigenvalue is returned; the roundings are independent,
  // so the eigenvalue moves by about 1e-10 relative (measured with the oracle
  // on 1/256: 4e-11 .. 1.4e-10), far inside the 1e-8 the mixed path promises.
  double *part, *Y1 = nullptr, *sepU = nullptr;
  T *wT, *vn, *mvn, *t, *r, *r2, *z, *zb, *pp[2];
  CS(ctx->getT(nm(kMixed ? "w32" : "w64").c_str(), batch * EW(nh), &wT));
  double* w64 = nullptr;  // the weights when stored in FP64
  float* w32 = nullptr;   // ... in FP32
  if constexpr (kMixed)
    w32 = wT;
  else
    w64 = wT;
  if (rx) CS(ctx->getT(nm("Y1").c_str(), batch * (s + 1), &Y1));
  if (sep) CS(ctx->getT(nm("sepU").c_str(), batch * (3 * nh + 2) * sep->kx, &sepU));
  double* sep_tri_t = nullptr;  // interval sums for the coarse-side set-up products
  if (sep) CS(ctx->sep_tri(sep, nh, nH, &sep_tri_t));
  // blocks per sample <= (rows + 7) / 8 strips x (column blocks <= 4): bound the
  // partial-sum buffer by the most strips any batch size can take, 3 partials each
  CS(ctx->getT(nm("part").c_str(), batch * (4 * ((nh + 6) / 8) + 4) * 6, &part));
  const char* vnames[] = {"vn", "t", "r", "z", "zb", "p0", "p1", "mvn", "r2"};
  T** vptr[] = {&vn, &t, &r, &z, &zb, &pp[0], &pp[1], &mvn, &r2};
  for (int k = 0; k < 9; ++k) {
    std::string key = nm(vnames[k]) + (kMixed ? "_f" : "_d");
    CS(ctx->getT(key.c_str(), batch * P(nh), vptr[k]));
  }
  std::vector<T*> W(nL + 1), X(nL + 1), Xb(nL + 1), Bv(nL + 1);
  W[0] = wT;
  for (size_t k = 1; k <= nL; ++k) {
    const int m = (k < nL) ? lv[k] : nb;
    char b1[64];
    const char* sfx = kMixed ? "f" : "d";
    snprintf(b1, sizeof b1, "w%zu%s", k, sfx);
    CS(ctx->getT(nm(b1).c_str(), batch * EW(m), &W[k]));
    snprintf(b1, sizeof b1, "X%zu%s", k, sfx);
    CS(ctx->getT(nm(b1).c_str(), batch * P(m), &X[k]));
    snprintf(b1, sizeof b1, "B%zu%s", k, sfx);
    CS(ctx->getT(nm(b1).c_str(), batch * P(m), &Bv[k]));
    if (k < nL) {
      snprintf(b1, sizeof b1, "Xb%zu%s", k, sfx);
      CS(ctx->getT(nm(b1).c_str(), batch * P(m), &Xb[k]));
    }
  }
  // Dirichlet positions of every padded vector are zero and stay zero: the
  // kernels write interior positions only.
  {
    hipStream_t st = ctx->stream;
    auto zero = [&](int m, std::initializer_list<void*> ptrs, int elem) -> mlqmc_status {
      std::vector<void*> todo;
      for (void* q : ptrs)
        if (!ctx->boundary_is_zero(q, m, elem, batch)) todo.push_back(q);
      if (todo.empty()) return MLQMC_OK;
      CK(launch_zero_boundary(m, batch, todo.data(), (int)todo.size(), elem, st), "zero boundary");
      for (void* q : todo) ctx->zeroed[q] = mlqmc_ctx::ZeroKey{m, elem, batch};
      return MLQMC_OK;
    };
    CS(zero(nh, {vn, t, r, z, zb, pp[0], pp[1], mvn, r2}, (int)sz));
    for (size_t k = 1; k <= nL; ++k) {
      const int m = (k < nL) ? lv[k] : nb;
      if (k < nL)
        CS(zero(m, {X[k], Bv[k], Xb[k]}, (int)sz));
      else
        CS(zero(m, {X[k], Bv[k]}, (int)sz));
    }
  }
  double* sc = nullptr;
  CS(ctx->getT(nm("scal").c_str(), batch * 12, &sc));
  int* its = nullptr;
  CS(ctx->getT(nm("its").c_str(), batch, &its));
  uint8_t *active = nullptr, *vact = nullptr;
  CS(ctx->getT(nm("active").c_str(), batch, &active));
  CS(ctx->getT(nm("vact").c_str(), batch, &vact));
  std::vector<uint8_t> h_active(batch);
  std::vector<int> h_its(batch);

  set_target_blocks(ctx->target_for(nh, kMixed ? MLQMC_MIXED : MLQMC_FP64));
  for (int64_t b0 = 0; b0 < n; b0 += batch) {
    const int64_t Bn = std::min<int64_t>(batch, n - b0);
    const int nblk0 = march_blocks(nh, Bn);
    FineState S{};
    S.mu = const_cast<double*>(lamH) + b0;
    S.vs = sc;
    S.rho = sc + batch;
    S.rz = sc + 2 * batch;
    S.rz0 = sc + 3 * batch;
    S.alpha = sc + 4 * batch;
    S.c = sc + 5 * batch;
    S.c2 = sc + 6 * batch;
    S.beta = sc + 7 * batch;
    S.f = sc + 8 * batch;
    S.m = sc + 9 * batch;
    S.dmp = sc + 10 * batch;
    S.rzp = sc + 11 * batch;
    S.lam = lam + b0;
    S.g = g ? g + b0 : nullptr;
    S.its = its;
    S.lin_acc = lin_iters ? lin_iters + b0 : nullptr;
    S.active = active;
    S.vact = vact;
    S.flags = flags + b0;
    hipStream_t st = ctx->stream;
    const uint8_t* act = vact;  // the V-cycle skips samples whose last step is taken

    // coefficient expansion straight into the edge weights (computed in FP64,
    // stored in the storage precision), then the coarser levels
    ctx->t_begin(MLQMC_K_COEFF);
    if (rx) {
      // (1, y) against the tables of a and b (row 0: the background values)
      CK(launch_prepend_one(Bn, s, Y + b0 * ldY, ldY, Y1, st), "points");
      CK(launch_expand(Bn, s + 1, 2 * P(nh), Y1, s + 1, tb->pad, 0.0, w64, w32, st, EW(nh)),
         "expand");
      CK(launch_expand(Bn, s + 1, 3 * P(nh), Y1, s + 1, tb->rpad, 0.0,
                       w64 ? w64 + 2 * P(nh) : nullptr, w32 ? w32 + 2 * P(nh) : nullptr, st,
                       EW(nh)),
         "expand");
    } else if (sep) {
      CK(launch_expand_separable(Bn, nh, s, sep->kx, sep->ky, Y + b0 * ldY, ldY, ctx->d_c,
                                 sep->cell_start, sep->cell_term, sep->S, sepU, ctx->a0, w64, w32,
                                 EW(nh), st),
         "expand (separable)");
    } else {
      CK(launch_expand(Bn, s, EW(nh), Y + b0 * ldY, ldY, tb->pad, ctx->a0, w64, w32, st),
         "expand");
    }
    // the weights out in the storage precision; in: Y and the table (dense),
    // or Y and the row sums U (separable: written and read once); flops of
    // the product actually formed
    const int rows = rx ? s + 1 : s;
    const double wout = (double)sz * (double)Bn * EW(nh);
    if (sep) {
      // U: 3 n + 2 rows stored, 2 n + 1 of them (the element centroids) formed
      const double M3 = 3.0 * nh + 2.0, Mc = 2.0 * nh + 1.0;
      ctx->t_end(MLQMC_K_COEFF, 8.0 * (double)Bn * s + 16.0 * (double)Bn * M3 * sep->kx + wout,
                 (double)Bn * (4.0 * sep->kx * P(nh) + 2.0 * Mc * sep->kx * sep->ky));
    } else {
      ctx->t_end(MLQMC_K_COEFF, 8.0 * ((double)Bn * rows + (double)rows * EW(nh)) + wout,
                 2.0 * rows * (double)EW(nh) * Bn);
    }
    for (size_t k = 0; k < nL; ++k)
      CK(launch_coarsen<T>(lv[k], Bn, W[k], W[k + 1], rx, st), "coarsen");

    // v = P u_H is evaluated inside these kernels from the coarse vectors.
    // With the separable expansion v^T M v and v^T A v come from coarse
    // quantities and the expansion's row sums instead of a pass over the fine
    // edge weights (the coefficient at the fine centroids, summed per coarse
    // triangle).
    const double* uHb = uH + b0 * D(nH);
    if (sep_tri_t) {
      CK(launch_sep_setup_dots(Bn, nh, nH, sep->kx, sepU, sep_tri_t, uHb, ctx->a0, part, st),
         "setup dots (separable)");
      CK(launch_scalar(PH_SETUP, nh, Bn, 1, part, S, 0.0, 0, st), "scalar");
    } else {
      CK(launch_setup_dots<T>(nh, Bn, uHb, nH, wT, part, rx, st), "setup dots");
      CK(launch_scalar(PH_SETUP, nh, Bn, nblk0, part, S, 0.0, 0, st), "scalar");
    }
    CK(launch_setup_rhs<T>(nh, Bn, uHb, nH, wT, S, r, vn, mvn, rx, st), "setup rhs");

    // z = K^{-1} r by one V-cycle: fused pre-smoothing + restriction per level,
    // the LDS bottom solve, fused coarse correction + post-smoothing per level;
    // the level-0 post-smoothing also forms the partials r.z, M vn.z, r.vn.
    // The result alternates between the two level-0 buffers (the post kernel
    // cannot write in place).  Timed launches are those in which every sample is
    // active (the set-up V-cycle, the first PCG step), so the byte model counts
    // exactly the work done: rhs, 2 edge weights per node in; X and rhs_c out.
    // (with the reaction three more weight arrays per node in every stencil kernel)
    const double pre_b = (double)sz * Bn * ((4.25 + 3 * rx) * D(nh));
    // post: Xin, rhs, mvn, 2 weights per node and 1/4 of a coarse vector in (and vn
    // for the product r.vn in FP32 storage only); Xout out
    const double post_b = (double)sz * Bn * ((kMixed ? 7.25 : 6.25) + 3 * rx) * D(nh);
    bool all_active = true;
    int cur = 0;  // pp[cur]: the current search direction
    T* zc = z;   // current preconditioned residual
    T* zo = zb;  // the other buffer
    T* rc = r;   // current residual
    T* ro = r2;  // the other buffer
    // upd: bring the residual up to date first, r <- r - alpha (q - c M vn),
    // inside the finest pre-smoothing kernel, which recomputes q = (A - mu M) p
    // from the current direction (the result lands in ro)
    auto vcycle = [&](bool upd) -> mlqmc_status {
      if (all_active) ctx->t_begin(MLQMC_K_PRE);
      if (upd) {
        CK(launch_pre<T>(nh, Bn, wT, rc, zc, Bv[1], act, pp[cur], mvn, &S, ro, rx, st), "pre");
        std::swap(rc, ro);
      } else {
        CK(launch_pre<T>(nh, Bn, wT, rc, zc, Bv[1], act, nullptr, nullptr, nullptr, nullptr, rx,
                         st),
           "pre");
      }
      if (all_active) ctx->t_end(MLQMC_K_PRE, pre_b);
      for (size_t k = 1; k < nL; ++k)
        CK(launch_pre<T>(lv[k], Bn, W[k], Bv[k], X[k], Bv[k + 1], act, nullptr, nullptr, nullptr,
                         nullptr, rx, st),
           "pre");
      CK(launch_bottom_vcycle<T>(nb, Bn, W[nL], Bv[nL], X[nL], act, rx, st), "bottom");
      const T* xc = X[nL];
      for (size_t k = nL - 1; k >= 1; --k) {
        CK(launch_post<T>(lv[k], Bn, W[k], Bv[k], X[k], xc, Xb[k], nullptr, nullptr, act, nullptr,
                          rx, st),
           "post");
        xc = Xb[k];
      }
      if (all_active) ctx->t_begin(MLQMC_K_SMOOTH);
      CK(launch_post<T>(nh, Bn, wT, rc, zc, xc, zo, vn, mvn, act, part, rx, st), "post");
      if (all_active) ctx->t_end(MLQMC_K_SMOOTH, post_b);
      std::swap(zc, zo);
      return MLQMC_OK;
    };
    CS(vcycle(false));
    all_active = false;
    const int nblk_post = post_strips(nh, Bn);
    CK(launch_scalar(PH_FIRST_RZ, nh, Bn, nblk_post, part, S, 0.0, 0, st), "scalar");
    // first apply: z, vn, 2 weights per node in (M vn is formed from vn; no
    // previous p; t = 0 not read); p out (q feeds only the partial sums)
    const double ab = (double)sz * Bn * ((5 + 3 * rx) * D(nh));
    // one PCG iteration: apply (with the previous step's t update), alpha and
    // the eigenvalue test, the V-cycle (with the residual update), beta
    auto iteration = [&](int it) -> mlqmc_status {
      if (it == 0) ctx->t_begin(MLQMC_K_APPLY);
      CK(launch_pupdate_apply<T>(nh, Bn, zc, vn, pp[cur], wT, t, S, it == 0, pp[1 - cur],
                                 nullptr, part, rx, st),
         "apply");
      if (it == 0) ctx->t_end(MLQMC_K_APPLY, ab);
      cur = 1 - cur;
      CK(launch_scalar(PH_ALPHA, nh, Bn, nblk0, part, S, lam_tol(o), 0, st), "scalar");
      // t += alpha p happens in the next apply (or the final dots)
      CS(vcycle(true));
      CK(launch_scalar(PH_BETA, nh, Bn, nblk_post, part, S, lin_tol(o), o->max_lin_iter, st),
         "scalar");
      return MLQMC_OK;
    };
    // any sample still active; with `steps` also the most PCG steps any
    // sample has taken
    auto any_active = [&](bool* any, int* steps = nullptr) -> mlqmc_status {
      CK(hipMemcpyAsync(h_active.data(), active, Bn, hipMemcpyDeviceToHost, st), "active");
      if (steps)
        CK(hipMemcpyAsync(h_its.data(), its, Bn * sizeof(int), hipMemcpyDeviceToHost, st),
           "steps");
      CS(ctx->sync("pcg"));
      *any = false;
      for (int64_t k = 0; k < Bn; ++k) *any |= h_active[k] != 0;
      if (steps) {
        *steps = 0;
        for (int64_t k = 0; k < Bn; ++k) *steps = std::max(*steps, h_its[k]);
      }
      return MLQMC_OK;
    };
    CS(iteration(0));
    int done_its = 1;
    if (o->pcg_graph) {
      // Iterations 1, 2, ... replayed two at a time from a captured graph: two
      // iterations bring every alternating buffer back to its parity, so one
      // graph serves every replay.  Samples that have converged exit at once.
      hipGraphExec_t exec = nullptr;
      const std::string gtag = std::string(tag) + std::to_string(b0);
      CS(pcg_graph(ctx, gtag.c_str(), Bn, [&](hipStream_t cs) -> mlqmc_status {
        const hipStream_t keep = st;
        st = cs;
        mlqmc_status r = iteration(1);
        if (r == MLQMC_OK) r = iteration(2);
        st = keep;
        return r;
      }, graph_key<T>(nh, Bn, o, S, {zc, zo, rc, ro, pp[0], pp[1], vn, mvn, wT, t, part, act,
                                     active, uHb, (const void*)(uintptr_t)nH},
                      W, X, Xb, Bv, nblk0, nblk_post), &exec));
      // Replays before the first read-back of the activity: as many as this
      // batch needed the last time it ran (converged samples exit at once, so
      // a replay too many costs only its empty launches), then one at a time.
      mlqmc_ctx::PcgGraph& pg = ctx->graphs[gtag];
      const int ahead = std::max(1, pg.pairs);
      int pairs = 0;
      while (done_its < o->max_lin_iter) {
        CK(hipGraphLaunch(exec, st), "graph launch");
        done_its += 2;
        if (++pairs < ahead && done_its < o->max_lin_iter) continue;
        bool any = false;
        int steps = 0;
        CS(any_active(&any, &steps));
        if (!any) {
          pg.pairs = steps / 2;  // steps 1 .. steps - 1 in replays of two
          break;
        }
      }
    } else {
      for (int it = 1; it < o->max_lin_iter; ++it) {
        CS(iteration(it));
        done_its = it + 1;
        if (it % 3 == 2 || it + 1 == o->max_lin_iter) {
          bool any = false;
          CS(any_active(&any));
          if (!any) break;
        }
      }
    }
    // The Rayleigh quotient of w = v_n + t.  The PCG tracks it step by step,
    // mu + f / m with f = w^T (A - mu M) w and m = w^T M w updated from the
    // step's own FP64 dot products; with FP64 storage that is the quotient of
    // the returned w up to the rounding of a few dot products, so no pass over
    // the fine vectors is needed.  In FP32 storage the tracked products carry
    // FP32 errors, and G needs the sum of w: there the final kernel forms
    // w^T A w and w^T M w in FP64 from the stored vectors.
    if (!kMixed && !g) {
      CK(launch_scalar(PH_FINAL_TRACKED, nh, Bn, 0, part, S, 0.0, 0, st), "scalar");
    } else {
      CK(launch_final_dots<T>(nh, Bn, uHb, nH, t, pp[0], pp[1], wT, S, part, rx, st),
         "final dots");
      CK(launch_scalar(PH_FINAL, nh, Bn, nblk0, part, S, 0.0, 0, st), "scalar");
    }
  }
  return MLQMC_OK;
}

// Two-grid update on mesh nh from the coarse pairs (uH on mesh nH, lamH).
mlqmc_status fine_update(mlqmc_ctx* ctx, const mlqmc_opts* o, int nh, int s, const double* Y,
                         int64_t ldY, const double* uH, const double* lamH, int nH, int64_t n,
                         double* lam, double* g, int* lin_iters, uint8_t* flags,
                         const char* tag) {
  // G is linear in the eigenvector, whose error is only the square root of
  // the eigenvalue's: with G requested the solve runs to the residual test
  mlqmc_opts og = *o;
  if (g) og.lam_rtol = -1.0;
  o = &og;
  if (nh <= 32) {
    Table* tb = nullptr;
    CS(ctx->table(nh, s, &tb));
    TgSmallArgs a{};
    a.Y = Y;
    a.ldY = ldY;
    a.s = s;
    a.phi = tb->pad;
    a.a0 = ctx->a0;
    a.rphi = tb->rpad;
    a.uH = uH;
    a.lamH = lamH;
    a.nH = nH;
    a.n = n;
    a.lin_rtol = lin_tol(o);
    a.lam_rtol = lam_tol(o);
    a.mixed = o->prec == MLQMC_MIXED ? 1 : 0;
    a.max_lin = o->max_lin_iter;
    a.lam = lam;
    a.g = g;
    a.lin_iters = lin_iters;
    a.flags = flags;
    ctx->t_begin(MLQMC_K_TG_LDS);
    CK(launch_tg_small(nh, a, ctx->stream), "two-grid (LDS)");
    ctx->t_end(MLQMC_K_TG_LDS, 0.0);
    return MLQMC_OK;
  }
  if (o->prec == MLQMC_MIXED)
    return fine_batched<float>(ctx, o, nh, s, Y, ldY, uH, lamH, nH, n, lam, g, lin_iters, flags,
                               tag);
  return fine_batched<double>(ctx, o, nh, s, Y, ldY, uH, lamH, nH, n, lam, g, lin_iters, flags,
                              tag);
}

// Arguments of the warm-started RQ eigensolve shared by every caller.
RqiArgs rqi_base(mlqmc_ctx* ctx, const mlqmc_opts* o, int64_t n, const double* Y, int64_t ldY,
                 int chain, int warm, int* rq_iters, int* lin_iters, uint8_t* flags) {
  RqiArgs a{};
  a.Y = Y;
  a.ldY = ldY;
  a.a0 = ctx->a0;
  a.n = n;
  a.chain_len = chain;
  a.warm = warm;
  a.eig_rtol = o->eig_rtol;
  a.eig_atol = o->eig_atol;
  a.max_rq = o->max_rq_iter;
  a.lin_rtol = o->rq_lin_rtol;
  a.max_lin = o->max_lin_iter;
  a.rq_iters = rq_iters;
  a.lin_iters = lin_iters;
  a.flags = flags;
  a.mixed = o->prec == MLQMC_MIXED ? 1 : 0;
  // the refinement step of a vector G is taken from: FP64 only (an FP32
  // correction solve cannot improve an FP32 vector, its right-hand side is
  // rounding noise)
  a.g_lin_rtol = a.mixed ? 0.0 : lin_tol(o);
  return a;
}

// Chain length for R shifts of N points each: a power of two dividing N, so
// no warm-start chain crosses from one shift to the next.
int shift_chain(mlqmc_ctx* ctx, int64_t N, int R, const mlqmc_opts* o, int mesh) {
  const int chain =
      default_chain(ctx, N * R, 1, o->chain_len, mesh, o->prec == MLQMC_MIXED ? 1 : 0);
  int c2 = 1;
  while (c2 < chain) c2 *= 2;
  return (int)std::min<int64_t>(c2, N);
}

// Whole level on device buffers (Y [n x ldY] on device); outputs on device.
// g, g_prev (nullable): G(u^l), G(u^{l-1}) of the normalised, sign-fixed
// eigenvector approximations.
mlqmc_status level_core(mlqmc_ctx* ctx, const mlqmc_level* L, const mlqmc_opts* o, int64_t n,
                        const double* Y, int64_t ldY, int warm, double* lam, double* lam_prev,
                        double* lam_coarse, int* rq_iters, int* lin_iters, uint8_t* flags,
                        double* g = nullptr, double* g_prev = nullptr,
                        const std::string& pfx = std::string()) {
  // named scratch of this call (a prefix keeps levels that run at the same
  // time on different streams apart)
  auto nm = [&](const char* x) { return pfx + x; };
  hipStream_t st = ctx->stream;
  if (n == 0) return MLQMC_OK;
  CK(hipMemsetAsync(flags, 0, n, st), "memset");
  CK(hipMemsetAsync(lin_iters, 0, n * sizeof(int), st), "memset");
  const int mixed = o->prec == MLQMC_MIXED ? 1 : 0;
  const int chain =
      default_chain(ctx, n, warm, o->chain_len, L->n_coarse ? L->n_coarse : L->n_fine, mixed);
  RqiArgs a = rqi_base(ctx, o, n, Y, ldY, chain, warm, rq_iters, lin_iters, flags);
  if (L->n_coarse == 0) {
    Table* tb = nullptr;
    CS(ctx->table(L->n_fine, L->s_fine, &tb));
    a.S = L->s_fine;
    a.phi = tb->pad;
    a.rphi = tb->rpad;
    a.lam = lam;
    a.u_out = nullptr;
    a.g_out = g;
    // 1/64: each chain's top level in a slice of global scratch (FP64)
    auto scratch_for = [&](int mesh, RqiArgs& ra) -> mlqmc_status {
      if (const int64_t per = rqi_scratch_doubles(mesh)) {
        ra.scratch_doubles = per * ((n + chain - 1) / chain);
        CS(ctx->getT(nm("rqi_scratch").c_str(), ra.scratch_doubles, &ra.scratch));
      }
      return MLQMC_OK;
    };
    CS(scratch_for(L->n_fine, a));
    ctx->t_begin(MLQMC_K_COARSE);
    CK(launch_rqi(L->n_fine, a, st), "eigensolve (LDS)");
    ctx->t_end(MLQMC_K_COARSE, 0.0);
    if (lam_coarse) {
      std::vector<double> nans(n, NAN);
      CK(hipMemcpyAsync(lam_coarse, nans.data(), n * sizeof(double), hipMemcpyHostToDevice, st),
         "nan fill");
      CS(ctx->sync("nan fill"));
    }
    if (L->n_prev && lam_prev) {
      uint8_t* f2 = nullptr;
      int* i2 = nullptr;
      CS(ctx->getT(nm("flags_prev").c_str(), n, &f2));
      CS(ctx->getT(nm("rq_prev").c_str(), n, &i2));
      CS(ctx->table(L->n_prev, L->s_prev, &tb));
      RqiArgs b = a;
      b.S = L->s_prev;
      b.phi = tb->pad;
      b.rphi = tb->rpad;
      b.lam = lam_prev;
      b.rq_iters = i2;
      b.lin_iters = nullptr;
      b.flags = f2;
      b.g_out = g_prev;
      b.scratch = nullptr;
      b.scratch_doubles = 0;
      CS(scratch_for(L->n_prev, b));
      ctx->t_begin(MLQMC_K_COARSE);
      CK(launch_rqi(L->n_prev, b, st), "eigensolve (LDS)");
      ctx->t_end(MLQMC_K_COARSE, 0.0);
      // the previous-level eigensolve's flags join the level's (on the device:
      // no host round trip)
      CK(launch_or_flags(n, flags, f2, st), "flags");
    }
    return MLQMC_OK;
  }
  // coarse pairs
  Table* tb = nullptr;
  CS(ctx->table(L->n_coarse, L->s_coarse, &tb));
  const int64_t DH = (int64_t)(L->n_coarse - 1) * (L->n_coarse - 1);
  double *uH = nullptr, *lamH = lam_coarse;
  CS(ctx->getT(nm("uH").c_str(), n * DH, &uH));
  if (!lamH) CS(ctx->getT(nm("lamH").c_str(), n, &lamH));
  a.S = L->s_coarse;
  a.phi = tb->pad;
  a.rphi = tb->rpad;
  a.lam = lamH;
  a.u_out = uH;
  const bool degenerate = L->n_prev == L->n_coarse && L->s_prev == L->s_coarse;
  // on the degenerate previous mesh the update's eigenvector is u_H itself
  a.g_out = (L->n_prev && lam_prev && degenerate) ? g_prev : nullptr;
  // The two-grid value is not stationary in u_H: an error e in the coarse
  // vector moves it by about |lambda_H - lambda_h| |e| (the Rayleigh quotient
  // of w is stationary only at the fine eigenvector).  The RQ iteration's
  // vectors carry e ~ 1e-7 or less on Problem 1 (two-grid values within 1e-11
  // of the oracle), not on Problem 2, where the one-step refinement brings
  // them to the linear tolerance; the fine updates' G inherit e linearly too.
  a.refine = (ctx->islands || g || (L->n_prev && g_prev)) ? 1 : 0;
  if (const int64_t per = rqi_scratch_doubles(L->n_coarse)) {
    a.scratch_doubles = per * ((n + chain - 1) / chain);
    CS(ctx->getT(nm("rqi_scratch").c_str(), a.scratch_doubles, &a.scratch));
  }
  ctx->t_begin(MLQMC_K_COARSE);
  CK(launch_rqi(L->n_coarse, a, st), "coarse eigensolve (LDS)");
  ctx->t_end(MLQMC_K_COARSE, 0.0);
  CS(fine_update(ctx, o, L->n_fine, L->s_fine, Y, ldY, uH, lamH, L->n_coarse, n, lam, g,
                 lin_iters, flags, "f_"));
  if (L->n_prev && lam_prev) {
    if (degenerate) {
      // (A - lambda_H M) is singular on the coarse space itself: its update is lambda_H
      CK(hipMemcpyAsync(lam_prev, lamH, n * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
    } else {
      CS(fine_update(ctx, o, L->n_prev, L->s_prev, Y, ldY, uH, lamH, L->n_coarse, n, lam_prev,
                     g_prev, lin_iters, flags, "p_"));
    }
  }
  return MLQMC_OK;
}

mlqmc_status any_flag(mlqmc_ctx* ctx, const uint8_t* flags_dev, int64_t n, bool* any) {
  std::vector<uint8_t> h(n);
  if (n) CK(hipMemcpyAsync(h.data(), flags_dev, n, hipMemcpyDeviceToHost, ctx->stream), "flags");
  CS(ctx->sync("flags"));
  *any = false;
  for (int64_t k = 0; k < n; ++k) *any |= h[k] != 0;
  return MLQMC_OK;
}

bool finite_host(const double* x, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(x[k])) return false;
  return true;
}

}  // namespace

namespace {
// checks that `device` exists and makes it current (context creation)
mlqmc_status bind_new_device(int device) {
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev) {
    g_create_error = std::string("no HIP device ") + std::to_string(device) +
                     (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
    return MLQMC_EDEVICE;
  }
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
    return MLQMC_EDEVICE;
  }
  return MLQMC_OK;
}
}  // namespace

extern "C" {

void mlqmc_default_opts(mlqmc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->prec = MLQMC_FP64;
  o->eig_rtol = 1e-8;
  o->max_rq_iter = 12;
  o->lin_rtol = 0.0;
  o->lam_rtol = 0.0;
  o->rq_lin_rtol = 1e-2;
  o->max_lin_iter = 60;
  o->chain_len = 0;
  o->batch = 0;
  o->pcg_graph = 1;
  o->io_on_device = 0;
  o->device_mem_cap = 0;
}

mlqmc_status mlqmc_create(mlqmc_ctx** out, const mlqmc_coeff* cf, int device, void* stream) {
  if (!out) {
    g_create_error = "out is NULL";
    return MLQMC_EINVAL;
  }
  *out = nullptr;
  if (!cf || cf->s_max < 0 || (cf->s_max > 0 && (!cf->c || !cf->k1 || !cf->k2))) {
    g_create_error = "invalid coefficient description";
    return MLQMC_EINVAL;
  }
  if (!std::isfinite(cf->a0)) {
    g_create_error = "a0 is not finite";
    return MLQMC_EINVAL;
  }
  double half = 0.0;
  for (int j = 0; j < cf->s_max; ++j) {
    if (!std::isfinite(cf->c[j]) || cf->k1[j] < 1 || cf->k2[j] < 1) {
      g_create_error = "coefficient term " + std::to_string(j) + " is invalid";
      return MLQMC_EINVAL;
    }
    half += 0.5 * std::fabs(cf->c[j]);
  }
  if (!(cf->a0 - half > 0.0)) {
    g_create_error = "a0 - 0.5 sum |c_j| <= 0: the coefficient is not uniformly positive";
    return MLQMC_EINVAL;
  }
  const bool host_only = device == MLQMC_HOST_ONLY;
  if (!host_only) CS(bind_new_device(device));
  mlqmc_ctx* ctx = new mlqmc_ctx();
  ctx->device = device;
  ctx->host_only = host_only;
  ctx->stream = static_cast<hipStream_t>(stream);
  // the no-allocation entry point's scratch on this device (device current)
  if (!host_only) ctx->scratch_err = scratch_address(device, &ctx->scratch_base);
  ctx->s_max = cf->s_max;
  ctx->a0 = cf->a0;
  const int sm = std::max(cf->s_max, 1);
  std::vector<double> c(sm, 0.0);
  std::vector<int> k1(sm, 1), k2(sm, 1);
  for (int j = 0; j < cf->s_max; ++j) {
    c[j] = cf->c[j];
    k1[j] = cf->k1[j];
    k2[j] = cf->k2[j];
  }
  ctx->h_k1.assign(k1.begin(), k1.begin() + cf->s_max);
  ctx->h_k2.assign(k2.begin(), k2.begin() + cf->s_max);
  if (host_only) {
    *out = ctx;
    return MLQMC_OK;
  }
  hipError_t e = hipMalloc(&ctx->d_c, sm * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&ctx->d_k1, sm * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&ctx->d_k2, sm * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(ctx->d_c, c.data(), sm * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_k1, k1.data(), sm * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_k2, k2.data(), sm * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    g_create_error = std::string("device setup: ") + hipGetErrorString(e);
    mlqmc_destroy(ctx);
    return MLQMC_EDEVICE;
  }
  *out = ctx;
  return MLQMC_OK;
}

mlqmc_status mlqmc_create_islands(mlqmc_ctx** out, const mlqmc_islands* cf, int device,
                                  void* stream) {
  if (!out) {
    g_create_error = "out is NULL";
    return MLQMC_EINVAL;
  }
  *out = nullptr;
  if (!cf || cf->s_max < 0 ||
      (cf->s_max > 0 && (!cf->ca || !cf->cb || !cf->k1 || !cf->k2 || !cf->region))) {
    g_create_error = "invalid islands description";
    return MLQMC_EINVAL;
  }
  for (double v : {cf->a0_in, cf->a0_out, cf->b0_in, cf->b0_out})
    if (!std::isfinite(v)) {
      g_create_error = "a background value is not finite";
      return MLQMC_EINVAL;
    }
  // bounds over |y_j| <= 1/2 on each region (Assumption A1 for a; b >= 0)
  double ha[2] = {0.0, 0.0}, hb[2] = {0.0, 0.0};
  for (int j = 0; j < cf->s_max; ++j) {
    const int r = cf->region[j];
    if (!std::isfinite(cf->ca[j]) || !std::isfinite(cf->cb[j]) || cf->k1[j] < 1 ||
        cf->k2[j] < 1 || (r != 1 && r != 2)) {
      g_create_error = "islands term " + std::to_string(j) + " is invalid";
      return MLQMC_EINVAL;
    }
    ha[r - 1] += 0.5 * std::fabs(cf->ca[j]);
    hb[r - 1] += 0.5 * std::fabs(cf->cb[j]);
  }
  if (!(cf->a0_in - ha[0] > 0.0) || !(cf->a0_out - ha[1] > 0.0)) {
    g_create_error = "the diffusion coefficient is not uniformly positive on a region";
    return MLQMC_EINVAL;
  }
  if (!(cf->b0_in - hb[0] >= 0.0) || !(cf->b0_out - hb[1] >= 0.0)) {
    g_create_error = "the reaction coefficient can be negative on a region";
    return MLQMC_EINVAL;
  }
  const bool host_only = device == MLQMC_HOST_ONLY;
  if (!host_only) CS(bind_new_device(device));
  mlqmc_ctx* ctx = new mlqmc_ctx();
  ctx->device = device;
  ctx->host_only = host_only;
  ctx->stream = static_cast<hipStream_t>(stream);
  // the no-allocation entry point's scratch on this device (device current)
  if (!host_only) ctx->scratch_err = scratch_address(device, &ctx->scratch_base);
  ctx->s_max = cf->s_max;
  ctx->islands = true;
  ctx->a_in = cf->a0_in;
  ctx->a_out = cf->a0_out;
  ctx->b_in = cf->b0_in;
  ctx->b_out = cf->b0_out;
  const int sm = std::max(cf->s_max, 1);
  std::vector<double> ca(sm, 0.0), cb(sm, 0.0);
  std::vector<int> k1(sm, 1), k2(sm, 1), rg(sm, 1);
  for (int j = 0; j < cf->s_max; ++j) {
    ca[j] = cf->ca[j];
    cb[j] = cf->cb[j];
    k1[j] = cf->k1[j];
    k2[j] = cf->k2[j];
    rg[j] = cf->region[j];
  }
  const size_t bd = sm * sizeof(double), bi = sm * sizeof(int);
  if (host_only) {
    *out = ctx;
    return MLQMC_OK;
  }
  hipError_t e = hipMalloc(&ctx->d_c, bd);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_cb, bd);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_k1, bi);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_k2, bi);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_region, bi);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_c, ca.data(), bd, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_cb, cb.data(), bd, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_k1, k1.data(), bi, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_k2, k2.data(), bi, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_region, rg.data(), bi, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    g_create_error = std::string("device setup: ") + hipGetErrorString(e);
    mlqmc_destroy(ctx);
    return MLQMC_EDEVICE;
  }
  *out = ctx;
  return MLQMC_OK;
}

void mlqmc_destroy(mlqmc_ctx* ctx) {
  if (!ctx) return;
  if (ctx->host_only) {  // holds host memory only
    delete ctx;
    return;
  }
  // teardown: errors here have nowhere to go, and every release is attempted
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto& kv : ctx->tables) kv.second.release();
  for (auto& kv : ctx->seps) {
    for (void* q : {(void*)kv.second.S, (void*)kv.second.cell_start, (void*)kv.second.cell_term})
      if (q) (void)hipFree(q);
    for (auto& tv : kv.second.tri)
      if (tv.second) (void)hipFree(tv.second);
  }
  for (auto& ev : ctx->ev_pool) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  for (auto& kv : ctx->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (hipStream_t ss : ctx->side) (void)hipStreamSynchronize(ss);
  for (hipStream_t ss : ctx->side) (void)hipStreamDestroy(ss);
  for (hipEvent_t ev : ctx->sync_ev) (void)hipEventDestroy(ev);
  if (ctx->d_c) (void)hipFree(ctx->d_c);
  if (ctx->d_k1) (void)hipFree(ctx->d_k1);
  if (ctx->d_k2) (void)hipFree(ctx->d_k2);
  if (ctx->d_cb) (void)hipFree(ctx->d_cb);
  if (ctx->d_region) (void)hipFree(ctx->d_region);
  delete ctx;
}

const char* mlqmc_last_error(const mlqmc_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

namespace {
mlqmc_status lattice_entry(mlqmc_ctx* ctx, int64_t N, int32_t s, const int64_t* z,
                           const double* shift, int64_t k0, int64_t count, double* Y,
                           int32_t on_dev, bool embedded) {
  if (!ctx) return MLQMC_EINVAL;
  if (!is_pow2(N) || N > ((int64_t)1 << 30)) return ctx->fail(MLQMC_EINVAL, "N must be a power of two <= 2^30");
  if (s < 0 || count < 0 || k0 < 0 || k0 + count > N)
    return ctx->fail(MLQMC_EINVAL, "need s >= 0 and 0 <= k0 <= k0+count <= N");
  if ((s > 0 && (!z || !shift)) || (count * s > 0 && !Y))
    return ctx->fail(MLQMC_EINVAL, "NULL buffer");
  for (int j = 0; j < s; ++j) {
    if (z[j] < 0 || z[j] >= N) return ctx->fail(MLQMC_EINVAL, "z[%d] outside [0, N)", j);
    if (!(shift[j] >= 0.0 && shift[j] < 1.0))
      return ctx->fail(MLQMC_EINVAL, "shift[%d] outside [0, 1)", j);
  }
  CS(ctx->bind());
  const int64_t* dz;
  const double* dsh;
  double* dY;
  CS(stage_in(ctx, "in_z", z, s, 0, &dz));
  CS(stage_in(ctx, "in_shift", shift, s, 0, &dsh));
  CS(out_buf(ctx, "out_Y", Y, (size_t)(count * s), on_dev, &dY));
  if (embedded)
    CK(launch_lattice_embedded(N, s, 1, dz, dsh, s, k0, count, dY, s, ctx->stream), "lattice");
  else
    CK(launch_lattice(N, s, dz, dsh, k0, count, dY, s, ctx->stream), "lattice");
  CS(stage_out(ctx, Y, dY, (size_t)(count * s), on_dev));
  return ctx->sync("lattice");
}
}  // namespace

mlqmc_status mlqmc_lattice_points(mlqmc_ctx* ctx, int64_t N, int32_t s, const int64_t* z,
                                  const double* shift, int64_t k0, int64_t count, double* Y,
                                  int32_t on_dev) {
  return lattice_entry(ctx, N, s, z, shift, k0, count, Y, on_dev, false);
}

mlqmc_status mlqmc_embedded_points(mlqmc_ctx* ctx, int64_t N, int32_t s, const int64_t* z,
                                   const double* shift, int64_t k0, int64_t count, double* Y,
                                   int32_t on_dev) {
  return lattice_entry(ctx, N, s, z, shift, k0, count, Y, on_dev, true);
}

mlqmc_status mlqmc_coefficient(mlqmc_ctx* ctx, int32_t n, int32_t s, int64_t B, const double* Y,
                               double* aK, int32_t on_dev) {
  if (!ctx) return MLQMC_EINVAL;
  if (!is_pow2(n) || n < 2 || n > 4096) return ctx->fail(MLQMC_EINVAL, "n must be a power of two in [2, 4096]");
  if (s < 0 || s > ctx->s_max) return ctx->fail(MLQMC_EINVAL, "s outside [0, s_max]");
  if (ctx->islands) return ctx->fail(MLQMC_EINVAL, "mlqmc_coefficient covers Problem 1 only");
  if (B < 0 || (B > 0 && (!aK || (s > 0 && !Y)))) return ctx->fail(MLQMC_EINVAL, "bad batch/buffers");
  if (!on_dev && B * s > 0 && !finite_host(Y, (size_t)(B * s)))
    return ctx->fail(MLQMC_EINVAL, "Y has non-finite entries");
  CS(ctx->bind());
  Table* tb = nullptr;
  CS(ctx->table(n, s, &tb));
  const double* dY;
  double* dA;
  const int E = 2 * n * n;
  CS(stage_in(ctx, "in_Y", Y, (size_t)(B * s), on_dev, &dY));
  CS(out_buf(ctx, "out_a", aK, (size_t)(B * E), on_dev, &dA));
  CK(launch_expand(B, s, E, dY, s, tb->el, ctx->a0, dA, nullptr, ctx->stream), "expand");
  CS(stage_out(ctx, aK, dA, (size_t)(B * E), on_dev));
  return ctx->sync("coefficient");
}

mlqmc_status mlqmc_apply_operator(mlqmc_ctx* ctx, int32_t n, int32_t s, int64_t B,
                                  const double* Y, const double* sigma, const double* x,
                                  double* out, int32_t on_dev) {
  if (!ctx) return MLQMC_EINVAL;
  if (!is_pow2(n) || n < 2 || n > 4096) return ctx->fail(MLQMC_EINVAL, "n must be a power of two in [2, 4096]");
  if (s < 0 || s > ctx->s_max) return ctx->fail(MLQMC_EINVAL, "s outside [0, s_max]");
  if (ctx->islands) return ctx->fail(MLQMC_EINVAL, "mlqmc_apply_operator covers Problem 1 only");
  if (B < 0 || (B > 0 && (!sigma || !x || !out || (s > 0 && !Y))))
    return ctx->fail(MLQMC_EINVAL, "bad batch/buffers");
  CS(ctx->bind());
  Table* tb = nullptr;
  CS(ctx->table(n, s, &tb));
  const int64_t D = (int64_t)(n - 1) * (n - 1), EW = 2LL * (n - 1) * n;
  const double *dY, *dsg, *dx;
  double *dout, *w;
  CS(stage_in(ctx, "in_Y", Y, (size_t)(B * s), on_dev, &dY));
  CS(stage_in(ctx, "in_sigma", sigma, (size_t)B, on_dev, &dsg));
  CS(stage_in(ctx, "in_x", x, (size_t)(B * D), on_dev, &dx));
  CS(out_buf(ctx, "out_x", out, (size_t)(B * D), on_dev, &dout));
  CS(ctx->getT("op_w", (size_t)(B * EW), &w));
  CK(launch_expand(B, s, EW, dY, s, tb->edge, ctx->a0, w, nullptr, ctx->stream), "expand");
  CK(launch_apply_plain(n, B, w, dsg, dx, dout, ctx->stream), "apply");
  CS(stage_out(ctx, out, dout, (size_t)(B * D), on_dev));
  return ctx->sync("apply");
}

mlqmc_status mlqmc_edge_weights(mlqmc_ctx* ctx, int32_t n, int32_t s, int64_t B,
                                const double* Y, double* w, int32_t on_dev) {
  if (!ctx) return MLQMC_EINVAL;
  if (!is_pow2(n) || n < 64 || n > 1024)
    return ctx->fail(MLQMC_EINVAL, "n must be a power of two in [64, 1024]");
  if (s < 0 || s > ctx->s_max) return ctx->fail(MLQMC_EINVAL, "s outside [0, s_max]");
  if (ctx->islands) return ctx->fail(MLQMC_EINVAL, "mlqmc_edge_weights covers Problem 1 only");
  if (B < 0 || (B > 0 && (!w || (s > 0 && !Y)))) return ctx->fail(MLQMC_EINVAL, "bad batch/buffers");
  if (!on_dev && B * s > 0 && !finite_host(Y, (size_t)(B * s)))
    return ctx->fail(MLQMC_EINVAL, "Y has non-finite entries");
  CS(ctx->bind());
  if (B == 0) return MLQMC_OK;
  const int64_t EW = 2 * padded_size(n);
  const double* dY = nullptr;
  double* dw;
  if (s > 0) CS(stage_in(ctx, "in_Y", Y, (size_t)(B * s), on_dev, &dY));
  CS(out_buf(ctx, "out_w", w, (size_t)(B * EW), on_dev, &dw));
  // the choice the fine-mesh solves make for this mesh and truncation
  mlqmc_ctx::SepTable* sep = nullptr;
  CS(ctx->sep_table(n, s, &sep));
  if (sep) {
    double* U;
    CS(ctx->getT("ew_U", (size_t)B * (3 * n + 2) * sep->kx, &U));
    CK(launch_expand_separable(B, n, s, sep->kx, sep->ky, dY, s, ctx->d_c, sep->cell_start,
                               sep->cell_term, sep->S, U, ctx->a0, dw, nullptr, EW, ctx->stream),
       "expand (separable)");
  } else {
    Table* tb = nullptr;
    CS(ctx->table(n, s, &tb));
    CK(launch_expand(B, s, EW, dY, s, tb->pad, ctx->a0, dw, nullptr, ctx->stream), "expand");
  }
  CS(stage_out(ctx, w, dw, (size_t)(B * EW), on_dev));
  return ctx->sync("edge weights");
}

mlqmc_status mlqmc_prolong(mlqmc_ctx* ctx, int32_t nH, int32_t nh, int64_t B, const double* uH,
                           double* uh, int32_t on_dev) {
  if (!ctx) return MLQMC_EINVAL;
  if (!is_pow2(nH) || !is_pow2(nh) || nH < 2 || nh < nH || nh > 4096)
    return ctx->fail(MLQMC_EINVAL, "need powers of two 2 <= nH <= nh <= 4096");
  if (B < 0 || (B > 0 && (!uH || !uh))) return ctx->fail(MLQMC_EINVAL, "bad batch/buffers");
  CS(ctx->bind());
  const int64_t DH = (int64_t)(nH - 1) * (nH - 1), Dh = (int64_t)(nh - 1) * (nh - 1);
  const double* du;
  double* dv;
  CS(stage_in(ctx, "in_uH", uH, (size_t)(B * DH), on_dev, &du));
  CS(out_buf(ctx, "out_uh", uh, (size_t)(B * Dh), on_dev, &dv));
  if (B > 0 && Dh > 0) CK(launch_prolong_interior(nH, nh, B, du, dv, ctx->stream), "prolong");
  CS(stage_out(ctx, uh, dv, (size_t)(B * Dh), on_dev));
  return ctx->sync("prolong");
}

mlqmc_status mlqmc_eig_level(mlqmc_ctx* ctx, const mlqmc_level* L, const mlqmc_opts* o,
                             int64_t n, const double* Y, int32_t warm, double* lam,
                             double* lam_prev, double* lam_coarse, int32_t* rq_iters,
                             int32_t* lin_iters, uint8_t* flags, double* g, double* g_prev) {
  if (!ctx) return MLQMC_EINVAL;
  CS(check_opts(ctx, o));
  CS(check_level(ctx, L));
  CS(check_islands_level(ctx, L));
  if (n < 0) return ctx->fail(MLQMC_EINVAL, "n < 0");
  if (n > 0 && (!Y || !lam || !flags)) return ctx->fail(MLQMC_EINVAL, "NULL buffer");
  if (n > 0 && L->n_prev && !lam_prev) return ctx->fail(MLQMC_EINVAL, "lam_prev is NULL but n_prev > 0");
  const int dev = o->io_on_device;
  const int64_t s = L->s_fine;
  if (!dev && n * s > 0 && !finite_host(Y, (size_t)(n * s)))
    return ctx->fail(MLQMC_EINVAL, "Y has non-finite entries");
  ctx->mem_cap = o->device_mem_cap;
  CS(ctx->bind());
  if (n == 0) return MLQMC_OK;
  const double* dY;
  double *dl, *dlp = nullptr, *dlc = nullptr;
  int *dri = nullptr, *dli = nullptr;
  uint8_t* dfl;
  CS(stage_in(ctx, "in_Y", Y, (size_t)(n * s), dev, &dY));
  CS(out_buf(ctx, "o_lam", lam, n, dev, &dl));
  if (L->n_prev) CS(out_buf(ctx, "o_lamp", lam_prev, n, dev, &dlp));
  if (lam_coarse) CS(out_buf(ctx, "o_lamc", lam_coarse, n, dev, &dlc));
  if (rq_iters) CS(out_buf(ctx, "o_rq", rq_iters, n, dev, &dri));
  CS(out_buf(ctx, "o_li", lin_iters, n, dev && lin_iters, &dli));
  CS(out_buf(ctx, "o_fl", flags, n, dev, &dfl));
  double *dg = nullptr, *dgp = nullptr;
  if (g) CS(out_buf(ctx, "o_g", g, n, dev, &dg));
  if (g_prev && L->n_prev) CS(out_buf(ctx, "o_gp", g_prev, n, dev, &dgp));
  CS(level_core(ctx, L, o, n, dY, s, warm, dl, dlp, dlc, dri, dli, dfl, dg, dgp));
  if (dg) CS(stage_out(ctx, g, dg, n, dev));
  if (dgp) CS(stage_out(ctx, g_prev, dgp, n, dev));
  CS(stage_out(ctx, lam, dl, n, dev));
  if (dlp) CS(stage_out(ctx, lam_prev, dlp, n, dev));
  if (dlc) CS(stage_out(ctx, lam_coarse, dlc, n, dev));
  if (dri) CS(stage_out(ctx, rq_iters, dri, n, dev));
  if (lin_iters) CS(stage_out(ctx, lin_iters, dli, n, dev));
  CS(stage_out(ctx, flags, dfl, n, dev));
  CS(ctx->sync("eig_level"));
  bool any = false;
  CS(any_flag(ctx, dfl, n, &any));
  return any ? ctx->fail(MLQMC_ENOCONV, "at least one sample is flagged") : MLQMC_OK;
}

}  // extern "C"

namespace {
// Upper bound of the scratch bytes level_core carves for this level without
// allocating (meshes up to 1/32: coefficient tables, the coarse vectors and
// eigenvalues, the previous-level eigensolve's flags and counts, the inner
// iteration counts when the caller passes none).
size_t noalloc_bytes(const mlqmc_ctx* ctx, const mlqmc_level* L, int64_t n, bool have_lamc,
                     bool have_lin) {
  auto table = [&](int m, int s) -> size_t {
    if (m == 0) return 0;
    const size_t rows = ctx->islands ? (size_t)s + 1 : (size_t)std::max(s, 1);
    size_t b = round256(rows * 2 * m * m * 8) + round256(rows * 2 * padded_size(m) * 8);
    if (ctx->islands)
      b += round256(rows * 2 * m * m * 8) + round256(rows * 3 * padded_size(m) * 8);
    return b;
  };
  size_t need = have_lin ? 0 : round256((size_t)n * 4);
  if (L->n_coarse == 0) {
    need += table(L->n_fine, L->s_fine);
    if (L->n_prev) need += table(L->n_prev, L->s_prev) + round256((size_t)n) + round256((size_t)n * 4);
    return need;
  }
  const size_t DH = (size_t)(L->n_coarse - 1) * (L->n_coarse - 1);
  need += table(L->n_coarse, L->s_coarse) + round256((size_t)n * DH * 8);
  if (!have_lamc) need += round256((size_t)n * 8);
  need += table(L->n_fine, L->s_fine);
  const bool degenerate = L->n_prev == L->n_coarse && L->s_prev == L->s_coarse;
  if (L->n_prev && !degenerate) need += table(L->n_prev, L->s_prev);
  return need;
}
}  // namespace

extern "C" {

mlqmc_status mlqmc_eig_level_noalloc(mlqmc_ctx* ctx, const mlqmc_level* L, const mlqmc_opts* o,
                                     int64_t n, const double* Y, int32_t warm, double* lam,
                                     double* lam_prev, double* lam_coarse, int32_t* rq_iters,
                                     int32_t* lin_iters, uint8_t* flags) {
  if (!ctx) return MLQMC_EINVAL;
  CS(check_opts(ctx, o));
  CS(check_level(ctx, L));
  CS(check_islands_level(ctx, L));
  if (!o->io_on_device)
    return ctx->fail(MLQMC_EINVAL, "the no-allocation entry point takes device pointers only "
                                   "(io_on_device = 1)");
  if (L->n_fine > 32 || L->n_coarse > 32 || L->n_prev > 32)
    return ctx->fail(MLQMC_EINVAL, "the no-allocation entry point covers meshes up to 1/32 "
                                   "(got %d, %d, %d)", L->n_fine, L->n_coarse, L->n_prev);
  if (n < 0) return ctx->fail(MLQMC_EINVAL, "n < 0");
  if (n > 0 && (!Y || !lam || !flags)) return ctx->fail(MLQMC_EINVAL, "NULL buffer");
  if (n > 0 && L->n_prev && !lam_prev)
    return ctx->fail(MLQMC_EINVAL, "lam_prev is NULL but n_prev > 0");
  const size_t need = noalloc_bytes(ctx, L, n, lam_coarse != nullptr, lin_iters != nullptr);
  if (need > (size_t)MLQMC_NOALLOC_SCRATCH_BYTES)
    return ctx->fail(MLQMC_EINVAL, "this call needs %zu bytes of scratch; the maximum is %zu "
                                   "(MLQMC_NOALLOC_SCRATCH_BYTES)",
                     need, (size_t)MLQMC_NOALLOC_SCRATCH_BYTES);
  CS(ctx->bind());
  if (!ctx->scratch_base)
    return ctx->hip_fail(ctx->scratch_err != hipSuccess ? ctx->scratch_err : hipErrorInvalidValue,
                         "address of the no-allocation scratch");
  if (n == 0) return MLQMC_OK;
  // every named buffer and table of this call comes from the scratch
  struct Arena {
    mlqmc_ctx* c;
    ~Arena() {
      c->arena = nullptr;
      c->arena_size = c->arena_used = 0;
      c->arena_tables.clear();
    }
  } guard{ctx};
  ctx->arena = static_cast<char*>(ctx->scratch_base);
  ctx->arena_size = MLQMC_NOALLOC_SCRATCH_BYTES;
  ctx->arena_used = 0;
  ctx->arena_tables.clear();
  int* dli = lin_iters;
  if (!dli) CS(ctx->getT("o_li", n, &dli));
  CS(level_core(ctx, L, o, n, Y, L->s_fine, warm, lam, L->n_prev ? lam_prev : nullptr,
                lam_coarse, rq_iters, dli, flags));
  CS(ctx->sync("eig_level_noalloc"));
  bool any = false;
  CS(any_flag(ctx, flags, n, &any));
  return any ? ctx->fail(MLQMC_ENOCONV, "at least one sample is flagged") : MLQMC_OK;
}

mlqmc_status mlqmc_estimate(mlqmc_ctx* ctx, int32_t nl, const mlqmc_level* lv, const int64_t* N,
                            int32_t R, const int64_t* z, const double* shifts,
                            const mlqmc_opts* o, double* Q_lr, double* Qhat, double* V,
                            double* est, double* g_stats) {
  if (!ctx) return MLQMC_EINVAL;
  CS(check_opts(ctx, o));
  if (nl < 1 || !lv || !N || !z || !shifts || R < 1)
    return ctx->fail(MLQMC_EINVAL, "need n_levels >= 1, R >= 1 and non-NULL inputs");
  if (!Q_lr || !Qhat || !V || !est) return ctx->fail(MLQMC_EINVAL, "NULL output");
  int64_t zoff = 0, soff = 0;
  for (int l = 0; l < nl; ++l) {
    CS(check_level(ctx, &lv[l]));
    CS(check_islands_level(ctx, &lv[l]));
    if (!is_pow2(N[l]) || N[l] > ((int64_t)1 << 30))
      return ctx->fail(MLQMC_EINVAL, "N[%d] must be a power of two <= 2^30", l);
    const int s = lv[l].s_fine;
    for (int j = 0; j < s; ++j)
      if (z[zoff + j] < 0 || z[zoff + j] >= N[l])
        return ctx->fail(MLQMC_EINVAL, "z of level %d outside [0, N)", l);
    for (int64_t k = 0; k < (int64_t)R * s; ++k)
      if (!(shifts[soff + k] >= 0.0 && shifts[soff + k] < 1.0))
        return ctx->fail(MLQMC_EINVAL, "shift of level %d outside [0, 1)", l);
    zoff += s;
    soff += (int64_t)R * s;
  }
  ctx->mem_cap = o->device_mem_cap;
  CS(ctx->bind());
  hipStream_t st = ctx->stream;
  const int dev = o->io_on_device;
  double *dQ, *dQh, *dV, *dest;
  CS(out_buf(ctx, "e_Q", Q_lr, (size_t)nl * R, dev, &dQ));
  CS(out_buf(ctx, "e_Qh", Qhat, nl, dev, &dQh));
  CS(out_buf(ctx, "e_V", V, nl, dev, &dV));
  CS(out_buf(ctx, "e_est", est, 2, dev, &dest));
  // G statistics: [Q_lr | Qhat | V | est] of the functional, same shapes
  const size_t gsz = (size_t)nl * R + 2 * (size_t)nl + 2;
  double* dG = nullptr;
  if (g_stats) CS(out_buf(ctx, "e_G", g_stats, gsz, dev, &dG));
  // The levels are independent (Algorithm 2).  Those whose every solve runs
  // per sample in LDS (meshes up to 1/32) need no host round trip: they are
  // enqueued first, each on a stream of its own, and run beside the batched
  // levels, which follow on the context's stream (their PCG reads back which
  // samples are still active).  Every level has its own buffers; the
  // coefficient tables are built before the fork, with the largest truncation
  // each mesh needs, so no table is rebuilt while a level reads it.
  auto lds_only = [](const mlqmc_level& L) {
    return L.n_fine <= 32 && L.n_coarse <= 32 && L.n_prev <= 32;
  };
  {
    std::map<int, int> smax;
    auto need = [&](int m, int sv) {
      if (m > 0) smax[m] = std::max(smax[m], sv);
    };
    for (int l = 0; l < nl; ++l) {
      need(lv[l].n_fine, lv[l].s_fine);
      need(lv[l].n_coarse, lv[l].s_coarse);
      need(lv[l].n_prev, lv[l].s_prev);
    }
    for (const auto& kv : smax) {
      Table* tb = nullptr;
      CS(ctx->table(kv.first, kv.second, &tb));
    }
  }
  std::vector<int64_t> zo(nl), so(nl);
  zoff = soff = 0;
  for (int l = 0; l < nl; ++l) {
    zo[l] = zoff;
    so[l] = soff;
    zoff += lv[l].s_fine;
    soff += (int64_t)R * lv[l].s_fine;
  }
  std::vector<uint8_t*> lflags(nl, nullptr);
  // one level on the context's current stream, buffers named by level
  auto run_level = [&](int l) -> mlqmc_status {
    const mlqmc_level& L = lv[l];
    const int s = L.s_fine;
    const int64_t n = (int64_t)R * N[l];
    const std::string p = "e" + std::to_string(l) + "_";
    auto nm = [&](const char* x) { return p + x; };
    hipStream_t ls = ctx->stream;
    const int64_t* dz;
    const double* dsh;
    CS(stage_in(ctx, nm("z").c_str(), z + zo[l], s, 0, &dz));
    CS(stage_in(ctx, nm("sh").c_str(), shifts + so[l], (size_t)R * s, 0, &dsh));
    double *Y, *lam, *lamp = nullptr;
    int *rqi, *lini;
    uint8_t* fl;
    CS(ctx->getT(nm("Y").c_str(), (size_t)(n * std::max(s, 1)), &Y));
    CS(ctx->getT(nm("lam").c_str(), n, &lam));
    if (L.n_prev) CS(ctx->getT(nm("lamp").c_str(), n, &lamp));
    CS(ctx->getT(nm("rq").c_str(), n, &rqi));
    CS(ctx->getT(nm("li").c_str(), n, &lini));
    CS(ctx->getT(nm("fl").c_str(), n, &fl));
    lflags[l] = fl;
    CK(launch_lattice_multi(N[l], s, R, dz, dsh, N[l], Y, std::max(s, 1), ls), "lattice");
    mlqmc_opts oo = *o;
    oo.chain_len = shift_chain(ctx, N[l], R, o, L.n_coarse ? L.n_coarse : L.n_fine);
    double *gv = nullptr, *gp = nullptr;
    if (dG) {
      CS(ctx->getT(nm("g").c_str(), n, &gv));
      if (L.n_prev) CS(ctx->getT(nm("gp").c_str(), n, &gp));
    }
    CS(level_core(ctx, &L, &oo, n, Y, std::max(s, 1), 1, lam, lamp, nullptr, rqi, lini, fl, gv,
                  gp, p));
    CK(launch_level_sums(N[l], R, lam, lamp, dQ + (int64_t)l * R, ls), "level sums");
    if (dG) CK(launch_level_sums(N[l], R, gv, gp, dG + (int64_t)l * R, ls), "level sums");
    return MLQMC_OK;
  };
  // fork: the side streams start after everything enqueued so far
  std::vector<hipEvent_t> joins;
  int side = 0;
  for (int l = 0; l < nl; ++l)
    if (lds_only(lv[l])) ++side;
  if (side > 1 || (side == 1 && side < nl)) {
    hipEvent_t fork = nullptr;
    CS(ctx->event(0, &fork));
    CK(hipEventRecord(fork, st), "fork");
    int k = 0;
    for (int l = 0; l < nl; ++l) {
      if (!lds_only(lv[l])) continue;
      hipStream_t ss = nullptr;
      CS(ctx->side_stream(k, &ss));
      CK(hipStreamWaitEvent(ss, fork, 0), "fork");
      const hipStream_t keep = ctx->stream;
      ctx->stream = ss;
      const mlqmc_status r = run_level(l);
      ctx->stream = keep;
      CS(r);
      hipEvent_t j = nullptr;
      CS(ctx->event(1 + k, &j));
      CK(hipEventRecord(j, ss), "join");
      joins.push_back(j);
      ++k;
    }
    for (int l = 0; l < nl; ++l)
      if (!lds_only(lv[l])) CS(run_level(l));
    for (hipEvent_t j : joins) CK(hipStreamWaitEvent(st, j, 0), "join");
  } else {
    for (int l = 0; l < nl; ++l) CS(run_level(l));
  }
  bool flagged = false;
  CK(launch_estimator_final(nl, R, dQ, dQh, dV, dest, 0, st), "estimator");
  if (dG) {
    double* q = dG + (size_t)nl * R;
    CK(launch_estimator_final(nl, R, dG, q, q + nl, q + 2 * nl, 0, st), "estimator");
  }
  CS(stage_out(ctx, Q_lr, dQ, (size_t)nl * R, dev));
  CS(stage_out(ctx, Qhat, dQh, nl, dev));
  CS(stage_out(ctx, V, dV, nl, dev));
  CS(stage_out(ctx, est, dest, 2, dev));
  if (dG) CS(stage_out(ctx, g_stats, dG, gsz, dev));
  CS(ctx->sync("estimate"));
  for (int l = 0; l < nl; ++l) {
    bool any = false;
    CS(any_flag(ctx, lflags[l], (int64_t)R * N[l], &any));
    flagged |= any;
  }
  return flagged ? ctx->fail(MLQMC_ENOCONV, "at least one sample is flagged") : MLQMC_OK;
}

// The levels, sizes and inputs of a nested estimate (host arrays): level 0
// direct, every coarse pair level 0's, each previous term the level below's
// value, N non-increasing and powers of two, 0 <= N_done <= N.
mlqmc_status check_nested(mlqmc_ctx* ctx, int32_t nl, const mlqmc_level* lv, const int64_t* Nd,
                          const int64_t* N, int32_t R, const int64_t* z, const double* shifts) {
  int s_max = 0;
  for (int l = 0; l < nl; ++l) {
    CS(check_level(ctx, &lv[l]));
    CS(check_islands_level(ctx, &lv[l]));
    if (!is_pow2(N[l]) || N[l] > ((int64_t)1 << 30))
      return ctx->fail(MLQMC_EINVAL, "N[%d] must be a power of two <= 2^30", l);
    if (l > 0 && N[l] > N[l - 1])
      return ctx->fail(MLQMC_EINVAL, "N must not increase with the level (N[%d] > N[%d])", l,
                       l - 1);
    const int64_t d = Nd ? Nd[l] : 0;
    if (d < 0 || d > N[l]) return ctx->fail(MLQMC_EINVAL, "N_done[%d] outside [0, N[%d]]", l, l);
    s_max = std::max(s_max, (int)lv[l].s_fine);
  }
  const mlqmc_level& L0 = lv[0];
  if (L0.n_coarse != 0 || L0.n_prev != 0)
    return ctx->fail(MLQMC_EINVAL, "level 0 must be direct with no previous term");
  for (int l = 1; l < nl; ++l) {
    if (lv[l].n_coarse != L0.n_fine || lv[l].s_coarse != L0.s_fine)
      return ctx->fail(MLQMC_EINVAL, "level %d: coarse mesh and truncation must be level 0's", l);
    if (lv[l].n_prev != lv[l - 1].n_fine || lv[l].s_prev != lv[l - 1].s_fine)
      return ctx->fail(MLQMC_EINVAL, "level %d: previous term must be on level %d's mesh", l,
                       l - 1);
  }
  // z: the generating vector of the largest rule the estimate may grow to;
  // a rule of N points uses it modulo N
  for (int j = 0; j < s_max; ++j)
    if (z[j] < 0 || z[j] >= ((int64_t)1 << 31))
      return ctx->fail(MLQMC_EINVAL, "z[%d] outside [0, 2^31)", j);
  for (int64_t k = 0; k < (int64_t)R * s_max; ++k)
    if (!(shifts[k] >= 0.0 && shifts[k] < 1.0))
      return ctx->fail(MLQMC_EINVAL, "shift entry %lld outside [0, 1)", (long long)k);
  return MLQMC_OK;
}


namespace {
// The nested estimator over the points [Nd[l], N[l]) of each level (Nd =
// nullptr: none done), added to running per-(level, shift) sums of Y_l on the
// device (dsum [nl x R]; dgsum the same for G, when g_stats is requested).
// The embedded rule makes the points independent of N (point k is the lattice
// point phi_2(k) z + shift for every rule size above k), so an estimate over
// N points continues to any larger N.  Level l is evaluated on [e_l, N[l]),
// e_l = min(Nd[l], Nd[l+1]): its own new points and those where level l+1
// needs lambda^l; level 0 provides the coarse pairs on [min_l Nd[l], N[0]).
mlqmc_status nested_core(mlqmc_ctx* ctx, int32_t nl, const mlqmc_level* lv, const int64_t* Nd,
                         const int64_t* N, int32_t R, const int64_t* z, const double* shifts,
                         const mlqmc_opts* o, double* dsum, double* dgsum, double* Q_lr,
                         double* Qhat, double* V, double* est, double* lam_out,
                         double* g_stats) {
  CS(check_nested(ctx, nl, lv, Nd, N, R, z, shifts));
  const mlqmc_level& L0 = lv[0];
  int s_max = 0;
  int64_t total = 0;
  std::vector<int64_t> a(nl), e(nl);
  for (int l = 0; l < nl; ++l) {
    a[l] = Nd ? Nd[l] : 0;
    s_max = std::max(s_max, (int)lv[l].s_fine);
    total += (int64_t)R * N[l];
  }
  // Level l is evaluated on [e_l, f_l): its own new points [a_l, N_l) and the
  // points [a_{l+1}, N_{l+1}) where level l+1 needs lambda^l; level 0 on the
  // union of the non-empty ranges (it supplies every level's coarse pairs).
  std::vector<int64_t> f(nl);
  for (int l = 0; l < nl; ++l) {
    e[l] = (l + 1 < nl) ? std::min(a[l], a[l + 1]) : a[l];
    f[l] = a[l] < N[l] ? N[l] : e[l];
    if (l + 1 < nl && a[l + 1] < N[l + 1]) f[l] = std::max(f[l], N[l + 1]);
  }
  {
    int64_t lo = -1, hi = -1;
    for (int l = 0; l < nl; ++l)
      if (f[l] > e[l]) {
        lo = lo < 0 ? e[l] : std::min(lo, e[l]);
        hi = std::max(hi, f[l]);
      }
    e[0] = lo < 0 ? N[0] : lo;
    f[0] = lo < 0 ? N[0] : hi;
  }
  if (lam_out && std::any_of(a.begin(), a.end(), [](int64_t v) { return v != 0; }))
    return ctx->fail(MLQMC_EINVAL, "lam_out needs every level to start at point 0");
  int64_t ymax = 1;
  for (int l = 0; l < nl; ++l)
    ymax = std::max<int64_t>(ymax, (int64_t)R * (f[l] - e[l]) * std::max(1, (int)lv[l].s_fine));
  hipStream_t st = ctx->stream;
  const int dev = o->io_on_device;
  double *dQ, *dQh, *dV, *dest, *dlo = nullptr;
  CS(out_buf(ctx, "e_Q", Q_lr, (size_t)nl * R, dev, &dQ));
  CS(out_buf(ctx, "e_Qh", Qhat, nl, dev, &dQh));
  CS(out_buf(ctx, "e_V", V, nl, dev, &dV));
  CS(out_buf(ctx, "e_est", est, 2, dev, &dest));
  if (lam_out) CS(out_buf(ctx, "e_lamout", lam_out, (size_t)total, dev, &dlo));
  const size_t gsz = (size_t)nl * R + 2 * (size_t)nl + 2;
  double *dG = nullptr, *g0 = nullptr;
  if (g_stats) CS(out_buf(ctx, "e_G", g_stats, gsz, dev, &dG));
  const int64_t* dz;
  const double* dsh;
  CS(stage_in(ctx, "e_z", z, s_max, 0, &dz));
  CS(stage_in(ctx, "e_sh", shifts, (size_t)R * s_max, 0, &dsh));
  const int64_t N0 = N[0], c0 = e[0], n0pts = f[0] - c0, B0 = (int64_t)R * n0pts;
  const int n0 = L0.n_fine, s0 = L0.s_fine;
  const int64_t D0 = (int64_t)(n0 - 1) * (n0 - 1);
  double *Y, *lam0 = nullptr, *u0 = nullptr;
  int *rqi, *lini;
  uint8_t* fl;
  const int64_t Bmax = std::max<int64_t>(B0, 1);
  CS(ctx->getT("n_Y", (size_t)ymax, &Y));
  CS(ctx->getT("n_lam0", Bmax, &lam0));
  if (nl > 1) CS(ctx->getT("n_u0", (size_t)(Bmax * D0), &u0));
  CS(ctx->getT("n_rq", Bmax, &rqi));
  CS(ctx->getT("n_li", Bmax, &lini));
  CS(ctx->getT("n_fl", Bmax, &fl));
  if (dG) CS(ctx->getT("n_g0", Bmax, &g0));
  bool flagged = false;
  // level 0: direct eigenpairs of its points; the eigenvectors are the
  // coarse pairs of the levels above
  if (B0 > 0) {
    CK(hipMemsetAsync(fl, 0, B0, st), "memset");
    CK(hipMemsetAsync(lini, 0, B0 * sizeof(int), st), "memset");
    CK(launch_lattice_embedded(N0, s0, R, dz, dsh, s_max, c0, n0pts, Y, std::max(s0, 1), st),
       "lattice");
    Table* tb = nullptr;
    CS(ctx->table(n0, s0, &tb));
    // a power of two dividing the points per shift: no chain crosses shifts
    int chain = shift_chain(ctx, n0pts, R, o, n0);
    while (n0pts % chain) chain /= 2;
    RqiArgs ra = rqi_base(ctx, o, B0, Y, std::max(s0, 1), chain, 1, rqi, lini, fl);
    ra.S = s0;
    ra.phi = tb->pad;
    ra.rphi = tb->rpad;
    ra.lam = lam0;
    ra.u_out = u0;
    ra.g_out = g0;
    ra.refine = ctx->islands ? 1 : 0;  // the coarse pairs of every level above
    if (const int64_t per = rqi_scratch_doubles(n0)) {
      ra.scratch_doubles = per * ((B0 + chain - 1) / chain);
      CS(ctx->getT("rqi_scratch", ra.scratch_doubles, &ra.scratch));
    }
    ctx->t_begin(MLQMC_K_COARSE);
    CK(launch_rqi(n0, ra, st), "eigensolve (LDS)");
    ctx->t_end(MLQMC_K_COARSE, 0.0);
  }
  CK(launch_level_sums_acc(N0 - a[0], N0, R, lam0, n0pts, a[0] - c0, nullptr, 0, 0, dsum, dQ, st),
     "level sums");
  if (dG)
    CK(launch_level_sums_acc(N0 - a[0], N0, R, g0, n0pts, a[0] - c0, nullptr, 0, 0, dgsum, dG,
                             st),
       "level sums");
  if (dlo) CK(hipMemcpyAsync(dlo, lam0, B0 * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  if (B0 > 0) {
    bool any = false;
    CS(any_flag(ctx, fl, B0, &any));
    flagged |= any;
  }
  // levels l >= 1: the two-grid update from the level-0 pair of the same
  // point, minus level l-1's value there
  const double* prev = lam0;
  const double* gprev = g0;
  int64_t prev_lo = c0, prev_cnt = n0pts, off = B0;
  // rows [lo - c0, lo - c0 + cnt) of every shift's n0pts rows of `width`
  // elements of a level-0 array
  auto rows0 = [&](const double* src, int64_t lo, int64_t cnt, int64_t width, const char* name,
                   const double** out) -> mlqmc_status {
    if (lo == c0 && cnt == n0pts) {
      *out = src;
      return MLQMC_OK;
    }
    double* dst = nullptr;
    CS(ctx->getT(name, (size_t)(R * cnt * width), &dst));
    CK(hipMemcpy2DAsync(dst, cnt * width * sizeof(double), src + (lo - c0) * width,
                        n0pts * width * sizeof(double), cnt * width * sizeof(double), R,
                        hipMemcpyDeviceToDevice, st),
       "gather");
    *out = dst;
    return MLQMC_OK;
  };
  for (int l = 1; l < nl; ++l) {
    const mlqmc_level& L = lv[l];
    const int64_t cnt = f[l] - e[l], Bl = (int64_t)R * cnt;
    const int sl = L.s_fine;
    double* lam = nullptr;
    double* gl = nullptr;
    CS(ctx->getT((l & 1) ? "n_lamA" : "n_lamB", std::max<int64_t>(Bl, 1), &lam));
    if (dG) CS(ctx->getT((l & 1) ? "n_gA" : "n_gB", std::max<int64_t>(Bl, 1), &gl));
    if (Bl > 0) {
      const double *uH, *lamH;
      CS(rows0(u0, e[l], cnt, D0, "n_uH", &uH));
      CS(rows0(lam0, e[l], cnt, 1, "n_lamH", &lamH));
      CK(launch_lattice_embedded(N0, sl, R, dz, dsh, s_max, e[l], cnt, Y, std::max(sl, 1), st),
         "lattice");
      CK(hipMemsetAsync(fl, 0, Bl, st), "memset");
      CK(hipMemsetAsync(lini, 0, Bl * sizeof(int), st), "memset");
      CS(fine_update(ctx, o, L.n_fine, sl, Y, std::max(sl, 1), uH, lamH, n0, Bl, lam, gl, lini,
                     fl, "f_"));
    }
    // Y_l over the new points [a_l, N_l): lambda^l at offset a_l - e_l of its
    // rows, lambda^{l-1} at a_l - e_{l-1} of level l-1's
    CK(launch_level_sums_acc(N[l] - a[l], N[l], R, lam, cnt, a[l] - e[l], prev, prev_cnt,
                             a[l] - prev_lo, dsum + (int64_t)l * R, dQ + (int64_t)l * R, st),
       "level sums");
    if (dG)
      CK(launch_level_sums_acc(N[l] - a[l], N[l], R, gl, cnt, a[l] - e[l], gprev, prev_cnt,
                               a[l] - prev_lo, dgsum + (int64_t)l * R, dG + (int64_t)l * R, st),
         "level sums");
    if (dlo && Bl > 0)
      CK(hipMemcpyAsync(dlo + off, lam, Bl * sizeof(double), hipMemcpyDeviceToDevice, st),
         "copy");
    if (Bl > 0) {
      bool any = false;
      CS(any_flag(ctx, fl, Bl, &any));
      flagged |= any;
    }
    prev = lam;
    gprev = gl;
    prev_lo = e[l];
    prev_cnt = cnt;
    off += Bl;
  }
  CK(launch_estimator_final(nl, R, dQ, dQh, dV, dest, 1, st), "estimator");
  if (dG) {
    double* q = dG + (size_t)nl * R;
    CK(launch_estimator_final(nl, R, dG, q, q + nl, q + 2 * nl, 1, st), "estimator");
  }
  CS(stage_out(ctx, Q_lr, dQ, (size_t)nl * R, dev));
  CS(stage_out(ctx, Qhat, dQh, nl, dev));
  CS(stage_out(ctx, V, dV, nl, dev));
  CS(stage_out(ctx, est, dest, 2, dev));
  if (dlo) CS(stage_out(ctx, lam_out, dlo, (size_t)total, dev));
  if (dG) CS(stage_out(ctx, g_stats, dG, gsz, dev));
  CS(ctx->sync("estimate_nested"));
  return flagged ? ctx->fail(MLQMC_ENOCONV, "at least one sample is flagged") : MLQMC_OK;
}
}  // namespace

mlqmc_status mlqmc_estimate_nested(mlqmc_ctx* ctx, int32_t nl, const mlqmc_level* lv,
                                   const int64_t* N, int32_t R, const int64_t* z,
                                   const double* shifts, const mlqmc_opts* o, double* Q_lr,
                                   double* Qhat, double* V, double* est, double* lam_out,
                                   double* g_stats) {
  if (!ctx) return MLQMC_EINVAL;
  CS(check_opts(ctx, o));
  if (nl < 1 || !lv || !N || !z || !shifts || R < 1)
    return ctx->fail(MLQMC_EINVAL, "need n_levels >= 1, R >= 1 and non-NULL inputs");
  if (!Q_lr || !Qhat || !V || !est) return ctx->fail(MLQMC_EINVAL, "NULL output");
  CS(check_nested(ctx, nl, lv, nullptr, N, R, z, shifts));
  ctx->mem_cap = o->device_mem_cap;
  CS(ctx->bind());
  double *dsum = nullptr, *dgsum = nullptr;
  CS(ctx->getT("e_sum", (size_t)nl * R, &dsum));
  CK(hipMemsetAsync(dsum, 0, (size_t)nl * R * sizeof(double), ctx->stream), "memset");
  if (g_stats) {
    CS(ctx->getT("e_gsum", (size_t)nl * R, &dgsum));
    CK(hipMemsetAsync(dgsum, 0, (size_t)nl * R * sizeof(double), ctx->stream), "memset");
  }
  return nested_core(ctx, nl, lv, nullptr, N, R, z, shifts, o, dsum, dgsum, Q_lr, Qhat, V, est,
                     lam_out, g_stats);
}

mlqmc_status mlqmc_estimate_nested_extend(mlqmc_ctx* ctx, int32_t nl, const mlqmc_level* lv,
                                          const int64_t* N_done, const int64_t* N, int32_t R,
                                          const int64_t* z, const double* shifts,
                                          const mlqmc_opts* o, double* sums, double* Q_lr,
                                          double* Qhat, double* V, double* est, double* g_sums,
                                          double* g_stats) {
  if (!ctx) return MLQMC_EINVAL;
  CS(check_opts(ctx, o));
  if (nl < 1 || !lv || !N || !N_done || !z || !shifts || R < 1 || !sums)
    return ctx->fail(MLQMC_EINVAL, "need n_levels >= 1, R >= 1 and non-NULL inputs");
  if (!Q_lr || !Qhat || !V || !est) return ctx->fail(MLQMC_EINVAL, "NULL output");
  if ((g_sums == nullptr) != (g_stats == nullptr))
    return ctx->fail(MLQMC_EINVAL, "g_sums and g_stats go together");
  CS(check_nested(ctx, nl, lv, N_done, N, R, z, shifts));
  ctx->mem_cap = o->device_mem_cap;
  CS(ctx->bind());
  const int dev = o->io_on_device;
  const size_t n = (size_t)nl * R;
  const hipMemcpyKind in = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const hipMemcpyKind back = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  double *dsum = nullptr, *dgsum = nullptr;
  // private copies: on an error the caller's sums stay as they were
  CS(ctx->getT("e_sum", n, &dsum));
  CK(hipMemcpyAsync(dsum, sums, n * sizeof(double), in, ctx->stream), "copy in");
  if (g_sums) {
    CS(ctx->getT("e_gsum", n, &dgsum));
    CK(hipMemcpyAsync(dgsum, g_sums, n * sizeof(double), in, ctx->stream), "copy in");
  }
  const mlqmc_status stc = nested_core(ctx, nl, lv, N_done, N, R, z, shifts, o, dsum, dgsum,
                                       Q_lr, Qhat, V, est, nullptr, g_stats);
  if (stc != MLQMC_OK && stc != MLQMC_ENOCONV) return stc;
  const std::string msg = ctx->err;
  CK(hipMemcpyAsync(sums, dsum, n * sizeof(double), back, ctx->stream), "copy out");
  if (g_sums) CK(hipMemcpyAsync(g_sums, dgsum, n * sizeof(double), back, ctx->stream), "copy out");
  CS(ctx->sync("estimate_nested_extend"));
  if (stc == MLQMC_ENOCONV) ctx->err = msg;
  return stc;
}

int32_t mlqmc_adaptive_decide(int32_t n_levels, int32_t max_levels, const double* Qhat,
                              const double* V, const int64_t* N, const double* cost, double eps,
                              double alpha, int64_t N_max, int32_t* level) {
  if (n_levels < 1 || n_levels > max_levels || !Qhat || !V || !N || !cost || !level ||
      !(eps > 0) || !(alpha > 0) || N_max < 1)
    return -1;
  // variance first: sum_l V_l <= eps^2 / 2 (summed left to right)
  double var = 0.0;
  for (int l = 0; l < n_levels; ++l) var += V[l];
  if (var > eps * eps / 2.0) {
    int best = 0;
    double score = -1.0;
    for (int l = 0; l < n_levels; ++l) {
      const double sc = V[l] / ((double)N[l] * cost[l]);
      if (sc > score) {
        best = l;
        score = sc;
      }
    }
    *level = best;
    return 2 * N[best] > N_max ? MLQMC_ADAPT_BUDGET : MLQMC_ADAPT_DOUBLE;
  }
  // then the bias of the finest level in use: |Qhat_{L-1}| / (2^alpha - 1)
  if (n_levels >= 2) {
    const double bias = std::fabs(Qhat[n_levels - 1]) / (std::pow(2.0, alpha) - 1.0);
    if (bias > eps / std::sqrt(2.0)) {
      if (n_levels >= max_levels) {
        *level = n_levels - 1;
        return MLQMC_ADAPT_LEVELS;
      }
      *level = n_levels;
      return MLQMC_ADAPT_ADD;
    }
  }
  *level = -1;
  return MLQMC_ADAPT_DONE;
}

mlqmc_status mlqmc_estimate_adaptive(mlqmc_ctx* ctx, int32_t max_levels, const mlqmc_level* lv,
                                     int32_t R, const int64_t* z, const double* shifts,
                                     const mlqmc_adaptive_opts* ao, const mlqmc_opts* o,
                                     int32_t* n_levels, int64_t* N_out, double* Q_lr,
                                     double* Qhat, double* V, double* est, int32_t* converged,
                                     int32_t* trace, int32_t trace_cap, int32_t* trace_len) {
  if (!ctx) return MLQMC_EINVAL;
  CS(check_opts(ctx, o));
  if (max_levels < 1 || !lv || !z || !shifts || !ao)
    return ctx->fail(MLQMC_EINVAL, "need max_levels >= 1 and non-NULL inputs");
  if (R < 2) return ctx->fail(MLQMC_EINVAL, "the adaptive rule needs R >= 2 shifts (V_l)");
  if (!n_levels || !N_out || !Q_lr || !Qhat || !V || !est || !converged || !trace_len ||
      (trace_cap > 0 && !trace) || trace_cap < 0)
    return ctx->fail(MLQMC_EINVAL, "NULL output");
  if (o->io_on_device) return ctx->fail(MLQMC_EINVAL, "the adaptive estimate takes host arrays");
  if (!(ao->eps > 0) || !(ao->alpha > 0) || !(ao->gamma > 0) || !is_pow2(ao->N_init) ||
      !is_pow2(ao->N_max) || ao->N_max < ao->N_init || ao->N_max > ((int64_t)1 << 30))
    return ctx->fail(MLQMC_EINVAL, "adaptive options: eps, alpha, gamma > 0; N_init <= N_max "
                                   "powers of two, N_max <= 2^30");
  // cost of one sample (section 4.2, d = 2): s_l h_l^-2 + h_l^-gamma
  std::vector<double> cost(max_levels);
  for (int l = 0; l < max_levels; ++l) {
    const double n = (double)lv[l].n_fine;
    cost[l] = (double)lv[l].s_fine * n * n + std::pow(n, ao->gamma);
  }
  mlqmc_opts oh = *o;
  oh.io_on_device = 0;
  // z [s_all] and shifts [R x s_all] cover every level allowed; a call over
  // the first L levels reads them with row length max_{l<L} s_l
  int s_all = 0;
  for (int l = 0; l < max_levels; ++l) s_all = std::max(s_all, (int)lv[l].s_fine);
  std::vector<double> sh_l;
  auto shifts_for = [&](int L) -> const double* {
    int s_l = 0;
    for (int l = 0; l < L; ++l) s_l = std::max(s_l, (int)lv[l].s_fine);
    sh_l.resize((size_t)R * s_l);
    for (int r = 0; r < R; ++r)
      for (int j = 0; j < s_l; ++j) sh_l[(size_t)r * s_l + j] = shifts[(size_t)r * s_all + j];
    return sh_l.data();
  };
  {
    // every hierarchy the rule may reach is a prefix of a valid nested level list
    const std::vector<int64_t> Nchk(max_levels, ao->N_init);
    CS(check_nested(ctx, max_levels, lv, nullptr, Nchk.data(), R, z, shifts));
  }
  CS(ctx->bind());
  ctx->mem_cap = o->device_mem_cap;
  double* dsum = nullptr;
  CS(ctx->getT("a_sum", (size_t)max_levels * R, &dsum));
  CK(hipMemsetAsync(dsum, 0, (size_t)max_levels * R * sizeof(double), ctx->stream), "memset");
  int L = std::min(2, (int)max_levels);
  std::vector<int64_t> N(L, ao->N_init), Nd(L, 0);
  std::vector<double> q((size_t)max_levels * R), qh(max_levels), vv(max_levels), e2(2);
  bool flagged = false;
  std::string flag_msg;
  int len = 0, act = MLQMC_ADAPT_DONE;
  for (;;) {
    const mlqmc_status st =
        nested_core(ctx, L, lv, Nd.data(), N.data(), R, z, shifts_for(L), &oh, dsum, nullptr,
                    q.data(), qh.data(), vv.data(), e2.data(), nullptr, nullptr);
    if (st == MLQMC_ENOCONV) {
      flagged = true;
      flag_msg = ctx->err;
    } else if (st != MLQMC_OK) {
      return st;
    }
    Nd = N;
    int lev = -1;
    act = mlqmc_adaptive_decide(L, max_levels, qh.data(), vv.data(), N.data(), cost.data(),
                                ao->eps, ao->alpha, ao->N_max, &lev);
    if (len < trace_cap) {
      trace[2 * len] = act;
      trace[2 * len + 1] = lev;
    }
    ++len;
    if (act == MLQMC_ADAPT_DOUBLE) {
      // nested rules: N non-increasing in l, so coarser levels follow
      N[lev] *= 2;
      for (int l = lev - 1; l >= 0; --l) N[l] = std::max(N[l], N[l + 1]);
    } else if (act == MLQMC_ADAPT_ADD) {
      N.push_back(ao->N_init);
      Nd.push_back(0);
      ++L;
    } else {
      break;
    }
  }
  *n_levels = L;
  for (int l = 0; l < L; ++l) {
    N_out[l] = N[l];
    Qhat[l] = qh[l];
    V[l] = vv[l];
    for (int r = 0; r < R; ++r) Q_lr[(size_t)l * R + r] = q[(size_t)l * R + r];
  }
  double vs = 0.0;
  for (int l = 0; l < L; ++l) vs += vv[l];
  est[0] = e2[0];
  est[1] = vs;
  *converged = act == MLQMC_ADAPT_DONE ? 1 : 0;
  *trace_len = len;
  if (flagged) {
    ctx->err = flag_msg;
    return MLQMC_ENOCONV;
  }
  return MLQMC_OK;
}

mlqmc_status mlqmc_set_tuning(mlqmc_ctx* ctx, int32_t n_fine, int32_t prec,
                              int64_t target_blocks) {
  if (!ctx) return MLQMC_EINVAL;
  if (!is_pow2(n_fine) || n_fine < 64 || n_fine > 1024)
    return ctx->fail(MLQMC_EINVAL, "tuning applies to batched meshes 64..1024 (got %d)", n_fine);
  if (prec != MLQMC_FP64 && prec != MLQMC_MIXED)
    return ctx->fail(MLQMC_EINVAL, "unknown precision %d", prec);
  if (target_blocks < 0 || target_blocks > (int64_t)1 << 30)
    return ctx->fail(MLQMC_EINVAL, "target_blocks %lld out of range", (long long)target_blocks);
  if (target_blocks == 0)
    ctx->target_blocks.erase({n_fine, prec});
  else
    ctx->target_blocks[{n_fine, prec}] = target_blocks;
  return MLQMC_OK;
}

mlqmc_status mlqmc_set_timing(mlqmc_ctx* ctx, int32_t cls) {
  if (!ctx) return MLQMC_EINVAL;
  if (cls < MLQMC_K_NONE || cls > MLQMC_K_TG_LDS)
    return ctx->fail(MLQMC_EINVAL, "unknown kernel class");
  ctx->timing_class = cls;
  ctx->t_launches = 0;
  ctx->t_ms = 0.0;
  ctx->t_bytes = 0.0;
  ctx->t_flops = 0.0;
  ctx->ev_used = 0;
  return MLQMC_OK;
}

mlqmc_status mlqmc_get_timing(mlqmc_ctx* ctx, int64_t* launches, double* total_ms,
                              double* model_bytes, double* model_flops) {
  if (!ctx) return MLQMC_EINVAL;
  CS(ctx->bind());
  CS(ctx->sync("timing"));
  if (launches) *launches = ctx->t_launches;
  if (total_ms) *total_ms = ctx->t_ms;
  if (model_bytes) *model_bytes = ctx->t_bytes;
  if (model_flops) *model_flops = ctx->t_flops;
  return MLQMC_OK;
}

}  // extern "C"
