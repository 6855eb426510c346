// C ABI of the lsq2l library: setup (Algorithm 1), the preconditioned CG
// solve on the normal equations (eq. normal), the adjoint solve, and the
// accessors used for validation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace lsq2l {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}
int32_t roundup32(int64_t x) { return (int32_t)((x + TS - 1) / TS * TS); }

// Lanes per row of the SpMV: the largest power of two not above half the
// mean row length, so that a lane takes about two entries of an average row
// (1.67 entries per row of A on the 1000 x 1000 grid: one lane, 5.0 TB/s
// against 4.4 with two; 5 per row of A^T: two lanes, 4.7 TB/s against 4.2,
// 3.6 and 3.4 with four, eight and one)
int pick_group(double avg) {
  int g = 1;
  while (g < 64 && 4 * g <= avg) g *= 2;
  return g;
}

// Device blocks of destroyed handles, kept for later handles on the same
// device: a setup allocates gigabytes in blocks of hundreds of megabytes,
// and allocating or releasing a block of that size costs a sizeable fraction
// of a millisecond.  A request takes the smallest cached block of its device
// that is at least as large and at most a quarter larger.  At most
// CACHE_LIMIT bytes stay cached; lsq2l_release_cache() frees them all, and an
// allocation that fails frees them and tries once more.
struct BlockCache {
  struct Block { void* p; size_t bytes; int dev; };
  static constexpr size_t CACHE_LIMIT = (size_t)32 << 30;
  std::mutex mu;
  std::vector<Block> blocks;
  size_t held = 0;
  void* take(size_t bytes, int dev, size_t* got) {
    std::lock_guard<std::mutex> g(mu);
    int best = -1;
    for (int i = 0; i < (int)blocks.size(); ++i) {
      const Block& b = blocks[i];
      if (b.dev != dev || b.bytes < bytes || b.bytes > bytes + bytes / 4) continue;
      if (best < 0 || b.bytes < blocks[best].bytes) best = i;
    }
    if (best < 0) return nullptr;
    void* p = blocks[best].p;
    *got = blocks[best].bytes;
    held -= *got;
    blocks.erase(blocks.begin() + best);
    return p;
  }
  // the caller has synchronized the work that used the block
  void give(void* p, size_t bytes, int dev) {
    std::lock_guard<std::mutex> g(mu);
    if (held + bytes > CACHE_LIMIT) {
      int cur = 0;
      (void)hipGetDevice(&cur);
      (void)hipSetDevice(dev);
      (void)hipFree(p);
      (void)hipSetDevice(cur);
      return;
    }
    blocks.push_back({p, bytes, dev});
    held += bytes;
  }
  void release() {
    std::lock_guard<std::mutex> g(mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (const Block& b : blocks) {
      (void)hipSetDevice(b.dev);
      (void)hipFree(b.p);
    }
    (void)hipSetDevice(cur);
    blocks.clear();
    held = 0;
  }
};

// never destroyed: device memory goes back with the process
BlockCache& block_cache() {
  static BlockCache* bc = new BlockCache();
  return *bc;
}

// Pinned host buffers for the copies setup reads back from the device (A's
// pattern, A^T's pattern), kept for later setups: a pageable copy runs at a
// sixth of the pinned rate, and pinning fresh memory costs more than the
// copy.  At most PINNED_LIMIT bytes stay cached.
struct PinnedPool {
  struct Buf { void* p; size_t bytes; };
  static constexpr size_t PINNED_LIMIT = (size_t)4 << 30;
  std::mutex mu;
  std::vector<Buf> bufs;
  size_t held = 0;
  void* take(size_t bytes, size_t* got) {
    {
      std::lock_guard<std::mutex> g(mu);
      int best = -1;
      for (int i = 0; i < (int)bufs.size(); ++i)
        if (bufs[i].bytes >= bytes && bufs[i].bytes <= 2 * bytes &&
            (best < 0 || bufs[i].bytes < bufs[best].bytes))
          best = i;
      if (best >= 0) {
        void* p = bufs[best].p;
        *got = bufs[best].bytes;
        held -= *got;
        bufs.erase(bufs.begin() + best);
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    *got = bytes;
    return p;
  }
  void give(void* p, size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    if (held + bytes > PINNED_LIMIT) {
      (void)hipHostFree(p);
      return;
    }
    bufs.push_back({p, bytes});
    held += bytes;
  }
  void release() {
    std::lock_guard<std::mutex> g(mu);
    for (const Buf& b : bufs) (void)hipHostFree(b.p);
    bufs.clear();
    held = 0;
  }
};

PinnedPool& pinned_pool() {
  static PinnedPool* pp = new PinnedPool();
  return *pp;
}

// A pinned host array of count elements from the pool, returned to it when
// the owner goes out of scope (the work that used it has been synchronized).
template <typename T>
struct PinnedArray {
  T* p = nullptr;
  size_t bytes = 0;
  lsq2l_status alloc(int64_t count) {
    const size_t want = (((size_t)std::max<int64_t>(count, 1) * sizeof(T)) + ((1 << 20) - 1)) >> 20 << 20;
    p = (T*)pinned_pool().take(want, &bytes);
    if (!p) {
      set_error("pinned host allocation of " + std::to_string(want) + " bytes failed");
      return LSQ2L_ENOMEM;
    }
    return LSQ2L_OK;
  }
  ~PinnedArray() {
    if (p) pinned_pool().give(p, bytes);
  }
};

}  // namespace
}  // namespace lsq2l

using namespace lsq2l;

struct lsq2l_ctx {
  hipStream_t st = nullptr;
  hipStream_t gst = nullptr;   // stream the PCG iteration graph is captured on
  lsq2l_options opt{};
  double tau = 0.0;
  int S = 1;
  int nsub = 0;
  std::vector<SegDesc> segs_h;
  std::vector<int64_t> seg_row_h, seg_col_h;
  int64_t* d_seg_row = nullptr;
  int64_t* d_seg_col = nullptr;
  DevMatrix M;
  DevMatrix Mi;             // row-permuted copy of A and its transpose for C p = A^T (A p)
  bool row_perm = false;    // Mi is in use
  DevPlan P;
  DevCoarse Cc;
  HostPlan H;
  CoarsePlan CP;
  bool coarse = false;
  int64_t n0tot = 0;        // padded coarse size over all instances
  int64_t n0 = 0;           // true coarse size
  int64_t etiles = 0;
  double *fac = nullptr, *dinv = nullptr, *scale = nullptr, *ctg = nullptr;
  float *fac32 = nullptr, *dinv32 = nullptr;
  float* X32 = nullptr;      // MIXED: FP32 copy of X for the restriction and prolongation
  double *X = nullptr, *W = nullptr, *efac = nullptr, *edinv = nullptr, *einv = nullptr;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *rhs = nullptr, *rold = nullptr;
  double *tm = nullptr, *tm2 = nullptr, *loc = nullptr, *cvec = nullptr, *dvec = nullptr;
  double *partial = nullptr, *partial2 = nullptr, *xwork = nullptr;
  double *bsave = nullptr, *xsave = nullptr;
  double *bal_u = nullptr, *bal_w = nullptr;   // balanced form: two n-vectors
  bool have_solution = false;
  Scalars sc{};
  int32_t* status = nullptr;
  int32_t* h_done = nullptr;      // pinned
  double* h_rn2 = nullptr;        // pinned
  double* h_r0n2 = nullptr;       // pinned
  std::vector<int32_t> p_h;
  int max_p = 0;
  lsq2l_setup_info info{};
  struct DevBlock { void* p; size_t bytes; int dev; };
  std::vector<DevBlock> dev_allocs;
  std::vector<void*> host_allocs;

  // Device memory of the handle: requests up to ARENA_SMALL bytes are carved
  // (256-byte aligned) from ARENA_CHUNK-sized allocations, larger ones get
  // their own; everything is released when the handle is destroyed.
  static constexpr size_t ARENA_CHUNK = (size_t)256 << 20, ARENA_SMALL = (size_t)64 << 20;
  char* arena_cur = nullptr;
  size_t arena_used = 0;
  lsq2l_status raw_alloc(void** v, size_t bytes) {
    int dev = 0;
    LSQ2L_HIP_TRY(hipGetDevice(&dev));
    size_t got = 0;
    if ((*v = block_cache().take(bytes, dev, &got)) != nullptr) {
      dev_allocs.push_back({*v, got, dev});
      return LSQ2L_OK;
    }
    hipError_t e = hipMalloc(v, bytes);
    if (e != hipSuccess) {
      block_cache().release();
      e = hipMalloc(v, bytes);
    }
    if (e != hipSuccess) {
      set_error("device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
      return LSQ2L_ENOMEM;
    }
    dev_allocs.push_back({*v, bytes, dev});
    return LSQ2L_OK;
  }
  template <typename T>
  lsq2l_status dalloc(T** ptr, int64_t count) {
    *ptr = nullptr;
    if (count <= 0) return LSQ2L_OK;
    const size_t bytes = ((size_t)count * sizeof(T) + 255) / 256 * 256;
    void* v = nullptr;
    if (bytes > ARENA_SMALL) {
      lsq2l_status s = raw_alloc(&v, bytes);
      if (s != LSQ2L_OK) return s;
    } else {
      if (!arena_cur || arena_used + bytes > ARENA_CHUNK) {
        lsq2l_status s = raw_alloc(&v, ARENA_CHUNK);
        if (s != LSQ2L_OK) return s;
        arena_cur = (char*)v;
        arena_used = 0;
      }
      v = arena_cur + arena_used;
      arena_used += bytes;
    }
    *ptr = (T*)v;
    return LSQ2L_OK;
  }
  template <typename T>
  lsq2l_status halloc(T** ptr, int64_t count) {
    void* v = nullptr;
    hipError_t e = hipHostMalloc(&v, (size_t)std::max<int64_t>(count, 1) * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) { set_error("pinned host allocation failed"); return LSQ2L_ENOMEM; }
    host_allocs.push_back(v);
    *ptr = (T*)v;
    return LSQ2L_OK;
  }
  template <typename T>
  lsq2l_status upload(T** dst, const std::vector<T>& src) {
    lsq2l_status s = dalloc(dst, (int64_t)src.size());
    if (s != LSQ2L_OK) return s;
    if (!src.empty()) LSQ2L_HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return LSQ2L_OK;
  }
  ~lsq2l_ctx() {
    if (st) (void)hipStreamSynchronize(st);
    else (void)hipDeviceSynchronize();
    if (gst) (void)hipStreamDestroy(gst);
    for (const DevBlock& b : dev_allocs) block_cache().give(b.p, b.bytes, b.dev);
    for (void* v : host_allocs) (void)hipHostFree(v);
  }
};

#define TRY(expr)                             \
  do {                                        \
    lsq2l_status _s = (expr);                 \
    if (_s != LSQ2L_OK) return _s;            \
  } while (0)

namespace {

lsq2l_status validate_csr(int32_t m, int32_t n, const int32_t* rp, const int32_t* ci, int64_t nnz) {
  if (rp[0] != 0) { set_error("rowptr[0] must be 0"); return LSQ2L_EINVAL; }
  // rows checked in parallel blocks, first every row's extent (so that the
  // column pass reads inside ci), then the columns; the first failing row of
  // the first failing pass is reported
  const unsigned nth = m < (1 << 16) ? 1u : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<int32_t> bad_row(nth, INT32_MAX);
  std::vector<int> bad_kind(nth, 0);
  auto run = [&](auto&& fn) {
    if (nth == 1) {
      fn(0u);
    } else {
      std::vector<std::thread> pool;
      for (unsigned t = 0; t < nth; ++t) pool.emplace_back(fn, t);
      for (auto& th : pool) th.join();
    }
  };
  auto rows_of = [&](unsigned t, int32_t& r0, int32_t& r1) {
    r0 = (int32_t)((int64_t)m * t / nth);
    r1 = (int32_t)((int64_t)m * (t + 1) / nth);
  };
  run([&](unsigned t) {
    int32_t r0, r1;
    rows_of(t, r0, r1);
    for (int32_t r = r0; r < r1; ++r)
      if (rp[r + 1] < rp[r] || rp[r + 1] > nnz) { bad_row[t] = r; bad_kind[t] = 1; return; }
  });
  bool extents_ok = true;
  for (unsigned t = 0; t < nth; ++t) extents_ok = extents_ok && !bad_kind[t];
  if (extents_ok)
    run([&](unsigned t) {
      int32_t r0, r1;
      rows_of(t, r0, r1);
      for (int32_t r = r0; r < r1; ++r)
        for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
          int kind = 0;
          if (ci[e] < 0 || ci[e] >= n) kind = 2;
          else if (e > rp[r] && ci[e] <= ci[e - 1]) kind = 3;
          if (kind) { bad_row[t] = r; bad_kind[t] = kind; return; }
        }
    });
  for (unsigned t = 0; t < nth; ++t) {
    if (!bad_kind[t]) continue;
    const std::string r = std::to_string(bad_row[t]);
    if (bad_kind[t] == 1) set_error("rowptr is not monotone (or exceeds nnz) at row " + r);
    else if (bad_kind[t] == 2) set_error("column index out of range in row " + r);
    else set_error("columns not strictly increasing in row " + r);
    return LSQ2L_EINVAL;
  }
  return LSQ2L_OK;
}

void spmv_it_A(lsq2l_ctx* c, const double* x, double* y);
void spmv_it_AT(lsq2l_ctx* c, const double* y, double* x);

// z = Q r = R_0^T E^{-1} R_0 r (restriction, symmetric E^{-1} product, prolongation)
void apply_Q(lsq2l_ctx* c, const double* r, double* z) {
  const hipStream_t st = c->st;
  if (c->X32) {
    launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X32, r, c->cvec);
    launch_einv_gemv(st, c->n0tot, c->S, c->Cc, c->einv, c->cvec, c->dvec);
    launch_scatter_local(st, c->M.n, c->P, c->scale, nullptr, c->X32, c->dvec, z);
  } else {
    launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X, r, c->cvec);
    launch_einv_gemv(st, c->n0tot, c->S, c->Cc, c->einv, c->cvec, c->dvec);
    launch_scatter_local(st, c->M.n, c->P, c->scale, nullptr, c->X, c->dvec, z);
  }
}

// z = M_ASM r = sum_i R_i^T C_ii^{-1} R_i r (eq. one_level_schwarz)
void apply_one_level(lsq2l_ctx* c, const double* r, double* z) {
  const hipStream_t st = c->st;
  launch_gather_local(st, c->nsub, c->P, c->scale, r, c->loc);
  if (c->opt.precision == LSQ2L_MIXED)
    launch_local_solve_f32(st, c->nsub, c->P, c->fac32, c->dinv32, c->loc);
  else
    launch_local_solve(st, c->nsub, c->P, c->fac, c->dinv, c->loc);
  if (c->X32) launch_scatter_local(st, c->M.n, c->P, c->scale, c->loc, c->X32, nullptr, z);
  else launch_scatter_local(st, c->M.n, c->P, c->scale, c->loc, c->X, nullptr, z);
}

// Balanced form (eq. balanced) with M_ASM as the first level:
// M r = Q r + (I - Q C) M_ASM (I - C Q) r, evaluated as
//   u = Q r;  y = M_ASM (r - C u);  z = y + Q (r - C y),
// C applied as A^T (A .).  Two coarse corrections, four SpMVs, one set of
// local solves per application.
void apply_M_balanced(lsq2l_ctx* c, const double* r, double* z) {
  const hipStream_t st = c->st;
  const int64_t n = c->M.n;
  if (z == r) {                 // r is read again after z is first written
    launch_copy(st, n, r, c->rold);
    r = c->rold;
  }
  apply_Q(c, r, c->bal_u);
  spmv_it_A(c, c->bal_u, c->tm2);
  spmv_it_AT(c, c->tm2, c->bal_w);
  launch_sub(st, n, r, c->bal_w, c->bal_w);            // (I - C Q) r
  apply_one_level(c, c->bal_w, z);                      // y
  spmv_it_A(c, z, c->tm2);
  spmv_it_AT(c, c->tm2, c->bal_w);
  launch_sub(st, n, r, c->bal_w, c->bal_w);            // r - C y
  apply_Q(c, c->bal_w, c->bal_u);
  launch_add(st, n, z, c->bal_u, z);
}

// z = M r: local solves (eq. one_level_schwarz) plus the coarse correction
// R_0^T E^{-1} R_0 r (eq. two_level_schwarz), or the balanced form.
void apply_M(lsq2l_ctx* c, const double* r, double* z) {
  if (c->opt.variant == LSQ2L_BALANCED) {
    if (c->coarse) apply_M_balanced(c, r, z);
    else apply_one_level(c, r, z);
    return;
  }
  const hipStream_t st = c->st;
  launch_gather_local(st, c->nsub, c->P, c->scale, r, c->loc);
  if (c->opt.precision == LSQ2L_MIXED)
    launch_local_solve_f32(st, c->nsub, c->P, c->fac32, c->dinv32, c->loc);
  else
    launch_local_solve(st, c->nsub, c->P, c->fac, c->dinv, c->loc);
  const bool x32 = c->X32 != nullptr;
  if (c->coarse) {
    if (x32) launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X32, r, c->cvec);
    else launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X, r, c->cvec);
    launch_einv_gemv(st, c->n0tot, c->S, c->Cc, c->einv, c->cvec, c->dvec);
  }
  if (x32) launch_scatter_local(st, c->M.n, c->P, c->scale, c->loc, c->X32, c->coarse ? c->dvec : nullptr, z);
  else launch_scatter_local(st, c->M.n, c->P, c->scale, c->loc, c->X, c->coarse ? c->dvec : nullptr, z);
}

// C p = A^T (A p) inside the iteration.  A p never leaves the library, so it
// may be formed with a row-permuted copy of A: C = A^T A is the same for any
// row order of A.
void spmv_it_A(lsq2l_ctx* c, const double* x, double* y) {
  const DevMatrix& M = c->row_perm ? c->Mi : c->M;
  launch_spmv(c->st, M.m, M.rowptr, M.colind, M.vals, x, y, M.spmv_group);
}
void spmv_it_AT(lsq2l_ctx* c, const double* y, double* x) {
  const DevMatrix& M = c->row_perm ? c->Mi : c->M;
  launch_spmv(c->st, M.n, M.trowptr, M.trow, M.tvals, y, x, M.spmvt_group);
}

void spmv_A(lsq2l_ctx* c, const double* x, double* y) {
  launch_spmv(c->st, c->M.m, c->M.rowptr, c->M.colind, c->M.vals, x, y, c->M.spmv_group);
}
void spmv_AT(lsq2l_ctx* c, const double* y, double* x) {
  launch_spmv(c->st, c->M.n, c->M.trowptr, c->M.trow, c->M.tvals, y, x, c->M.spmvt_group);
}

lsq2l_status read_flags(lsq2l_ctx* c) {
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_done, c->sc.done, sizeof(int32_t) * c->S, hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_rn2, c->sc.rn2, sizeof(double) * c->S, hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_r0n2, c->sc.r0n2, sizeof(double) * c->S, hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  return LSQ2L_OK;
}

// PCG on C x = rhs (x_0 = 0), C = A^T A applied as A^T (A p).  x is written.
// One PCG iteration as a HIP graph: both SpMVs, alpha, the x and r update,
// the residual norm (which sets the per-instance done flags), M r, beta and
// the direction update, in the order of the loop in pcg().  The graph is
// captured on an internal stream (the handle's stream may be the null
// stream) and launched on the handle's stream.  It holds kernel nodes only.
lsq2l_status capture_iteration(lsq2l_ctx* c, double* x, double tol2, hipGraphExec_t* out) {
  *out = nullptr;
  if (!c->gst) LSQ2L_HIP_TRY(hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking));
  const hipStream_t saved = c->st;
  const int S = c->S;
  const int64_t n = c->M.n;
  const int flexible = c->opt.flexible;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    c->st = c->gst;
    const hipStream_t st = c->st;
    spmv_it_A(c, c->p, c->tm);
    spmv_it_AT(c, c->tm, c->q);
    launch_dot(st, S, c->d_seg_col, c->p, c->q, c->partial);
    launch_scalar(st, OP_ALPHA, S, c->partial, nullptr, c->sc, tol2, flexible);
    if (flexible) launch_copy(st, n, c->r, c->rold);
    launch_axpy_xr(st, n, S, c->d_seg_col, c->sc.alpha, c->p, c->q, x, c->r);
    launch_dot(st, S, c->d_seg_col, c->r, c->r, c->partial);
    launch_scalar(st, OP_RNORM, S, c->partial, nullptr, c->sc, tol2, flexible);
    apply_M(c, c->r, c->z);
    launch_dot(st, S, c->d_seg_col, c->r, c->z, c->partial);
    if (flexible) launch_dot(st, S, c->d_seg_col, c->rold, c->z, c->partial2);
    launch_scalar(st, OP_BETA, S, c->partial, flexible ? c->partial2 : nullptr, c->sc, tol2, flexible);
    launch_xpby(st, n, S, c->d_seg_col, c->sc.beta, c->z, c->p);
    c->st = saved;
    e = hipStreamEndCapture(c->gst, &g);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    set_error(std::string("capturing the PCG iteration: ") + hipGetErrorString(e));
    return LSQ2L_EHIP;
  }
  return LSQ2L_OK;
}

lsq2l_status pcg(lsq2l_ctx* c, double* x, int* its_out, int* restarts_out, double* relres_true,
                 double* relres_rec) {
  const hipStream_t st = c->st;
  const int S = c->S;
  const int64_t n = c->M.n;
  const double tol2 = c->opt.tol * c->opt.tol;
  const int flexible = c->opt.flexible;
  launch_fill(st, n, 0.0, x);
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->r, c->rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  launch_dot(st, S, c->d_seg_col, c->r, c->r, c->partial);
  launch_scalar(st, OP_R0, S, c->partial, nullptr, c->sc, tol2, flexible);
  int its = 0, restarts = 0;
  bool breakdown = false;
  while (true) {
    apply_M(c, c->r, c->z);
    launch_dot(st, S, c->d_seg_col, c->r, c->z, c->partial);
    launch_scalar(st, OP_RHO_INIT, S, c->partial, nullptr, c->sc, tol2, flexible);
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->p, c->z, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    TRY(read_flags(c));
    bool all_done = true;
    for (int s = 0; s < S; ++s) all_done &= (c->h_done[s] != 0);
    // graph replay: the iteration runs whole (M r and the direction update
    // after a converged residual norm change neither x nor r)
    hipGraphExec_t gexec = nullptr;
    if (c->opt.use_graph && !all_done) TRY(capture_iteration(c, x, tol2, &gexec));
    while (gexec && !all_done && its < c->opt.max_it) {
      const hipError_t ge = hipGraphLaunch(gexec, st);
      if (ge != hipSuccess) {
        (void)hipGraphExecDestroy(gexec);
        set_error(std::string("launching the PCG iteration graph: ") + hipGetErrorString(ge));
        return LSQ2L_EHIP;
      }
      ++its;
      if (its % std::max(1, c->opt.check_every) == 0 || its >= c->opt.max_it) {
        const lsq2l_status fs = read_flags(c);
        if (fs != LSQ2L_OK) { (void)hipGraphExecDestroy(gexec); return fs; }
        all_done = true;
        for (int s = 0; s < S; ++s) {
          all_done &= (c->h_done[s] != 0);
          breakdown |= (c->h_done[s] == 2);
        }
      }
    }
    if (gexec) (void)hipGraphExecDestroy(gexec);
    while (!all_done && its < c->opt.max_it) {
      spmv_it_A(c, c->p, c->tm);
      spmv_it_AT(c, c->tm, c->q);
      launch_dot(st, S, c->d_seg_col, c->p, c->q, c->partial);
      launch_scalar(st, OP_ALPHA, S, c->partial, nullptr, c->sc, tol2, flexible);
      if (flexible) LSQ2L_HIP_TRY(hipMemcpyAsync(c->rold, c->r, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      launch_axpy_xr(st, n, S, c->d_seg_col, c->sc.alpha, c->p, c->q, x, c->r);
      launch_dot(st, S, c->d_seg_col, c->r, c->r, c->partial);
      launch_scalar(st, OP_RNORM, S, c->partial, nullptr, c->sc, tol2, flexible);
      ++its;
      if (its % std::max(1, c->opt.check_every) == 0 || its >= c->opt.max_it) {
        TRY(read_flags(c));
        all_done = true;
        for (int s = 0; s < S; ++s) {
          all_done &= (c->h_done[s] != 0);
          breakdown |= (c->h_done[s] == 2);
        }
        if (all_done) break;
      }
      apply_M(c, c->r, c->z);
      launch_dot(st, S, c->d_seg_col, c->r, c->z, c->partial);
      if (flexible) launch_dot(st, S, c->d_seg_col, c->rold, c->z, c->partial2);
      launch_scalar(st, OP_BETA, S, c->partial, flexible ? c->partial2 : nullptr, c->sc, tol2, flexible);
      launch_xpby(st, n, S, c->d_seg_col, c->sc.beta, c->z, c->p);
    }
    // true residual rhs - A^T A x
    spmv_it_A(c, x, c->tm);
    spmv_it_AT(c, c->tm, c->q);
    launch_sub(st, n, c->rhs, c->q, c->q);
    launch_dot(st, S, c->d_seg_col, c->q, c->q, c->partial);
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_done, c->sc.done, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
    std::vector<double> part((size_t)S * RED_BLOCKS);
    LSQ2L_HIP_TRY(hipMemcpyAsync(part.data(), c->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_rn2, c->sc.rn2, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_r0n2, c->sc.r0n2, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));
    bool all_ok = true;
    for (int s = 0; s < S; ++s) {
      double t = 0.0;
      for (int b = 0; b < RED_BLOCKS; ++b) t += part[(size_t)s * RED_BLOCKS + b];
      const double r0 = c->h_r0n2[s];
      relres_true[s] = r0 > 0 ? std::sqrt(t / r0) : 0.0;
      relres_rec[s] = r0 > 0 ? std::sqrt(c->h_rn2[s] / r0) : 0.0;
      if (c->h_done[s] == 2) breakdown = true;
      if (!(relres_true[s] <= c->opt.tol)) all_ok = false;
    }
    if (all_ok || breakdown || restarts == 3 || its >= c->opt.max_it) break;
    // restart from the true residual; converged instances re-check immediately
    ++restarts;
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->r, c->q, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_dot(st, S, c->d_seg_col, c->r, c->r, c->partial);
    LSQ2L_HIP_TRY(hipMemsetAsync(c->sc.done, 0, sizeof(int32_t) * S, st));
    launch_scalar(st, OP_RNORM, S, c->partial, nullptr, c->sc, tol2, flexible);
  }
  *its_out = its;
  *restarts_out = restarts;
  if (breakdown) { set_error("PCG breakdown (non-positive curvature or non-finite value)"); return LSQ2L_PCG_BREAKDOWN; }
  for (int s = 0; s < S; ++s)
    if (!(relres_true[s] <= c->opt.tol)) {
      set_error("PCG did not reach the tolerance within max_it iterations");
      return LSQ2L_NOT_CONVERGED;
    }
  return LSQ2L_OK;
}

// The overlap maps of the plan, built on a host thread while the device
// assembles, factors and selects; joined before their first use.
struct MapsJob {
  std::thread th;
  bool ok = true;
  std::string err;
  void start(int32_t m, int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* part,
             HostPlan* H) {
    th = std::thread([this, m, n, rp, ci, part, H]() { ok = plan_maps(m, n, rp, ci, part, *H, err); });
  }
  bool join() {
    if (th.joinable()) th.join();
    return ok;
  }
  ~MapsJob() { if (th.joinable()) th.join(); }
};

// Everything after the matrix is resident in the handle (c->M rowptr/colind/vals).
// a thread joined on every exit from the scope that owns it
struct JoiningThread {
  std::thread t;
  ~JoiningThread() {
    if (t.joinable()) t.join();
  }
};

lsq2l_status setup_core(lsq2l_ctx* c, const int32_t* rp, const int32_t* ci,
                        const std::vector<int32_t>& part, int32_t nparts,
                        const std::vector<int32_t>& seg_of_part) {
  const hipStream_t st = c->st;
  const int32_t m = c->M.m, n = c->M.n;
  const int64_t nnz = c->M.nnz;
  auto t_all = clk::now();
  auto t0 = clk::now();
  // --- transpose and index sets
  // A^T on the device; the planner reads its pattern back
  PinnedArray<int32_t> trp, tcol;
  TRY(trp.alloc((int64_t)n + 1));
  TRY(tcol.alloc(nnz));
  int32_t *keys = nullptr, *vals = nullptr, *rows = nullptr;
  char* temp = nullptr;
  const size_t tb = transpose_temp_bytes(nnz, n);
  {
    TRY(c->dalloc(&c->M.trowptr, (int64_t)n + 1));
    TRY(c->dalloc(&c->M.trow, nnz));
    TRY(c->dalloc(&c->M.tperm, nnz));
    TRY(c->dalloc(&keys, nnz));
    TRY(c->dalloc(&vals, nnz));
    TRY(c->dalloc(&rows, nnz));
    TRY(c->dalloc(&temp, (int64_t)std::max<size_t>(tb, 1)));
    LSQ2L_HIP_TRY(launch_transpose(st, m, n, nnz, c->M.rowptr, c->M.colind, c->M.trowptr, c->M.trow,
                                   c->M.tperm, keys, vals, rows, temp, tb));
    LSQ2L_HIP_TRY(hipMemcpyAsync(trp.p, c->M.trowptr, ((size_t)n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (nnz) LSQ2L_HIP_TRY(hipMemcpyAsync(tcol.p, c->M.trow, (size_t)nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  }
  TRY(c->dalloc(&c->M.tvals, nnz));
  launch_gather_values(st, nnz, c->M.tperm, c->M.vals, c->M.tvals);
  c->M.spmv_group = pick_group(m ? (double)nnz / m : 1.0);
  c->M.spmvt_group = pick_group(n ? (double)nnz / n : 1.0);
  // Row order of the copy used for C p = A^T (A p), found on a host thread
  // while the device assembles, factors and selects (see row_order).
  RowOrder ro;
  JoiningThread ro_thread{std::thread([&ro, m, n, rp, ci]() { row_order(m, n, rp, ci, ro); })};
  std::string err;
  if (!plan_build(m, n, rp, ci, trp.p, tcol.p, part.data(), nparts, seg_of_part, c->H, err)) {
    set_error(err);
    return LSQ2L_EINVAL;
  }
  HostPlan& H = c->H;
  c->nsub = nparts;
  MapsJob maps;
  maps.start(m, n, rp, ci, part.data(), &H);
  TRY(c->upload(&c->P.subs, H.subs));
  TRY(c->upload(&c->P.omega, H.omega));
  TRY(c->upload(&c->P.xi, H.xi));
  TRY(c->upload(&c->P.part, part));
  TRY(c->upload(&c->P.locown, H.locown));
  TRY(c->upload(&c->P.tileF, H.tileF));
  TRY(c->upload(&c->P.tileOff, H.tileOff));
  for (const SubDesc& d : H.subs) c->P.max_np = std::max(c->P.max_np, (int)d.np);
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  c->info.t_plan_ms = ms_since(t0);
  // --- local matrices
  t0 = clk::now();
  TRY(c->dalloc(&c->fac, H.total_fac));
  TRY(c->dalloc(&c->dinv, H.total_dinv));
  TRY(c->dalloc(&c->scale, H.total_loc));
  TRY(c->dalloc(&c->ctg, H.total_g));
  TRY(c->dalloc(&c->status, 8));
  LSQ2L_HIP_TRY(hipMemsetAsync(c->status, 0, 8 * sizeof(int32_t), st));
  LSQ2L_HIP_TRY(hipMemsetAsync(c->fac, 0, H.total_fac * sizeof(double), st));
  if (H.total_g) LSQ2L_HIP_TRY(hipMemsetAsync(c->ctg, 0, H.total_g * sizeof(double), st));
  launch_assemble(st, nparts, c->P, c->M, c->fac, c->ctg);
  launch_equilibrate(st, nparts, c->P, c->fac, c->ctg, c->scale);
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  c->info.t_assemble_ms = ms_since(t0);
  // --- batched local Cholesky
  t0 = clk::now();
  launch_chol_local(st, nparts, c->P, c->fac, c->dinv, c->status);
  int32_t hstat[8];
  LSQ2L_HIP_TRY(hipMemcpyAsync(hstat, c->status, sizeof(hstat), hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  c->info.t_factor_ms = ms_since(t0);
  if (hstat[0] != 0) {
    set_error("local Cholesky breakdown in subdomain " + std::to_string(hstat[0] - 1));
    return LSQ2L_CHOL_BREAKDOWN;
  }
  // --- coarse space
  c->p_h.assign(nparts, 0);
  c->coarse = false;
  c->n0 = 0;
  c->n0tot = 0;
  t0 = clk::now();
  if (c->opt.variant != LSQ2L_ONE_LEVEL) {
    double *Tg = nullptr, *work = nullptr, *sig = nullptr;
    int32_t* pc = nullptr;
    TRY(c->dalloc(&Tg, H.total_g));
    TRY(c->dalloc(&work, SEL_WORK_MATS * H.total_g));
    TRY(c->dalloc(&sig, H.total_loc));
    TRY(c->dalloc(&pc, nparts + 1));
    if (H.total_g) LSQ2L_HIP_TRY(hipMemsetAsync(work, 0, SEL_WORK_MATS * H.total_g * sizeof(double), st));
    LSQ2L_HIP_TRY(hipMemsetAsync(pc, 0, (nparts + 1) * sizeof(int32_t), st));
    launch_gamma_T(st, nparts, c->P, c->fac, Tg);
    launch_select(st, nparts, c->P, c->ctg, Tg, work, c->tau, c->opt.nev_max, pc, sig);
    std::vector<int32_t> ph(nparts + 1);
    LSQ2L_HIP_TRY(hipMemcpyAsync(ph.data(), pc, (nparts + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));
    if (ph[nparts] != 0) {
      set_error(ph[nparts] == 2 ? "interface larger than the eigensolver limit (1024)"
                                : "non-finite entries in a coarse eigenproblem");
      return LSQ2L_EINVAL;
    }
    CoarsePlan& CP = c->CP;
    if (!maps.join()) { set_error(maps.err); return LSQ2L_EINVAL; }
    plan_coarse(H, c->S, m, ph, CP);
    c->segs_h = CP.segs;
    for (int i = 0; i < nparts; ++i) c->p_h[i] = ph[i];
    c->max_p = *std::max_element(ph.begin(), ph.begin() + nparts);
    c->n0 = CP.n0;
    c->n0tot = CP.n0tot;
    c->etiles = CP.etiles;
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->P.subs, H.subs.data(), H.subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice, st));
    TRY(c->upload(&c->Cc.segs, c->segs_h));
    if (c->n0 > 0) {
      c->coarse = true;
      TRY(c->dalloc(&c->X, CP.xtot));
      TRY(c->dalloc(&c->W, CP.wtot));
      launch_coarse_X(st, nparts, c->P, c->fac, c->dinv, c->scale, work, sig, c->X);
      launch_coarse_W(st, nparts, c->P, c->M, c->X, c->W);
      if (c->opt.precision == LSQ2L_MIXED) {
        // E below is built from the FP64 X; the per-iteration restriction
        // and prolongation both read the same rounded copy, so the coarse
        // term R_0^T E^{-1} R_0 stays symmetric positive semidefinite
        TRY(c->dalloc(&c->X32, CP.xtot));
        launch_to_float(st, CP.xtot, c->X, c->X32);
      }
      LSQ2L_HIP_TRY(hipStreamSynchronize(st));
      c->info.t_eigen_ms = ms_since(t0);
      t0 = clk::now();
      TRY(c->upload(&c->Cc.pairs, CP.pairs));
      TRY(c->upload(&c->Cc.pair_rows, CP.pair_rows));
      TRY(c->upload(&c->Cc.eF, CP.eF));
      TRY(c->upload(&c->Cc.eOff, CP.eOff));
      TRY(c->upload(&c->Cc.e_seg_of_tile, CP.seg_of_tile));
      int64_t* d_pad = nullptr;
      TRY(c->upload(&d_pad, CP.pad_idx));
      TRY(c->dalloc(&c->efac, CP.efac_tiles * TT));
      TRY(c->dalloc(&c->edinv, c->etiles * TT));
      LSQ2L_HIP_TRY(hipMemsetAsync(c->efac, 0, CP.efac_tiles * TT * sizeof(double), st));
      launch_set_values(st, (int64_t)CP.pad_idx.size(), d_pad, 1.0, c->efac);
      {
        int32_t* d_items = nullptr;
        TRY(c->upload(&d_items, CP.items));
        c->Cc.e_items = (int4*)d_items;
      }
      launch_coarse_E(st, (int)(CP.items.size() / 4), c->P, c->Cc, c->W, c->efac);
      // right-looking Cholesky of E, one tile column per launch, each launch
      // also applying the previous column to the tiles right of the current
      // one (rows of column J - 1 below J: its list without row J)
      TRY(c->upload(&c->Cc.erows, CP.erows));
      TRY(c->upload(&c->Cc.eptr, CP.eptr));
      int32_t* d_erows = c->Cc.erows;
      for (int64_t J = 0; J < c->etiles; ++J) {
        const int nr = (int)(CP.eptr[J + 1] - CP.eptr[J]);
        int64_t p0 = 0, p1 = 0;
        if (J > 0) {
          p0 = CP.eptr[J - 1];
          p1 = CP.eptr[J];
          if (p0 < p1 && CP.erows[p0] == J) ++p0;
        }
        launch_echol_step(st, c->Cc, (int)J, d_erows + CP.eptr[J], nr, d_erows + p0, (int)(p1 - p0),
                          c->efac, c->edinv, c->status + 1);
      }
      TRY(c->dalloc(&c->einv, CP.einv_tot));
      TRY(c->dalloc(&c->Cc.e_part, CP.einv_tot / TS));
      {
        // chunks of the lower block triangle of E^{-1} for the coarse solve:
        // up to ESYM_ROWTILES row tiles of one tile column each
        std::vector<int32_t> ch, cptr(1, 0);
        for (const SegDesc& sg : CP.segs)
          for (int64_t cc = 0; cc < sg.etiles; ++cc) {
            for (int64_t i0 = cc; i0 < sg.etiles; i0 += ESYM_ROWTILES) {
              ch.push_back((int32_t)(sg.etile0 + cc));
              ch.push_back((int32_t)i0);
              ch.push_back((int32_t)std::min<int64_t>(ESYM_ROWTILES, sg.etiles - i0));
              ch.push_back(0);
            }
            cptr.push_back((int32_t)(ch.size() / 4));
          }
        c->Cc.e_nchunks = (int)(ch.size() / 4);
        int32_t* d_ch = nullptr;
        TRY(c->upload(&d_ch, ch));
        c->Cc.e_chunks = (int4*)d_ch;
        TRY(c->upload(&c->Cc.e_chunk_ptr, cptr));
        TRY(c->dalloc(&c->Cc.e_u, (int64_t)c->Cc.e_nchunks * TS));
      }
      {
        // column blocks of E^{-1} onto one workgroup per compute unit, longest
        // first to the least loaded (block c of an instance with nt tile rows
        // costs 2 (nt - c) + 1 tile-row steps)
        int ncu = 0;
        LSQ2L_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, 0));
        const int nbins = (int)std::min<int64_t>(std::max(1, ncu), c->etiles);
        std::vector<std::pair<int64_t, int32_t>> items;
        for (const SegDesc& sg : CP.segs)
          for (int64_t cc = 0; cc < sg.etiles; ++cc)
            items.push_back({2 * (sg.etiles - cc) + 1, (int32_t)(sg.etile0 + cc)});
        std::stable_sort(items.begin(), items.end(),
                         [](const auto& x, const auto& y) { return x.first > y.first; });
        std::vector<std::vector<int32_t>> bins(nbins);
        std::vector<std::pair<int64_t, int>> load;   // min-heap of (load, bin)
        for (int bb = 0; bb < nbins; ++bb) load.push_back({0, bb});
        auto cmp = [](const auto& x, const auto& y) { return x > y; };
        for (const auto& it : items) {
          std::pop_heap(load.begin(), load.end(), cmp);
          auto& top = load.back();
          bins[top.second].push_back(it.second);
          top.first += it.first;
          std::push_heap(load.begin(), load.end(), cmp);
        }
        // workgroup w runs on XCD w % 8: lists ordered by their first column
        // block go to the XCDs in runs, so that blocks close in the triangle
        // (which read the same factor rows at about the same time) share an
        // L2
        std::vector<int> order(nbins);
        for (int b = 0; b < nbins; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
          const int32_t fx = bins[x].empty() ? INT32_MAX : bins[x][0];
          const int32_t fy = bins[y].empty() ? INT32_MAX : bins[y][0];
          return fx < fy;
        });
        std::vector<int> slot(nbins);
        const int G = nbins / 8;
        for (int k = 0; k < nbins; ++k) slot[k] = (nbins % 8 == 0) ? (k % G) * 8 + k / G : k;
        std::vector<std::vector<int32_t>> placed(nbins);
        for (int k = 0; k < nbins; ++k) placed[slot[k]] = bins[order[k]];
        std::vector<int32_t> bptr(1, 0), bcols;
        for (const auto& bl : placed) {
          bcols.insert(bcols.end(), bl.begin(), bl.end());
          bptr.push_back((int32_t)bcols.size());
        }
        TRY(c->upload(&c->Cc.einv_bin_ptr, bptr));
        TRY(c->upload(&c->Cc.einv_bin_cols, bcols));
        double *efacT = nullptr, *edinvT = nullptr;
        TRY(c->dalloc(&efacT, CP.efac_tiles * TT));
        TRY(c->dalloc(&edinvT, c->etiles * TT));
        launch_tile_transpose(st, CP.efac_tiles, c->efac, efacT);
        launch_tile_transpose(st, c->etiles, c->edinv, edinvT);
        launch_einv(st, nbins, c->Cc, c->efac, c->edinv, efacT, edinvT, c->einv);
      }
      TRY(c->dalloc(&c->cvec, c->n0tot));
      TRY(c->dalloc(&c->dvec, c->n0tot));
      LSQ2L_HIP_TRY(hipMemsetAsync(c->cvec, 0, c->n0tot * sizeof(double), st));
      LSQ2L_HIP_TRY(hipMemcpyAsync(hstat, c->status, sizeof(hstat), hipMemcpyDeviceToHost, st));
      LSQ2L_HIP_TRY(hipStreamSynchronize(st));
      if (hstat[1] != 0) {
        set_error("coarse Cholesky breakdown at tile " + std::to_string(hstat[1] - 1));
        return LSQ2L_CHOL_BREAKDOWN;
      }
      c->info.t_coarse_ms = ms_since(t0);
    } else {
      LSQ2L_HIP_TRY(hipStreamSynchronize(st));
      c->info.t_eigen_ms = ms_since(t0);
    }
  }
  // --- overlap maps (owners of every column, for the scatter)
  if (!maps.join()) { set_error(maps.err); return LSQ2L_EINVAL; }
  TRY(c->upload(&c->P.own_ptr, H.own_ptr));
  TRY(c->upload(&c->P.own_pos, H.own_pos));
  // --- mixed precision copy of the local factors
  if (c->opt.precision == LSQ2L_MIXED) {
    TRY(c->dalloc(&c->fac32, H.total_fac));
    TRY(c->dalloc(&c->dinv32, H.total_dinv));
    launch_to_float(st, H.total_fac, c->fac, c->fac32);
    launch_to_float(st, H.total_dinv, c->dinv, c->dinv32);
  }
  // --- row-permuted iteration copy of A
  ro_thread.t.join();
  c->row_perm = ro.use;
  if (c->row_perm) {
    DevMatrix& Mi = c->Mi;
    Mi.m = m;
    Mi.n = n;
    Mi.nnz = nnz;
    Mi.spmv_group = c->M.spmv_group;
    Mi.spmvt_group = c->M.spmvt_group;
    int32_t* dperm = nullptr;
    TRY(c->upload(&dperm, ro.perm));
    TRY(c->upload(&Mi.rowptr, ro.prp));
    TRY(c->dalloc(&Mi.colind, nnz));
    TRY(c->dalloc(&Mi.vals, nnz));
    TRY(c->dalloc(&Mi.trowptr, (int64_t)n + 1));
    TRY(c->dalloc(&Mi.trow, nnz));
    TRY(c->dalloc(&Mi.tperm, nnz));
    TRY(c->dalloc(&Mi.tvals, nnz));
    launch_permute_rows(st, m, dperm, c->M.rowptr, c->M.colind, c->M.vals, Mi.rowptr, Mi.colind, Mi.vals);
    LSQ2L_HIP_TRY(launch_transpose(st, m, n, nnz, Mi.rowptr, Mi.colind, Mi.trowptr, Mi.trow, Mi.tperm,
                                   keys, vals, rows, temp, tb));
    launch_gather_values(st, nnz, Mi.tperm, Mi.vals, Mi.tvals);
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));   // ro's vectors are uploaded from pageable memory
  }
  // --- solve workspace
  TRY(c->dalloc(&c->r, n));
  TRY(c->dalloc(&c->z, n));
  TRY(c->dalloc(&c->p, n));
  TRY(c->dalloc(&c->q, n));
  TRY(c->dalloc(&c->rhs, n));
  TRY(c->dalloc(&c->rold, n));
  TRY(c->dalloc(&c->xwork, n));
  TRY(c->dalloc(&c->xsave, n));
  TRY(c->dalloc(&c->tm, m));
  TRY(c->dalloc(&c->tm2, m));
  if (c->opt.variant == LSQ2L_BALANCED) {
    TRY(c->dalloc(&c->bal_u, n));
    TRY(c->dalloc(&c->bal_w, n));
  }
  TRY(c->dalloc(&c->bsave, m));
  TRY(c->dalloc(&c->loc, H.total_loc));
  TRY(c->dalloc(&c->partial, (int64_t)c->S * RED_BLOCKS));
  TRY(c->dalloc(&c->partial2, (int64_t)c->S * RED_BLOCKS));
  double* scal = nullptr;
  TRY(c->dalloc(&scal, 6 * (int64_t)c->S));
  c->sc.rho = scal; c->sc.alpha = scal + c->S; c->sc.beta = scal + 2 * c->S;
  c->sc.rn2 = scal + 3 * c->S; c->sc.r0n2 = scal + 4 * c->S; c->sc.pq = scal + 5 * c->S;
  TRY(c->dalloc(&c->sc.done, c->S));
  TRY(c->halloc(&c->h_done, c->S));
  TRY(c->halloc(&c->h_rn2, c->S));
  TRY(c->halloc(&c->h_r0n2, c->S));
  TRY(c->upload(&c->d_seg_col, c->seg_col_h));
  TRY(c->upload(&c->d_seg_row, c->seg_row_h));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  // --- info
  lsq2l_setup_info& inf = c->info;
  inf.m = m; inf.n = n; inf.nnz = nnz; inf.nparts = nparts; inf.ninstances = c->S;
  inf.n0 = c->n0;
  inf.max_ni = 0; inf.max_p = 0;
  int64_t dense = 0;
  for (const SubDesc& d : H.subs) {
    inf.max_ni = std::max(inf.max_ni, d.nI + d.nG);
    inf.max_p = std::max(inf.max_p, d.p);
    dense += (int64_t)(d.nI + d.nG) * (d.nI + d.nG + 1) / 2 * (int64_t)sizeof(double);
  }
  inf.factor_tiles = H.total_fac / TT;
  inf.factor_bytes = H.total_fac * (c->opt.precision == LSQ2L_MIXED ? sizeof(float) : sizeof(double));
  inf.factor_dense_bytes = dense;
  inf.t_total_ms = ms_since(t_all);
  return LSQ2L_OK;
}

lsq2l_status check_common(double tau, const lsq2l_options* opt) {
  if (!(tau > 0.0 && tau <= 1.0)) { set_error("tau must lie in (0, 1]"); return LSQ2L_EINVAL; }
  if (opt) {
    if (!(opt->tol > 0.0)) { set_error("tol must be positive"); return LSQ2L_EINVAL; }
    if (opt->max_it < 1) { set_error("max_it must be >= 1"); return LSQ2L_EINVAL; }
    if (opt->precision != LSQ2L_FP64 && opt->precision != LSQ2L_MIXED) { set_error("bad precision"); return LSQ2L_EINVAL; }
    if (opt->variant != LSQ2L_ADDITIVE && opt->variant != LSQ2L_ONE_LEVEL &&
        opt->variant != LSQ2L_BALANCED) { set_error("bad variant"); return LSQ2L_EINVAL; }
    if (opt->nev_max < 0) { set_error("nev_max must be >= 0"); return LSQ2L_EINVAL; }
  }
  return LSQ2L_OK;
}

lsq2l_status solve_impl(lsq2l_ctx* c, double* x, lsq2l_solve_info* info) {
  auto t0 = clk::now();
  std::vector<double> rt(c->S), rr(c->S);
  int its = 0, restarts = 0;
  lsq2l_status s = pcg(c, x, &its, &restarts, rt.data(), rr.data());
  const double ms = ms_since(t0);
  if (info)
    for (int k = 0; k < c->S; ++k) {
      info[k].iterations = its;
      info[k].restarts = restarts;
      info[k].relres = rt[k];
      info[k].relres_rec = rr[k];
      info[k].solve_ms = ms;
    }
  return s;
}

}  // namespace

extern "C" {

void lsq2l_default_options(lsq2l_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->tol = 1e-8;
  opt->max_it = 10000;
  opt->precision = LSQ2L_FP64;
  opt->flexible = 0;
  opt->variant = LSQ2L_ADDITIVE;
  opt->nev_max = 0;
  opt->check_every = 1;
  opt->use_graph = 0;
}

const char* lsq2l_last_error(void) { return g_err.c_str(); }

lsq2l_status lsq2l_setup(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                         const int32_t* colind, const double* vals, const int32_t* part,
                         int32_t nparts, int32_t overlap, double tau, const lsq2l_options* opt,
                         void* hip_stream, lsq2l_handle* out) {
  g_err.clear();
  if (!out) { set_error("out is NULL"); return LSQ2L_EINVAL; }
  *out = nullptr;
  if (m < 1 || n < 1 || m < n) { set_error("need m >= n >= 1"); return LSQ2L_EINVAL; }
  if (nnz < 0 || !rowptr || (nnz > 0 && (!colind || !vals)) || !part) { set_error("bad CSR pointers"); return LSQ2L_EINVAL; }
  if (nparts < 1 || nparts > n) { set_error("nparts must lie in [1, n]"); return LSQ2L_EINVAL; }
  if (overlap != 1) { set_error("only overlap = 1 (one layer, Section 3) is supported"); return LSQ2L_EINVAL; }
  TRY(check_common(tau, opt));
  for (int32_t j = 0; j < n; ++j)
    if (part[j] < 0 || part[j] >= nparts) { set_error("part[" + std::to_string(j) + "] out of range"); return LSQ2L_EINVAL; }
  lsq2l_ctx* c = new lsq2l_ctx();
  c->st = (hipStream_t)hip_stream;
  lsq2l_default_options(&c->opt);
  if (opt) c->opt = *opt;
  c->tau = tau;
  c->S = 1;
  c->M.m = m; c->M.n = n; c->M.nnz = nnz;
  c->seg_row_h = {0, m};
  c->seg_col_h = {0, n};
  auto fail = [&](lsq2l_status s) { delete c; return s; };
  std::vector<int32_t> pt(part, part + n);
  PinnedArray<int32_t> rp, ci;
  lsq2l_status s;
  if ((s = rp.alloc((int64_t)m + 1)) != LSQ2L_OK) return fail(s);
  if ((s = ci.alloc(nnz)) != LSQ2L_OK) return fail(s);
  if ((s = c->dalloc(&c->M.rowptr, m + 1)) != LSQ2L_OK) return fail(s);
  if ((s = c->dalloc(&c->M.colind, nnz)) != LSQ2L_OK) return fail(s);
  if ((s = c->dalloc(&c->M.vals, nnz)) != LSQ2L_OK) return fail(s);
  hipError_t e = hipMemcpyAsync(rp.p, rowptr, (m + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess && nnz) e = hipMemcpyAsync(ci.p, colind, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) { set_error(std::string("reading A: ") + hipGetErrorString(e)); return fail(LSQ2L_EHIP); }
  if (rp.p[m] != nnz) { set_error("rowptr[m] != nnz"); return fail(LSQ2L_EINVAL); }
  if ((s = validate_csr(m, n, rp.p, ci.p, nnz)) != LSQ2L_OK) return fail(s);
  e = hipMemcpyAsync(c->M.rowptr, rowptr, (m + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, c->st);
  if (e == hipSuccess && nnz) e = hipMemcpyAsync(c->M.colind, colind, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, c->st);
  if (e == hipSuccess && nnz) e = hipMemcpyAsync(c->M.vals, vals, nnz * sizeof(double), hipMemcpyDeviceToDevice, c->st);
  if (e != hipSuccess) { set_error(std::string("copying A: ") + hipGetErrorString(e)); return fail(LSQ2L_EHIP); }
  std::vector<int32_t> seg_of_part(nparts, 0);
  s = setup_core(c, rp.p, ci.p, pt, nparts, seg_of_part);
  if (s != LSQ2L_OK) return fail(s);
  *out = c;
  return LSQ2L_OK;
}

lsq2l_status lsq2l_setup_batched(int32_t count, const lsq2l_problem* probs, double tau,
                                 const lsq2l_options* opt, void* hip_stream, lsq2l_handle* out) {
  g_err.clear();
  if (!out || !probs || count < 1) { set_error("bad arguments"); return LSQ2L_EINVAL; }
  *out = nullptr;
  TRY(check_common(tau, opt));
  int64_t M = 0, N = 0, NNZ = 0, NP = 0;
  for (int k = 0; k < count; ++k) {
    const lsq2l_problem& pr = probs[k];
    if (pr.m < 1 || pr.n < 1 || pr.m < pr.n || pr.nnz < 0 || pr.nparts < 1 || pr.nparts > pr.n ||
        !pr.rowptr || !pr.part || (pr.nnz > 0 && (!pr.colind || !pr.vals))) {
      set_error("bad problem " + std::to_string(k));
      return LSQ2L_EINVAL;
    }
    M += pr.m; N += pr.n; NNZ += pr.nnz; NP += pr.nparts;
  }
  if (M >= INT32_MAX || NNZ >= INT32_MAX) { set_error("batch too large for int32 indices"); return LSQ2L_EINVAL; }
  lsq2l_ctx* c = new lsq2l_ctx();
  c->st = (hipStream_t)hip_stream;
  lsq2l_default_options(&c->opt);
  if (opt) c->opt = *opt;
  c->tau = tau;
  c->S = count;
  c->M.m = (int32_t)M; c->M.n = (int32_t)N; c->M.nnz = NNZ;
  auto fail = [&](lsq2l_status s) { delete c; return s; };
  std::vector<int32_t> rp(M + 1, 0), ci(NNZ), pt(N), seg_of_part(NP);
  c->seg_row_h.assign(count + 1, 0);
  c->seg_col_h.assign(count + 1, 0);
  lsq2l_status s;
  if ((s = c->dalloc(&c->M.rowptr, M + 1)) != LSQ2L_OK) return fail(s);
  if ((s = c->dalloc(&c->M.colind, NNZ)) != LSQ2L_OK) return fail(s);
  if ((s = c->dalloc(&c->M.vals, NNZ)) != LSQ2L_OK) return fail(s);
  int64_t r0 = 0, c0 = 0, e0 = 0, p0 = 0;
  for (int k = 0; k < count; ++k) {
    const lsq2l_problem& pr = probs[k];
    std::vector<int32_t> lrp(pr.m + 1), lci(pr.nnz);
    hipError_t e = hipMemcpyAsync(lrp.data(), pr.rowptr, (pr.m + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && pr.nnz) e = hipMemcpyAsync(lci.data(), pr.colind, pr.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess && pr.nnz) e = hipMemcpyAsync(c->M.vals + e0, pr.vals, pr.nnz * sizeof(double), hipMemcpyDeviceToDevice, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) { set_error(std::string("reading problem: ") + hipGetErrorString(e)); return fail(LSQ2L_EHIP); }
    if (lrp[pr.m] != pr.nnz) { set_error("rowptr[m] != nnz in problem " + std::to_string(k)); return fail(LSQ2L_EINVAL); }
    if ((s = validate_csr(pr.m, pr.n, lrp.data(), lci.data(), pr.nnz)) != LSQ2L_OK) return fail(s);
    for (int32_t rr = 0; rr < pr.m; ++rr) rp[r0 + rr + 1] = (int32_t)(e0 + lrp[rr + 1]);
    for (int32_t q = 0; q < pr.nnz; ++q) ci[e0 + q] = (int32_t)(c0 + lci[q]);
    for (int32_t j = 0; j < pr.n; ++j) {
      if (pr.part[j] < 0 || pr.part[j] >= pr.nparts) { set_error("part out of range in problem " + std::to_string(k)); return fail(LSQ2L_EINVAL); }
      pt[c0 + j] = (int32_t)(p0 + pr.part[j]);
    }
    for (int32_t q = 0; q < pr.nparts; ++q) seg_of_part[p0 + q] = k;
    r0 += pr.m; c0 += pr.n; e0 += pr.nnz; p0 += pr.nparts;
    c->seg_row_h[k + 1] = r0;
    c->seg_col_h[k + 1] = c0;
  }
  hipError_t e = hipMemcpyAsync(c->M.rowptr, rp.data(), (M + 1) * sizeof(int32_t), hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess && NNZ) e = hipMemcpyAsync(c->M.colind, ci.data(), NNZ * sizeof(int32_t), hipMemcpyHostToDevice, c->st);
  if (e != hipSuccess) { set_error(std::string("copying A: ") + hipGetErrorString(e)); return fail(LSQ2L_EHIP); }
  s = setup_core(c, rp.data(), ci.data(), pt, (int32_t)NP, seg_of_part);
  if (s != LSQ2L_OK) return fail(s);
  *out = c;
  return LSQ2L_OK;
}

lsq2l_status lsq2l_solve(lsq2l_handle c, const double* b, double* x, lsq2l_solve_info* info) {
  g_err.clear();
  if (!c || !b || !x) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->bsave, b, c->M.m * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  spmv_AT(c, b, c->rhs);
  lsq2l_status s = solve_impl(c, x, info);
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->xsave, x, c->M.n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  c->have_solution = (s == LSQ2L_OK || s == LSQ2L_NOT_CONVERGED);
  return s;
}

lsq2l_status lsq2l_backward(lsq2l_handle c, const double* g, double* dLdb, double* dLdvals,
                            lsq2l_solve_info* info) {
  g_err.clear();
  if (!c || !g) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  if (!c->have_solution) { set_error("backward needs a previous solve"); return LSQ2L_EINVAL; }
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->rhs, g, c->M.n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  lsq2l_status s = solve_impl(c, c->xwork, info);       // lambda = C^{-1} g
  if (s != LSQ2L_OK && s != LSQ2L_NOT_CONVERGED) return s;
  spmv_A(c, c->xwork, c->tm);                            // A lambda
  if (dLdb) LSQ2L_HIP_TRY(hipMemcpyAsync(dLdb, c->tm, c->M.m * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  if (dLdvals) {
    spmv_A(c, c->xsave, c->tm2);                         // r = b - A x
    launch_sub(c->st, c->M.m, c->bsave, c->tm2, c->tm2);
    launch_grad_vals(c->st, c->M.m, c->M.rowptr, c->M.colind, c->tm2, c->xwork, c->tm, c->xsave, dLdvals);
  }
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  return s;
}

lsq2l_status lsq2l_spmv(lsq2l_handle c, int32_t trans, const double* x, double* y) {
  g_err.clear();
  if (!c || !x || !y) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  if (trans) spmv_AT(c, x, y); else spmv_A(c, x, y);
  LSQ2L_HIP_TRY(hipGetLastError());
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  return LSQ2L_OK;
}

lsq2l_status lsq2l_apply_preconditioner(lsq2l_handle c, const double* r, double* z) {
  g_err.clear();
  if (!c || !r || !z) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  apply_M(c, r, z);
  LSQ2L_HIP_TRY(hipGetLastError());
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  return LSQ2L_OK;
}

lsq2l_status lsq2l_get_info(lsq2l_handle c, lsq2l_setup_info* out) {
  if (!c || !out) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  *out = c->info;
  return LSQ2L_OK;
}

lsq2l_status lsq2l_get_subdomain(lsq2l_handle c, int32_t i, int32_t* sizes, int32_t* interior,
                                 int32_t* xi, int32_t* gamma) {
  if (!c) { set_error("NULL handle"); return LSQ2L_EINVAL; }
  if (i < 0 || i >= c->nsub) { set_error("subdomain index out of range"); return LSQ2L_EINVAL; }
  const SubDesc& d = c->H.subs[i];
  if (sizes) { sizes[0] = d.nI; sizes[1] = d.nXi; sizes[2] = d.nG; sizes[3] = d.p; }
  if (interior) std::memcpy(interior, &c->H.omega[d.omega_off], sizeof(int32_t) * d.nI);
  if (gamma) std::memcpy(gamma, &c->H.omega[d.omega_off + d.nI], sizeof(int32_t) * d.nG);
  if (xi) std::memcpy(xi, &c->H.xi[d.xi_off], sizeof(int32_t) * d.nXi);
  return LSQ2L_OK;
}

lsq2l_status lsq2l_get_coarse_basis(lsq2l_handle c, int32_t i, double* X) {
  if (!c || !X) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  if (i < 0 || i >= c->nsub) { set_error("subdomain index out of range"); return LSQ2L_EINVAL; }
  const SubDesc& d = c->H.subs[i];
  if (d.p == 0) return LSQ2L_OK;
  std::vector<double> tmp((size_t)d.nIp * d.p);
  LSQ2L_HIP_TRY(hipMemcpyAsync(tmp.data(), c->X + d.x_off, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  for (int k = 0; k < d.p; ++k)
    std::memcpy(X + (size_t)k * d.nI, tmp.data() + (size_t)k * d.nIp, sizeof(double) * d.nI);
  return LSQ2L_OK;
}

lsq2l_status lsq2l_time_kernel(lsq2l_handle c, int32_t kernel, int32_t reps, double* avg_ms,
                               double* bytes) {
  g_err.clear();
  if (!c || !avg_ms || !bytes || reps < 1) { set_error("bad arguments"); return LSQ2L_EINVAL; }
  if (kernel < 0 || kernel > 3 || (kernel == 3 && !c->coarse)) { set_error("unknown or unused kernel"); return LSQ2L_EINVAL; }
  const double m = c->M.m, n = c->M.n, nnz = (double)c->M.nnz;
  const double eb = (c->opt.precision == LSQ2L_MIXED) ? 4.0 : 8.0;
  switch (kernel) {
    case 0: *bytes = 12.0 * nnz + 4.0 * (m + 1) + 8.0 * n + 8.0 * m; break;
    case 1: *bytes = 12.0 * nnz + 4.0 * (n + 1) + 8.0 * m + 8.0 * n; break;
    // each sweep reads every stored off-diagonal tile and every diagonal
    // inverse once (as many elements as the stored factor), plus y in and out
    case 2: *bytes = 2.0 * eb * (double)c->H.total_fac + 16.0 * (double)c->H.total_loc; break;
    default: {
      double tri = 0, parts = 0;
      for (const SegDesc& sg : c->segs_h) {
        const double nt = (double)sg.etiles;
        tri += (double)TT * nt * (nt + 1) / 2;
        parts += (double)TS * nt * (nt + 1) / 2;
      }
      // the triangle once; row and chunk column partials written and read
      // back; c in and d out
      *bytes = 8.0 * tri + 16.0 * parts + 16.0 * TS * (double)c->Cc.e_nchunks + 16.0 * (double)c->n0tot;
    }
  }
  launch_fill(c->st, c->M.n, 1.0, c->p);
  launch_fill(c->st, c->M.m, 1.0, c->tm);
  launch_fill(c->st, c->H.total_loc, 1.0, c->loc);
  if (c->coarse) launch_fill(c->st, c->n0tot, 1.0, c->cvec);
  hipEvent_t e0, e1;
  LSQ2L_HIP_TRY(hipEventCreate(&e0));
  LSQ2L_HIP_TRY(hipEventCreate(&e1));
  auto once = [&]() {
    switch (kernel) {
      case 0: spmv_it_A(c, c->p, c->tm); break;
      case 1: spmv_it_AT(c, c->tm, c->q); break;
      case 2:
        if (c->opt.precision == LSQ2L_MIXED) launch_local_solve_f32(c->st, c->nsub, c->P, c->fac32, c->dinv32, c->loc);
        else launch_local_solve(c->st, c->nsub, c->P, c->fac, c->dinv, c->loc);
        break;
      default: launch_einv_gemv(c->st, c->n0tot, c->S, c->Cc, c->einv, c->cvec, c->dvec);
    }
  };
  once();
  LSQ2L_HIP_TRY(hipEventRecord(e0, c->st));
  for (int k = 0; k < reps; ++k) once();
  LSQ2L_HIP_TRY(hipEventRecord(e1, c->st));
  LSQ2L_HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  LSQ2L_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / reps;
  return LSQ2L_OK;
}

void lsq2l_destroy(lsq2l_handle c) { delete c; }

void lsq2l_release_cache(void) {
  block_cache().release();
  pinned_pool().release();
}

}  // extern "C"
