// C ABI of the lsq2l library: setup (Algorithm 1), the preconditioners of
// Section 2 (eqs. one_level_schwarz, RAS, two_level_schwarz, balanced,
// deflated), the CG solve on the normal equations (eq. normal; LSQR and
// GMRES live in krylov.cpp), the adjoint solve, and the accessors used for
// validation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <functional>
#include <thread>
#include <vector>

#include "ctx.hpp"
#include "krylov.hpp"

namespace lsq2l {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace {

// Launch shape of the SpMV: row blocks staged through LDS (0) for every
// matrix; lsq2l_autotune replaces it by a measured choice among that and
// 1 .. 64 lanes per row.
int pick_group(double) { return 0; }

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
// pattern, A^T's pattern) and stages its uploads through, kept for later
// setups: a pageable copy runs at a sixth of the pinned rate, and pinning
// fresh memory costs more than the copy.  At most PINNED_LIMIT bytes stay
// cached.
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

}  // namespace

void* cache_take(size_t bytes, int dev, size_t* got) { return block_cache().take(bytes, dev, got); }
void cache_give(void* p, size_t bytes, int dev) { block_cache().give(p, bytes, dev); }
void cache_release() { block_cache().release(); }
void* pinned_take(size_t bytes, size_t* got) { return pinned_pool().take(bytes, got); }
void pinned_give(void* p, size_t bytes) { pinned_pool().give(p, bytes); }
void pinned_release() { pinned_pool().release(); }

// host arrays of the planner: from 1 MiB up in the pinned pool (whole MiB),
// smaller ones from the heap
void* host_block_take(size_t bytes, size_t* got) {
  constexpr size_t MiB = (size_t)1 << 20;
  if (bytes < MiB) {
    *got = bytes;
    return std::malloc(bytes);
  }
  return pinned_take((bytes + MiB - 1) / MiB * MiB, got);
}
void host_block_give(void* p, size_t bytes) {
  if (bytes < ((size_t)1 << 20)) std::free(p);
  else pinned_give(p, bytes);
}

}  // namespace lsq2l

using namespace lsq2l;

lsq2l_status lsq2l_ctx::raw_alloc(void** v, size_t bytes) {
  int dev = 0;
  LSQ2L_HIP_TRY(hipGetDevice(&dev));
  size_t got = 0;
  if ((*v = cache_take(bytes, dev, &got)) != nullptr) {
    dev_allocs.push_back({*v, got, dev});
    return LSQ2L_OK;
  }
  hipError_t e = hipMalloc(v, bytes);
  if (e != hipSuccess) {
    cache_release();
    e = hipMalloc(v, bytes);
  }
  if (e != hipSuccess) {
    set_error("device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    return LSQ2L_ENOMEM;
  }
  dev_allocs.push_back({*v, bytes, dev});
  return LSQ2L_OK;
}

lsq2l_ctx::~lsq2l_ctx() {
  if (st) (void)hipStreamSynchronize(st);
  else (void)hipDeviceSynchronize();
  release_staged();
  if (st2) (void)hipStreamSynchronize(st2);
  if (gst) (void)hipStreamDestroy(gst);
  if (st2) (void)hipStreamDestroy(st2);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  for (const DevBlock& b : dev_allocs) cache_give(b.p, b.bytes, b.dev);
  for (void* v : host_allocs) (void)hipHostFree(v);
}

namespace lsq2l {

// ---------------------------------------------------------------------------
// products with A, A^T and the preconditioners
// ---------------------------------------------------------------------------

// C p = A^T (A p) inside the iteration.  A p never leaves the library, so it
// may be formed with a row-permuted copy of A: C = A^T A is the same for any
// row order of A.
void spmv_it_A(lsq2l_ctx* c, const double* x, double* y) {
  const DevMatrix& M = c->row_perm ? c->Mi : c->M;
  launch_spmv(c->st, M.m, M.rowptr, M.colind, M.vals, x, y, M.spmv_group, M.nnz, M.blk);
}
void spmv_it_AT(lsq2l_ctx* c, const double* y, double* x) {
  const DevMatrix& M = c->row_perm ? c->Mi : c->M;
  launch_spmv(c->st, M.n, M.trowptr, M.trow, M.tvals, y, x, M.spmvt_group, M.nnz, M.tblk);
}
void spmv_A(lsq2l_ctx* c, const double* x, double* y) {
  launch_spmv(c->st, c->M.m, c->M.rowptr, c->M.colind, c->M.vals, x, y, c->M.spmv_group, c->M.nnz, c->M.blk);
}
void spmv_AT(lsq2l_ctx* c, const double* y, double* x) {
  launch_spmv(c->st, c->M.n, c->M.trowptr, c->M.trow, c->M.tvals, y, x, c->M.spmvt_group, c->M.nnz, c->M.tblk);
}
// y = C x = A^T (A x), with tmp (m doubles) for A x
void apply_C(lsq2l_ctx* c, const double* x, double* y, double* tmp) {
  spmv_it_A(c, x, tmp);
  spmv_it_AT(c, tmp, y);
}

void local_solves(lsq2l_ctx* c) {
  if (c->opt.precision == LSQ2L_MIXED)
    launch_local_solve_f32(c->st, c->nsub, c->Ps, c->fac32, c->dinv32, c->loc);
  else if (c->solve_plan)
    launch_local_solve(c->st, c->nsub, c->Ps, c->sfac, c->sdinv, c->loc);
  else
    launch_local_solve(c->st, c->nsub, c->P, c->fac, c->dinv, c->loc);
}

namespace {

void scatter(lsq2l_ctx* c, const double* loc, const double* dcoarse, double* z, bool restricted) {
  if (c->X32) launch_scatter_local(c->st, c->M.n, c->P, c->scale, loc, c->X32, dcoarse, z, restricted);
  else launch_scatter_local(c->st, c->M.n, c->P, c->scale, loc, c->X, dcoarse, z, restricted);
}

// z = Q r = R_0^T E^{-1} R_0 r (restriction, symmetric E^{-1} product, prolongation)
void apply_Q(lsq2l_ctx* c, const double* r, double* z) {
  const hipStream_t st = c->st;
  if (c->X32) launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X32, r, c->cvec);
  else launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X, r, c->cvec);
  launch_einv_gemv(st, c->n0tot, c->S, c->Cc, c->einv, c->cvec, c->dvec);
  scatter(c, nullptr, c->dvec, z, false);
}

// z = M_ASM r = sum_i R_i^T C_ii^{-1} R_i r (eq. one_level_schwarz), or with
// `restricted` M_RAS r = sum_i R_i^T D_i C_ii^{-1} R_i r (eq. RAS)
void apply_one_level(lsq2l_ctx* c, const double* r, double* z, bool restricted) {
  launch_gather_local(c->st, c->nsub, c->P, c->scale, r, c->loc);
  local_solves(c);
  scatter(c, c->loc, nullptr, z, restricted);
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
  apply_C(c, c->bal_u, c->bal_w, c->tm2);
  launch_sub(st, n, r, c->bal_w, c->bal_w);            // (I - C Q) r
  apply_one_level(c, c->bal_w, z, false);              // y
  apply_C(c, z, c->bal_w, c->tm2);
  launch_sub(st, n, r, c->bal_w, c->bal_w);            // r - C y
  apply_Q(c, c->bal_w, c->bal_u);
  launch_add(st, n, z, c->bal_u, z);
}

// Deflated form (eq. deflated) with M_RAS as the first level:
// M r = Q r + M_RAS (I - C Q) r = u + M_RAS (r - C u), u = Q r.  One coarse
// correction, two SpMVs, one set of local solves per application.
void apply_M_deflated(lsq2l_ctx* c, const double* r, double* z) {
  const hipStream_t st = c->st;
  const int64_t n = c->M.n;
  apply_Q(c, r, c->bal_u);
  apply_C(c, c->bal_u, c->bal_w, c->tm2);
  launch_sub(st, n, r, c->bal_w, c->bal_w);            // (I - C Q) r
  apply_one_level(c, c->bal_w, z, true);               // M_RAS (I - C Q) r
  launch_add(st, n, z, c->bal_u, z);
}

}  // namespace

// z = M r for the variant of the handle (z == r allowed).
void apply_M(lsq2l_ctx* c, const double* r, double* z) {
  const int v = c->opt.variant;
  if (v == LSQ2L_ONE_LEVEL || (v == LSQ2L_BALANCED && !c->coarse)) { apply_one_level(c, r, z, false); return; }
  if (v == LSQ2L_RAS || (v == LSQ2L_DEFLATED && !c->coarse)) { apply_one_level(c, r, z, true); return; }
  if (v == LSQ2L_BALANCED) { apply_M_balanced(c, r, z); return; }
  if (v == LSQ2L_DEFLATED) {
    if (z == r) {               // r is read again after z is first written
      launch_copy(c->st, c->M.n, r, c->rold);
      r = c->rold;
    }
    apply_M_deflated(c, r, z);
    return;
  }
  // additive: local solves plus the coarse correction R_0^T E^{-1} R_0 r
  // (eq. two_level_schwarz), the coarse restriction and solve between the
  // local solves and the scatter that adds both
  const hipStream_t st = c->st;
  launch_gather_local(st, c->nsub, c->P, c->scale, r, c->loc);
  local_solves(c);
  if (c->coarse) {
    if (c->X32) launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X32, r, c->cvec);
    else launch_coarse_restrict(st, c->nsub, c->P, c->max_p, c->X, r, c->cvec);
    launch_einv_gemv(st, c->n0tot, c->S, c->Cc, c->einv, c->cvec, c->dvec);
  }
  scatter(c, c->loc, c->coarse ? c->dvec : nullptr, z, false);
}

// per-instance sums of the RED_BLOCKS partials (host, fixed order)
lsq2l_status read_seg_sums(lsq2l_ctx* c, const double* partial, std::vector<double>& out) {
  const int S = c->S;
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_part, partial, sizeof(double) * S * RED_BLOCKS,
                               hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  out.assign(S, 0.0);
  for (int s = 0; s < S; ++s) {
    double t = 0.0;
    for (int b = 0; b < RED_BLOCKS; ++b) t += c->h_part[(size_t)s * RED_BLOCKS + b];
    out[s] = t;
  }
  return LSQ2L_OK;
}

// ||C||_2 per instance, from below, by 30 steps of the power method on C
// (device-side normalisation, one read-back at the end).  Kept in the handle.
lsq2l_status norm_C(lsq2l_ctx* c) {
  if (!c->normC.empty()) return LSQ2L_OK;
  const hipStream_t st = c->st;
  const int S = c->S;
  const int64_t n = c->M.n;
  double* v = c->rold;
  double* w = c->q;
  double* nrm = c->sc.pq;          // S doubles, free outside the iteration
  launch_hash_fill(st, n, v);
  launch_dot(st, S, c->d_seg_col, v, v, c->partial);
  launch_seg_sum(st, S, c->partial, nrm);
  launch_normalize_seg(st, n, S, c->d_seg_col, nrm, nullptr, v, v);
  for (int it = 0; it < 30; ++it) {
    apply_C(c, v, w, c->tm);
    launch_dot(st, S, c->d_seg_col, w, w, c->partial);
    launch_seg_sum(st, S, c->partial, nrm);
    launch_normalize_seg(st, n, S, c->d_seg_col, nrm, nullptr, w, v);
  }
  std::vector<double> h(S);
  LSQ2L_HIP_TRY(hipMemcpyAsync(h.data(), nrm, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  c->normC.resize(S);
  for (int s = 0; s < S; ++s) c->normC[s] = std::sqrt(h[s]);
  return LSQ2L_OK;
}

namespace {

lsq2l_status read_flags(lsq2l_ctx* c) {
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_done, c->sc.done, sizeof(int32_t) * c->S, hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_rn2, c->sc.rn2, sizeof(double) * c->S, hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_r0n2, c->sc.r0n2, sizeof(double) * c->S, hipMemcpyDeviceToHost, c->st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  return LSQ2L_OK;
}

// The residual-norm step of a CG iteration (sets the done flags).
void rnorm_step(lsq2l_ctx* c, double tol2, int flexible) {
  launch_dot(c->st, c->S, c->d_seg_col, c->r, c->r, c->partial);
  launch_scalar(c->st, OP_RNORM, c->S, c->partial, nullptr, c->sc, tol2, flexible);
}

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
    apply_C(c, c->p, c->q, c->tm);
    launch_dot(st, S, c->d_seg_col, c->p, c->q, c->partial);
    launch_scalar(st, OP_ALPHA, S, c->partial, nullptr, c->sc, tol2, flexible);
    if (flexible) launch_copy(st, n, c->r, c->rold);
    launch_axpy_xr(st, n, S, c->d_seg_col, c->sc.alpha, c->p, c->q, x, c->r);
    rnorm_step(c, tol2, flexible);
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

}  // namespace

// PCG on C x = rhs (x_0 = 0), C = A^T A applied as A^T (A p).  x is written.
// It stops on the relative residual ||rhs - C x|| <= tol ||rhs||.  With
// adjoint set, an instance whose true residual still misses that after the
// restarts (the attainable accuracy of CG on an ill-conditioned C) is
// accepted if its normwise backward error
// ||rhs - C x|| / (||C||_2 ||x|| + ||rhs||) is at most tol (c->normC known).
lsq2l_status pcg(lsq2l_ctx* c, double* x, bool adjoint, double tol, KrylovResult& res) {
  const hipStream_t st = c->st;
  const int S = c->S;
  const int64_t n = c->M.n;
  const double tol2 = tol * tol;
  const int flexible = c->opt.flexible;
  launch_fill(st, n, 0.0, x);
  launch_fill_i32(st, S, 0, c->sc.its);
  launch_copy(st, n, c->rhs, c->r);
  launch_dot(st, S, c->d_seg_col, c->r, c->r, c->partial);
  launch_scalar(st, OP_R0, S, c->partial, nullptr, c->sc, tol2, flexible);
  int its = 0, restarts = 0;
  bool breakdown = false;
  res.relres.assign(S, 0.0);
  res.relres_rec.assign(S, 0.0);
  res.backward_err.assign(S, 0.0);
  res.converged.assign(S, 0);
  while (true) {
    apply_M(c, c->r, c->z);
    launch_dot(st, S, c->d_seg_col, c->r, c->z, c->partial);
    launch_scalar(st, OP_RHO_INIT, S, c->partial, nullptr, c->sc, tol2, flexible);
    launch_copy(st, n, c->z, c->p);
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
      apply_C(c, c->p, c->q, c->tm);
      launch_dot(st, S, c->d_seg_col, c->p, c->q, c->partial);
      launch_scalar(st, OP_ALPHA, S, c->partial, nullptr, c->sc, tol2, flexible);
      if (flexible) launch_copy(st, n, c->r, c->rold);
      launch_axpy_xr(st, n, S, c->d_seg_col, c->sc.alpha, c->p, c->q, x, c->r);
      rnorm_step(c, tol2, flexible);
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
    apply_C(c, x, c->q, c->tm);
    launch_sub(st, n, c->rhs, c->q, c->q);
    launch_dot(st, S, c->d_seg_col, c->q, c->q, c->partial);
    std::vector<double> t2, x2;
    TRY(read_seg_sums(c, c->partial, t2));
    if (adjoint) {
      launch_dot(st, S, c->d_seg_col, x, x, c->partial2);
      TRY(read_seg_sums(c, c->partial2, x2));
    }
    TRY(read_flags(c));
    bool all_ok = true;
    const bool last = restarts == 3 || its >= c->opt.max_it;
    for (int s = 0; s < S; ++s) {
      const double r0 = c->h_r0n2[s];
      res.relres[s] = r0 > 0 ? std::sqrt(t2[s] / r0) : 0.0;
      res.relres_rec[s] = r0 > 0 ? std::sqrt(c->h_rn2[s] / r0) : 0.0;
      bool ok = res.relres[s] <= tol;
      if (adjoint) {
        const double bound = c->normC[s] * std::sqrt(x2[s]) + std::sqrt(r0);
        res.backward_err[s] = bound > 0 ? std::sqrt(t2[s]) / bound : 0.0;
        if (last && res.backward_err[s] <= tol) ok = true;
      }
      res.converged[s] = ok ? 1 : 0;
      if (c->h_done[s] == 2) breakdown = true;
      if (!ok) all_ok = false;
    }
    if (all_ok || breakdown || last) break;
    // restart from the true residual; converged instances re-check immediately
    ++restarts;
    launch_copy(st, n, c->q, c->r);
    launch_fill_i32(st, S, 0, c->sc.done);
    rnorm_step(c, tol2, flexible);
  }
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->h_its, c->sc.its, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  res.its.assign(c->h_its, c->h_its + S);
  res.restarts = restarts;
  res.total_its = its;
  if (breakdown) { set_error("PCG breakdown (non-positive curvature or non-finite value)"); return LSQ2L_PCG_BREAKDOWN; }
  for (int s = 0; s < S; ++s)
    if (!res.converged[s]) {
      set_error("PCG did not reach the tolerance within max_it iterations");
      return LSQ2L_NOT_CONVERGED;
    }
  return LSQ2L_OK;
}

// True relative normal-equation residual ||rhs - C x|| / ||rhs|| per
// instance (and ||x||^2 if asked), through the work vectors q and tm.
lsq2l_status true_residual(lsq2l_ctx* c, const double* x, std::vector<double>& rel,
                           std::vector<double>* x2) {
  const hipStream_t st = c->st;
  const int S = c->S;
  apply_C(c, x, c->q, c->tm);
  launch_sub(st, c->M.n, c->rhs, c->q, c->q);
  std::vector<double> t2, r2;
  launch_dot(st, S, c->d_seg_col, c->q, c->q, c->partial);
  TRY(read_seg_sums(c, c->partial, t2));
  launch_dot(st, S, c->d_seg_col, c->rhs, c->rhs, c->partial);
  TRY(read_seg_sums(c, c->partial, r2));
  if (x2) {
    launch_dot(st, S, c->d_seg_col, x, x, c->partial);
    TRY(read_seg_sums(c, c->partial, *x2));
  }
  rel.assign(S, 0.0);
  for (int s = 0; s < S; ++s) rel[s] = r2[s] > 0 ? std::sqrt(t2[s] / r2[s]) : 0.0;
  return LSQ2L_OK;
}

namespace {

// The overlap maps of the plan, built on a host thread while the device
// assembles, factors and selects; joined before their first use.
struct MapsJob {
  std::thread th;
  bool ok = true;
  std::string err;
  void start(int32_t n, HostPlan* H) {
    th = std::thread([this, n, H]() { ok = plan_maps(n, *H, err); });
  }
  bool join() {
    if (th.joinable()) th.join();
    return ok;
  }
  ~MapsJob() { if (th.joinable()) th.join(); }
};

// a thread joined on every exit from the scope that owns it
struct JoiningThread {
  std::thread t;
  ~JoiningThread() {
    if (t.joinable()) t.join();
  }
};

lsq2l_status autotune_spmv(lsq2l_ctx* c, int reps);

// Layout of the factors the local solves read.  C_ii^{-1} r does not depend
// on the order of Omega_i; the order [Omega_Ii, Omega_Gamma_i] that the
// coarse selection needs makes the interface rows of L_i dense across the
// interior.  Per subdomain, the global-column order of Omega_i is taken
// when its tile envelope (found by the assembly, see k_assemble) has at
// most 0.85 of the tiles of the [I, Gamma] one (opt.solve_order may force
// either).  The mixed path always gets a solve layout (its float factors are
// computed on their own); the FP64 path only when some subdomain is
// permuted, else it solves with the selection's factors.
//
// solve_layout_begin, before the assembly: the candidate global-order
// layouts and the position map, and the envelope's initial value.
lsq2l_status solve_layout_begin(lsq2l_ctx* c) {
  const hipStream_t st = c->st;
  const HostPlan& H = c->H;
  const bool mixed = c->opt.precision == LSQ2L_MIXED;
  const bool qr = c->opt.local_factor == LSQ2L_FACTOR_QR;
  c->sl_inv = nullptr;
  if (!mixed && !qr && c->opt.solve_order == LSQ2L_ORDER_SPLIT) return LSQ2L_OK;
  // global-order layouts: np = roundup(n_i), local-vector slices of
  // max(np, [I, Gamma] np) entries
  c->sl_g.assign(H.subs.begin(), H.subs.end());
  int64_t tb = 0, lo = 0;
  for (SubDesc& d : c->sl_g) {
    const int32_t np_main = d.np;
    d.np = (d.nI + d.nG + TS - 1) / TS * TS;
    d.ntiles = d.np / TS;
    d.tile_base = tb; tb += d.ntiles;
    d.loc_off = lo; lo += std::max(np_main, d.np);
  }
  c->sl_tiles = tb;
  c->sl_loc = lo;
  TRY(c->upload(&c->sl_dg, c->sl_g));
  TRY(c->dalloc(&c->sl_inv, H.total_loc));
  TRY(c->dalloc(&c->sl_Fg, std::max<int64_t>(tb, 1)));
  launch_solve_inv(st, c->nsub, c->P, c->sl_inv);
  launch_solve_env_init(st, c->nsub, c->sl_dg, c->sl_Fg);
  return LSQ2L_OK;
}

// solve_layout, after the assembly and equilibration (c->fac holds the
// equilibrated C_ii, not yet factored): the choice, the layout Ps on the
// device, and the gather of its matrix into *s64 (double), enqueued;
// c->solve_plan tells whether it is used.  With the QR local factors (no
// C_ii assembled) the solve layout is always used and *s64 comes zeroed.
lsq2l_status solve_layout(lsq2l_ctx* c, double** s64) {
  const hipStream_t st = c->st;
  const HostPlan& H = c->H;
  const int nsub = c->nsub;
  const bool mixed = c->opt.precision == LSQ2L_MIXED;
  const bool qr = c->opt.local_factor == LSQ2L_FACTOR_QR;
  *s64 = nullptr;
  c->solve_plan = false;
  c->info.split_tiles = H.total_fac / TT;
  c->info.solve_permuted = 0;
  if (!c->sl_inv) return LSQ2L_OK;
  const std::vector<SubDesc>& g = c->sl_g;
  const int64_t tb = c->sl_tiles, lo = c->sl_loc;
  int32_t* inv = c->sl_inv;
  std::vector<int32_t> hF((size_t)tb);
  if (tb) LSQ2L_HIP_TRY(hipMemcpyAsync(hF.data(), c->sl_Fg, sizeof(int32_t) * tb, hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  // choose per subdomain, then the layout's offsets
  std::vector<SubDesc> s(g);
  std::vector<int32_t> sF;
  std::vector<int64_t> sOff, tiles(nsub);
  int64_t ftiles = 0, dtiles = 0, stb = 0, split_tiles = 0;
  int permuted = 0;
  for (int i = 0; i < nsub; ++i) {
    const SubDesc& m = H.subs[i];
    int64_t tm = 0, tg = 0;
    for (int32_t t = 0; t < m.ntiles; ++t) tm += t - H.tileF[m.tile_base + t] + 1;
    for (int32_t t = 0; t < g[i].ntiles; ++t) tg += t - hF[g[i].tile_base + t] + 1;
    split_tiles += tm;
    const int order = c->opt.solve_order;
    const bool use_g = order == LSQ2L_ORDER_GLOBAL || (order == LSQ2L_ORDER_AUTO && tg * 100 <= tm * 85);
    SubDesc& d = s[i];
    d.np = use_g ? g[i].np : m.np;
    d.ntiles = use_g ? g[i].ntiles : m.ntiles;
    d.spare = use_g ? 1 : 0;
    d.tile_base = stb; stb += d.ntiles;
    d.fac_off = ftiles * TT;
    d.dinv_off = dtiles * TT; dtiles += d.ntiles;
    int64_t run = 0;
    for (int32_t t = 0; t < d.ntiles; ++t) {
      const int32_t f = use_g ? hF[g[i].tile_base + t] : H.tileF[m.tile_base + t];
      sF.push_back(f);
      sOff.push_back(run);
      run += t - f + 1;
    }
    ftiles += run;
    tiles[i] = run;
    permuted += use_g;
  }
  c->info.split_tiles = split_tiles;
  c->info.solve_permuted = permuted;
  if (!mixed && !qr && permuted == 0) return LSQ2L_OK;
  c->solve_plan = true;
  c->s_total_fac = ftiles * TT;
  c->s_total_dinv = dtiles * TT;
  c->s_total_tiles = stb;
  c->s_total_np = 0;
  DevPlan& Ps = c->Ps;
  Ps.max_np = 0;
  for (const SubDesc& d : s) { c->s_total_np += d.np; Ps.max_np = std::max(Ps.max_np, (int)d.np); }
  std::vector<int32_t> order(nsub);
  for (int i = 0; i < nsub; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tiles[x] > tiles[y]; });
  std::vector<SubDesc> so(nsub);
  for (int i = 0; i < nsub; ++i) so[i] = s[order[i]];
  TRY(c->upload(&Ps.subs, s));
  TRY(c->upload(&Ps.subs_ord, so));
  TRY(c->upload(&Ps.solve_order, order));
  TRY(c->upload(&Ps.tileF, sF));
  TRY(c->upload(&Ps.tileOff, sOff));
  TRY(c->dalloc(&Ps.sperm, std::max<int64_t>(lo, 1)));
  launch_fill_i32(st, lo, -1, Ps.sperm);
  launch_solve_perm(st, nsub, c->P, Ps.subs, inv, Ps.sperm);
  if (Ps.max_np > 12544) TRY(c->dalloc(&Ps.yscratch, std::max<int64_t>(lo, 1)));
  TRY(c->dalloc(s64, std::max<int64_t>(c->s_total_fac, 1)));
  if (qr) LSQ2L_HIP_TRY(hipMemsetAsync(*s64, 0, c->s_total_fac * sizeof(double), st));
  else launch_gather_solve(st, nsub, c->P, Ps, c->fac, *s64);
  return LSQ2L_OK;
}

// Everything after the matrix is resident in the handle (c->M rowptr/colind/vals).
lsq2l_status setup_core(lsq2l_ctx* c, const int32_t* rp, const int32_t* ci,
                        const HostVec<int32_t>& part, int32_t nparts,
                        const std::vector<int32_t>& seg_of_part,
                        const std::function<void(int64_t)>& wait_nnz) {
  const hipStream_t st = c->st;
  const int32_t m = c->M.m, n = c->M.n;
  const int64_t nnz = c->M.nnz;
  auto t_all = clk::now();
  auto t0 = clk::now();
  // --- transpose and index sets
  // A^T on the device, while the host plans from A's pattern
  char* temp = nullptr;
  const size_t tb = transpose_temp_bytes(nnz, n);
  TRY(c->dalloc(&c->M.trowptr, (int64_t)n + 1));
  TRY(c->dalloc(&c->M.trow, nnz));
  TRY(c->dalloc(&c->M.tperm, nnz));
  TRY(c->dalloc(&c->M.tvals, nnz));
  TRY(c->dalloc(&temp, (int64_t)std::max<size_t>(tb, 1)));
  LSQ2L_HIP_TRY(launch_transpose(st, m, n, nnz, c->M.rowptr, c->M.colind, c->M.vals, c->M.trowptr,
                                 c->M.trow, c->M.tvals, c->M.tperm, temp, tb));
  TRY(c->dalloc(&c->M.blk, spmv_table_len(nnz)));
  TRY(c->dalloc(&c->M.tblk, spmv_table_len(nnz)));
  launch_row_blocks(st, m, c->M.rowptr, nnz, c->M.blk);
  launch_row_blocks(st, n, c->M.trowptr, nnz, c->M.tblk);
  c->M.spmv_group = pick_group(m ? (double)nnz / m : 1.0);
  c->M.spmvt_group = pick_group(n ? (double)nnz / n : 1.0);
  std::string err;
  if (!plan_build(m, n, rp, ci, part.data(), nparts, seg_of_part, c->H, err, wait_nnz)) {
    set_error(err);
    return LSQ2L_EINVAL;
  }
  // Row order of the copy used for C p = A^T (A p), found on a host thread
  // while the device assembles, factors and selects (see row_order); started
  // once the planner's threads are done, so that it takes none of their cores.
  RowOrder ro;
  JoiningThread ro_thread{std::thread([&ro, m, n, rp, ci, nnz, &wait_nnz]() {
    if (wait_nnz) wait_nnz(nnz);
    row_order(m, n, rp, ci, ro);
  })};
  HostPlan& H = c->H;
  c->nsub = nparts;
  MapsJob maps;
  maps.start(n, &H);
  TRY(c->upload(&c->P.subs, H.subs));
  TRY(c->upload(&c->P.omega, H.omega));
  TRY(c->upload(&c->P.xi, H.xi));
  TRY(c->upload(&c->P.part, part));
  TRY(c->upload(&c->P.locown, H.locown));
  TRY(c->upload(&c->P.tileF, H.tileF));
  TRY(c->upload(&c->P.tileOff, H.tileOff));
  c->P.min_nG = INT32_MAX;
  for (const SubDesc& d : H.subs) {
    c->P.max_np = std::max(c->P.max_np, (int)d.np);
    c->P.min_nG = std::min(c->P.min_nG, (int)d.nG);
    c->P.max_nG = std::max(c->P.max_nG, (int)d.nG);
  }
  // the local solves and the one-workgroup-per-subdomain setup kernels start
  // the subdomains with the most stored tiles first: one launch holds all of
  // them, and the largest set its length
  std::vector<int32_t> order(nparts);
  auto upload_ordered = [&]() -> lsq2l_status {
    std::vector<SubDesc> so(nparts);
    for (int i = 0; i < nparts; ++i) so[i] = H.subs[order[i]];
    return c->upload(&c->P.subs_ord, so);
  };
  {
    std::vector<int64_t> tiles(nparts);
    for (int i = 0; i < nparts; ++i) {
      order[i] = i;
      const int64_t f0 = H.subs[i].fac_off / TT;
      const int64_t f1 = i + 1 < nparts ? H.subs[i + 1].fac_off / TT : H.total_fac / TT;
      tiles[i] = f1 - f0;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tiles[x] > tiles[y]; });
    TRY(c->upload(&c->P.solve_order, order));
    TRY(upload_ordered());
    static std::once_flag once;
    static hipError_t conf = hipSuccess;
    std::call_once(once, []() { conf = local_solve_configure(); });
    LSQ2L_HIP_TRY(conf);
  }
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
  TRY(solve_layout_begin(c));
  const bool qr = c->opt.local_factor == LSQ2L_FACTOR_QR;
  if (qr) {
    // QR local factors (Remarks 3.1, 3.2): no C_ii is formed.  The pattern
    // pass of the assembly still gives the envelope of the global-order
    // layouts; the equilibration's scaling comes from the column norms of A.
    if (c->sl_inv) launch_assemble(st, nparts, c->P, c->M, nullptr, nullptr, c->sl_inv, c->sl_dg, c->sl_Fg);
    launch_col_scale(st, nparts, c->P, c->M, c->scale);
  } else if (c->opt.diag_shift_rel <= 0.0) {
    // S = diag(C_ii)^{-1/2} = 1 / ||A(:, c)|| first, then S C_ii S and
    // S Ct_GG S assembled in one pass
    c->shift = 0.0;
    launch_col_scale(st, nparts, c->P, c->M, c->scale);
    launch_assemble(st, nparts, c->P, c->M, c->fac, c->ctg, c->sl_inv, c->sl_dg, c->sl_Fg,
                    c->scale);
  } else {
  launch_assemble(st, nparts, c->P, c->M, c->fac, c->ctg, c->sl_inv, c->sl_dg, c->sl_Fg);
  // Global shift of Section 4.1 ("Setup phase"): the preconditioner is built
  // for C + s I, s = diag_shift_rel ||C||_F, i.e. for the least-squares
  // matrix [A; sqrt(s) I].  Its rows sqrt(s) e_j enter Xi_i for j in
  // Omega_Ii only, so C_ii gains s I, Ct_GG is unchanged, and the diagonal
  // blocks of E gain s X_i^T X_i.  ||C||_F^2 sums, over the subdomains, the
  // squares of their interior rows of C.
  c->shift = 0.0;
  if (c->opt.diag_shift_rel > 0.0) {
    double* fr = nullptr;
    TRY(c->dalloc(&fr, nparts));
    launch_frob_interior(st, nparts, c->P, c->fac, fr);
    std::vector<double> h(nparts);
    LSQ2L_HIP_TRY(hipMemcpyAsync(h.data(), fr, sizeof(double) * nparts, hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));
    // a batch uses the largest instance norm (the shift only guards
    // definiteness of the local and coarse factorizations)
    std::vector<double> f2(c->S, 0.0);
    for (int i = 0; i < nparts; ++i) f2[seg_of_part[i]] += h[i];
    double fmax = 0.0;
    for (double v : f2) fmax = std::max(fmax, v);
    c->shift = c->opt.diag_shift_rel * std::sqrt(fmax);
    if (c->shift > 0.0) launch_add_diag(st, nparts, c->P, c->shift, c->fac);
  }
  launch_equilibrate(st, nparts, c->P, c->fac, c->ctg, c->scale);
  }
  // the layout of the solve factors and the gather of its matrix (before
  // c->fac is factored in place)
  double* s64 = nullptr;
  TRY(solve_layout(c, &s64));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  c->info.t_assemble_ms = ms_since(t0);
  // --- batched local Cholesky: the selection's factors (FP64, [I, Gamma])
  // on st; then the solve factors (FP64, or FP32 on MFMA in the mixed path)
  // on st2, where they overlap the selection and the coarse operator (joined
  // at the end of the setup, finish_solve_factors).  Both factorizations
  // are bound by the tile-column chains of the largest subdomains and slow
  // each other down when they run together; the selection's kernels leave
  // room beside them.
  t0 = clk::now();
  const bool mixed = c->opt.precision == LSQ2L_MIXED;
  // with solve factors of their own, the selection's factor needs L_I and
  // L_GI only (T = L_GI L_GI^T and X = L_I^{-T} L_GI^T Y).  The QR route
  // merges the rows of A into R; its row strips (zero between uses) are one
  // per stream.
  double* qstrip = nullptr;
  int32_t* qscr = nullptr;
  const int64_t strip_len = (int64_t)QR_STRIP_ROWS * H.total_loc;
  const int64_t qscr_len = 2 * H.total_loc + nparts;
  if (qr) {
    // the two QR factorizations are bound by the row-block chains of the
    // largest subdomains and leave room beside each other: the solve
    // factors start first on st2 (below), the selection's on st after them
    TRY(c->dalloc(&qstrip, strip_len));
    TRY(c->dalloc(&qscr, qscr_len));
    LSQ2L_HIP_TRY(hipMemsetAsync(qstrip, 0, strip_len * sizeof(double), st));
  } else {
    launch_chol_local(st, nparts, c->P, c->fac, c->dinv, c->status, c->solve_plan);
  }
  if (c->solve_plan) {
    double* qdinv = nullptr;     // FP64 inverse diagonal tiles of the QR solve factors
    double* qstrip2 = nullptr;
    int32_t* qscr2 = nullptr;
    if (mixed) {
      TRY(c->dalloc(&c->fac32, c->s_total_fac));
      TRY(c->dalloc(&c->dinv32, c->s_total_dinv));
      if (qr) TRY(c->dalloc(&qdinv, c->s_total_dinv));
    } else {
      c->sfac = s64;
      TRY(c->dalloc(&c->sdinv, c->s_total_dinv));
      qdinv = c->sdinv;
    }
    if (qr) {
      TRY(c->dalloc(&qstrip2, strip_len));
      TRY(c->dalloc(&qscr2, qscr_len));
      LSQ2L_HIP_TRY(hipMemsetAsync(qstrip2, 0, strip_len * sizeof(double), st));
    }
    if (!c->st2) LSQ2L_HIP_TRY(hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking));
    if (!c->ev_fork) LSQ2L_HIP_TRY(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    if (!c->ev_join) LSQ2L_HIP_TRY(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    LSQ2L_HIP_TRY(hipEventRecord(c->ev_fork, st));   // after the gather (Cholesky: and the first factor)
    LSQ2L_HIP_TRY(hipStreamWaitEvent(c->st2, c->ev_fork, 0));
    if (qr) {
      launch_qr_local(c->st2, QR_SOLVE, nparts, c->P, c->Ps, c->M, c->sl_inv, c->scale, s64, qdinv,
                      qstrip2, qscr2, H.total_loc, c->status + 2);
      if (mixed) {
        launch_to_float(c->st2, c->s_total_fac, s64, c->fac32);
        launch_to_float(c->st2, c->s_total_dinv, qdinv, c->dinv32);
      }
    } else if (mixed) {
      launch_to_float(c->st2, c->s_total_fac, s64, c->fac32);
      launch_chol_local_f32(c->st2, nparts, c->Ps, c->fac32, c->dinv32, c->status + 2);
    } else {
      launch_chol_local(c->st2, nparts, c->Ps, c->sfac, c->sdinv, c->status + 2);
    }
    LSQ2L_HIP_TRY(hipEventRecord(c->ev_join, c->st2));
  }
  if (qr)
    launch_qr_local(st, QR_SEL, nparts, c->P, c->P, c->M, nullptr, c->scale, c->fac, c->dinv, qstrip,
                    qscr, H.total_loc, c->status);
  int32_t hstat[8];
  LSQ2L_HIP_TRY(hipMemcpyAsync(hstat, c->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  if (hstat[0] != 0) {
    if (qr)
      set_error("QR local factor failed in subdomain " + std::to_string(hstat[0] - 1) +
                " (A(Xi_i, Omega_Ii) rank deficient, or more than 32,768 positions)");
    else
      set_error("local Cholesky breakdown in subdomain " + std::to_string(hstat[0] - 1));
    if (c->st2) (void)hipStreamSynchronize(c->st2);
    return LSQ2L_CHOL_BREAKDOWN;
  }
  c->info.t_factor_ms = ms_since(t0);
  // joins st2 and checks the solve factors; a broken float factorization
  // is replaced by the double one, rounded
  auto finish_solve_factors = [&]() -> lsq2l_status {
    c->info.mixed_fallback = 0;
    if (!c->solve_plan) return LSQ2L_OK;
    LSQ2L_HIP_TRY(hipStreamWaitEvent(st, c->ev_join, 0));
    int32_t hs = 0;
    LSQ2L_HIP_TRY(hipMemcpyAsync(&hs, c->status + 2, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));
    if (hs != 0 && qr) {
      set_error("QR solve factor failed in subdomain " + std::to_string(hs - 1) +
                " (A(:, Omega_i) rank deficient, or more than 32,768 positions)");
      return LSQ2L_CHOL_BREAKDOWN;
    }
    if (hs != 0 && mixed) {
      c->info.mixed_fallback = 1;
      double* d64 = nullptr;
      TRY(c->dalloc(&d64, c->s_total_dinv));
      launch_chol_local(st, nparts, c->Ps, s64, d64, c->status + 3);
      launch_to_float(st, c->s_total_fac, s64, c->fac32);
      launch_to_float(st, c->s_total_dinv, d64, c->dinv32);
      LSQ2L_HIP_TRY(hipMemcpyAsync(&hs, c->status + 3, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      LSQ2L_HIP_TRY(hipStreamSynchronize(st));
      if (hs != 0) {
        set_error("local Cholesky breakdown in subdomain " + std::to_string(hs - 1));
        return LSQ2L_CHOL_BREAKDOWN;
      }
    } else if (hs != 0) {
      set_error("local Cholesky breakdown in subdomain " + std::to_string(hs - 1) +
                " (global-column order)");
      return LSQ2L_CHOL_BREAKDOWN;
    }
    return LSQ2L_OK;
  };
  // --- coarse space
  c->p_h.assign(nparts, 0);
  c->coarse = false;
  c->n0 = 0;
  c->n0tot = 0;
  t0 = clk::now();
  const bool two_level = c->opt.variant != LSQ2L_ONE_LEVEL && c->opt.variant != LSQ2L_RAS;
  if (two_level) {
    double *Tg = nullptr, *work = nullptr, *sig = nullptr;
    int32_t* pc = nullptr;
    TRY(c->dalloc(&Tg, H.total_g));
    TRY(c->dalloc(&work, SEL_WORK_MATS * H.total_g));
    TRY(c->dalloc(&sig, H.total_loc));
    TRY(c->dalloc(&pc, nparts + 1));
    if (H.total_g) LSQ2L_HIP_TRY(hipMemsetAsync(work, 0, SEL_WORK_MATS * H.total_g * sizeof(double), st));
    LSQ2L_HIP_TRY(hipMemsetAsync(pc, 0, (nparts + 1) * sizeof(int32_t), st));
    launch_gamma_T(st, nparts, c->P, c->fac, Tg);
    // QR route: the interface factors R_G of A(Xi_i, Omega_Gamma_i) replace Ct_GG
    if (qr)
      launch_qr_local(st, QR_GAMMA, nparts, c->P, c->P, c->M, nullptr, c->scale, c->ctg, nullptr,
                      qstrip, qscr, H.total_loc, c->status + 4);
    launch_select(st, nparts, c->P, c->ctg, Tg, work, c->tau, c->opt.nev_max, pc, sig, qr ? 1 : 0);
    std::vector<int32_t> ph(nparts + 1);
    int32_t gstat = 0;
    LSQ2L_HIP_TRY(hipMemcpyAsync(ph.data(), pc, (nparts + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (qr) LSQ2L_HIP_TRY(hipMemcpyAsync(&gstat, c->status + 4, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));
    if (gstat != 0) {
      set_error("QR interface factor failed in subdomain " + std::to_string(gstat - 1) +
                " (interface beyond the QR kernel's tables)");
      return LSQ2L_CHOL_BREAKDOWN;
    }
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
    {
      SubDesc* d_subs = nullptr;       // the coarse offsets filled in by plan_coarse
      TRY(c->upload(&d_subs, H.subs));
      c->P.subs = d_subs;
      TRY(upload_ordered());
    }
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
      if (c->shift > 0.0)
        launch_coarse_E_shift(st, (int)(CP.items.size() / 4), c->P, c->Cc, c->X, c->shift, c->efac);
      // right-looking Cholesky of E, one tile column per launch, each launch
      // also applying the previous column to the tiles right of the current
      // one (rows of column J - 1 below J: its list without row J).  E is
      // block diagonal over the instances of a batch, so launch s takes
      // tile column s of every instance that has one.
      TRY(c->upload(&c->Cc.erows, CP.erows));
      TRY(c->upload(&c->Cc.eptr, CP.eptr));
      {
        int64_t steps = 0;
        for (const SegDesc& sg : CP.segs) steps = std::max(steps, sg.etiles);
        std::vector<int32_t> jobs;
        std::vector<int64_t> first(1, 0);       // first job of every step
        std::vector<int32_t> nblk;              // workgroups of every step
        for (int64_t sidx = 0; sidx < steps; ++sidx) {
          int32_t blocks = 0;
          for (const SegDesc& sg : CP.segs) {
            if (sg.etiles <= sidx) continue;
            const int64_t J = sg.etile0 + sidx;
            const int nr = (int)(CP.eptr[J + 1] - CP.eptr[J]);
            int64_t p0 = CP.eptr[J], p1 = CP.eptr[J];
            if (sidx > 0) {
              p0 = CP.eptr[J - 1];
              p1 = CP.eptr[J];
              if (p0 < p1 && CP.erows[p0] == J) ++p0;
            }
            jobs.insert(jobs.end(), {(int32_t)J, (int32_t)CP.eptr[J], nr, (int32_t)p0,
                                     (int32_t)(p1 - p0), blocks});
            blocks += echol_job_blocks(nr, (int)(p1 - p0));
          }
          first.push_back((int64_t)(jobs.size() / EJOB_INTS));
          nblk.push_back(blocks);
        }
        int32_t* d_jobs = nullptr;
        TRY(c->upload(&d_jobs, jobs));
        for (int64_t sidx = 0; sidx < steps; ++sidx)
          launch_echol_step(st, c->Cc, d_jobs + EJOB_INTS * first[sidx],
                            (int)(first[sidx + 1] - first[sidx]), nblk[sidx], c->efac, c->edinv,
                            c->status + 1);
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
        int ncu = 0, dev = 0;
        LSQ2L_HIP_TRY(hipGetDevice(&dev));
        LSQ2L_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
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
    TRY(c->dalloc(&Mi.colind, nnz));
    TRY(c->dalloc(&Mi.vals, nnz));
    TRY(c->dalloc(&Mi.trowptr, (int64_t)n + 1));
    TRY(c->dalloc(&Mi.trow, nnz));
    TRY(c->dalloc(&Mi.tperm, nnz));
    TRY(c->dalloc(&Mi.tvals, nnz));
    TRY(c->upload(&dperm, ro.perm));
    TRY(c->upload(&Mi.rowptr, ro.prp));
    launch_permute_rows(st, m, dperm, c->M.rowptr, c->M.colind, c->M.vals, Mi.rowptr, Mi.colind, Mi.vals);
    LSQ2L_HIP_TRY(launch_transpose(st, m, n, nnz, Mi.rowptr, Mi.colind, Mi.vals, Mi.trowptr, Mi.trow,
                                   Mi.tvals, Mi.tperm, temp, tb));
    TRY(c->dalloc(&Mi.blk, spmv_table_len(nnz)));
    TRY(c->dalloc(&Mi.tblk, spmv_table_len(nnz)));
    launch_row_blocks(st, m, Mi.rowptr, nnz, Mi.blk);
    launch_row_blocks(st, n, Mi.trowptr, nnz, Mi.tblk);
  }
  // --- solve workspace
  const int S = c->S;
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
  if (c->opt.variant == LSQ2L_BALANCED || c->opt.variant == LSQ2L_DEFLATED) {
    TRY(c->dalloc(&c->bal_u, n));
    TRY(c->dalloc(&c->bal_w, n));
  }
  TRY(c->dalloc(&c->bsave, m));
  TRY(c->dalloc(&c->loc, H.total_loc));
  TRY(c->dalloc(&c->partial, (int64_t)S * RED_BLOCKS));
  TRY(c->dalloc(&c->partial2, (int64_t)S * RED_BLOCKS));
  double* scal = nullptr;
  TRY(c->dalloc(&scal, 6 * (int64_t)S));
  c->sc.rho = scal; c->sc.alpha = scal + S; c->sc.beta = scal + 2 * S;
  c->sc.rn2 = scal + 3 * S; c->sc.r0n2 = scal + 4 * S; c->sc.pq = scal + 5 * S;
  TRY(c->dalloc(&c->sc.done, S));
  TRY(c->dalloc(&c->sc.its, S));
  TRY(c->halloc(&c->h_done, S));
  TRY(c->halloc(&c->h_its, S));
  TRY(c->halloc(&c->h_rn2, S));
  TRY(c->halloc(&c->h_r0n2, S));
  TRY(c->halloc(&c->h_part, (int64_t)S * RED_BLOCKS));
  TRY(c->upload(&c->d_seg_col, c->seg_col_h));
  TRY(c->upload(&c->d_seg_row, c->seg_row_h));
  TRY(krylov_alloc(c));
  TRY(finish_solve_factors());
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  c->release_staged();
  if (c->opt.autotune) TRY(autotune_spmv(c, 10));
  // --- info
  lsq2l_setup_info& inf = c->info;
  inf.m = m; inf.n = n; inf.nnz = nnz; inf.nparts = nparts; inf.ninstances = S;
  inf.n0 = c->n0;
  inf.max_ni = 0; inf.max_p = 0;
  int64_t dense = 0;
  for (const SubDesc& d : H.subs) {
    inf.max_ni = std::max(inf.max_ni, d.nI + d.nG);
    inf.max_p = std::max(inf.max_p, d.p);
    dense += (int64_t)(d.nI + d.nG) * (d.nI + d.nG + 1) / 2 * (int64_t)sizeof(double);
  }
  const int64_t solve_fac = c->solve_plan ? c->s_total_fac : H.total_fac;
  inf.factor_tiles = solve_fac / TT;
  inf.factor_bytes = solve_fac * (c->opt.precision == LSQ2L_MIXED ? sizeof(float) : sizeof(double));
  inf.factor_dense_bytes = dense;
  inf.factor_nnz_min = -1;
  inf.shift = c->shift;
  inf.spmv_lanes_A = c->M.spmv_group;
  inf.spmv_lanes_AT = c->M.spmvt_group;
  inf.t_total_ms = ms_since(t_all);
  return LSQ2L_OK;
}

lsq2l_status check_common(double tau, const lsq2l_options* opt) {
  if (!(tau > 0.0 && tau <= 1.0)) { set_error("tau must lie in (0, 1]"); return LSQ2L_EINVAL; }
  if (opt) {
    if (!(opt->tol > 0.0)) { set_error("tol must be positive"); return LSQ2L_EINVAL; }
    if (opt->max_it < 1) { set_error("max_it must be >= 1"); return LSQ2L_EINVAL; }
    if (opt->precision != LSQ2L_FP64 && opt->precision != LSQ2L_MIXED) { set_error("bad precision"); return LSQ2L_EINVAL; }
    if (opt->variant < LSQ2L_ADDITIVE || opt->variant > LSQ2L_DEFLATED) { set_error("bad variant"); return LSQ2L_EINVAL; }
    if (opt->krylov < LSQ2L_PCG || opt->krylov > LSQ2L_GMRES) { set_error("bad krylov method"); return LSQ2L_EINVAL; }
    if (opt->krylov != LSQ2L_GMRES && (opt->variant == LSQ2L_RAS || opt->variant == LSQ2L_DEFLATED)) {
      set_error("RAS and DEFLATED are nonsymmetric preconditioners: use them with GMRES");
      return LSQ2L_EINVAL;
    }
    if (opt->krylov == LSQ2L_GMRES && (opt->restart < 1 || opt->restart > 1000)) {
      set_error("restart must lie in [1, 1000]");
      return LSQ2L_EINVAL;
    }
    if (opt->nev_max < 0) { set_error("nev_max must be >= 0"); return LSQ2L_EINVAL; }
    if (opt->solve_order < LSQ2L_ORDER_AUTO || opt->solve_order > LSQ2L_ORDER_GLOBAL) {
      set_error("bad solve_order");
      return LSQ2L_EINVAL;
    }
    if (!(opt->diag_shift_rel >= 0.0) || !(opt->adjoint_tol >= 0.0)) {
      set_error("diag_shift_rel and adjoint_tol must be >= 0");
      return LSQ2L_EINVAL;
    }
    if (opt->local_factor != LSQ2L_FACTOR_CHOLESKY && opt->local_factor != LSQ2L_FACTOR_QR) {
      set_error("bad local_factor");
      return LSQ2L_EINVAL;
    }
    if (opt->local_factor == LSQ2L_FACTOR_QR && opt->diag_shift_rel > 0.0) {
      set_error("the QR local factors take no diagonal shift (diag_shift_rel must be 0)");
      return LSQ2L_EINVAL;
    }
  }
  return LSQ2L_OK;
}

// Memory allocated on a device with hipMalloc (anything else, plain or
// pinned host memory, is read on the host).
bool is_device_ptr(const void* p) {
  hipPointerAttribute_t at;
  const hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

// Device-to-host copy of the concatenated column indices in chunks, each
// closed by an event.  head closes everything queued before the chunks.  The
// destructor waits for the last chunk, so the pinned buffer is never handed
// back while a copy into it is in flight (also on early error returns).
struct PatternChunks {
  static constexpr int NCH = 8;
  hipEvent_t head = nullptr;
  hipEvent_t ev[NCH] = {};
  int64_t bound[NCH + 1] = {};
  int nch = 0;
  lsq2l_status start(hipStream_t st, int32_t* host, const int32_t* dev, int64_t nnz) {
    LSQ2L_HIP_TRY(hipEventCreateWithFlags(&head, hipEventDisableTiming));
    LSQ2L_HIP_TRY(hipEventRecord(head, st));
    const int want = nnz >= ((int64_t)1 << 20) ? NCH : (nnz > 0 ? 1 : 0);
    for (int q = 0; q < want; ++q) {
      const int64_t a = nnz * q / want, b = nnz * (q + 1) / want;
      LSQ2L_HIP_TRY(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming));
      nch = q + 1;
      bound[q] = a;
      bound[q + 1] = b;
      if (b > a)
        LSQ2L_HIP_TRY(hipMemcpyAsync(host + a, dev + a, (b - a) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      LSQ2L_HIP_TRY(hipEventRecord(ev[q], st));
    }
    return LSQ2L_OK;
  }
  // returns once entries [0, upto) are in place
  void wait(int64_t upto) const {
    for (int q = nch - 1; q >= 0; --q)
      if (bound[q] < upto) {              // chunks complete in order: the last one needed suffices
        (void)hipEventSynchronize(ev[q]);
        return;
      }
  }
  ~PatternChunks() {
    if (nch > 0) (void)hipEventSynchronize(ev[nch - 1]);
    for (int q = 0; q < nch; ++q) (void)hipEventDestroy(ev[q]);
    if (head) (void)hipEventDestroy(head);
  }
};

// Setup of one or several instances: their CSR arrays are concatenated and
// checked on the device in three launches (launch_concat), and the
// concatenated pattern is read back once into pinned memory for the planner.
lsq2l_status setup_instances(lsq2l_ctx* c, int count, const lsq2l_problem* probs) {
  auto t_prep = clk::now();
  const hipStream_t st = c->st;
  int64_t M = 0, N = 0, NNZ = 0, NP = 0;
  for (int k = 0; k < count; ++k) {
    const lsq2l_problem& pr = probs[k];
    if (pr.m < 1 || pr.n < 1 || pr.m < pr.n || pr.nnz < 0 || pr.nparts < 1 || pr.nparts > pr.n ||
        !pr.rowptr || !pr.part || (pr.nnz > 0 && (!pr.colind || !pr.vals))) {
      set_error(count == 1 ? std::string("bad sizes or pointers: need m >= n >= 1, 1 <= nparts <= n")
                           : "bad problem " + std::to_string(k));
      return LSQ2L_EINVAL;
    }
    M += pr.m; N += pr.n; NNZ += pr.nnz; NP += pr.nparts;
  }
  if (M >= INT32_MAX || N >= INT32_MAX || NNZ >= INT32_MAX) {
    set_error("m, n and nnz (summed over the instances) must stay below 2^31");
    return LSQ2L_EINVAL;
  }
  c->S = count;
  c->M.m = (int32_t)M; c->M.n = (int32_t)N; c->M.nnz = NNZ;
  c->seg_row_h.assign(count + 1, 0);
  c->seg_col_h.assign(count + 1, 0);
  TRY(c->dalloc(&c->M.rowptr, M + 1));
  TRY(c->dalloc(&c->M.colind, NNZ));
  TRY(c->dalloc(&c->M.vals, NNZ));
  std::vector<int64_t> r0(count + 1, 0), c0(count + 1, 0), e0(count + 1, 0), p0(count + 1, 0);
  std::vector<InstDesc> desc(count);
  for (int k = 0; k < count; ++k) {
    r0[k + 1] = r0[k] + probs[k].m;
    c0[k + 1] = c0[k] + probs[k].n;
    e0[k + 1] = e0[k] + probs[k].nnz;
    p0[k + 1] = p0[k] + probs[k].nparts;
    desc[k] = InstDesc{probs[k].rowptr, probs[k].colind, probs[k].vals, probs[k].m, probs[k].n,
                       probs[k].nnz, r0[k], c0[k], e0[k]};
  }
  for (int k = 0; k <= count; ++k) {
    c->seg_row_h[k] = r0[k];
    c->seg_col_h[k] = c0[k];
  }
  InstDesc* d_desc = nullptr;
  unsigned long long* d_bad = nullptr;
  TRY(c->upload(&d_desc, desc));
  TRY(c->dalloc(&d_bad, CSR_KINDS));
  launch_concat(st, count, d_desc, M, NNZ, c->M.rowptr, c->M.colind, c->M.vals, d_bad);
  PinnedArray<int32_t> rp, ci;
  TRY(rp.alloc(M + 1));
  TRY(ci.alloc(NNZ));
  unsigned long long hbad[CSR_KINDS];
  LSQ2L_HIP_TRY(hipMemcpyAsync(hbad, d_bad, sizeof(hbad), hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(rp.p, c->M.rowptr, (M + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  // partitions: host arrays are read in place, device arrays copied back
  HostVec<int32_t> pt;
  std::vector<int32_t> seg_of_part(NP);
  if (!pt.resize(N)) { set_error("host allocation failed"); return LSQ2L_ENOMEM; }
  std::vector<PinnedArray<int32_t>> pdev(count);
  for (int k = 0; k < count; ++k)
    if (is_device_ptr(probs[k].part)) {
      TRY(pdev[k].alloc(probs[k].n));
      LSQ2L_HIP_TRY(hipMemcpyAsync(pdev[k].p, probs[k].part, probs[k].n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    }
  // the column indices come back in chunks, each closed by an event, so that
  // the planner starts on the rows that have arrived while the rest is in
  // flight (the checks, row pointers and parts are waited for here)
  PatternChunks chunks;
  TRY(chunks.start(st, ci.p, c->M.colind, NNZ));
  const hipError_t e = hipEventSynchronize(chunks.head);
  if (e != hipSuccess) { set_error(std::string("reading A: ") + hipGetErrorString(e)); return LSQ2L_EHIP; }
  // the first failure in the order of the checks: row extents, then columns
  // (reported only when the extents hold)
  for (int kind : {CSR_FIRST, CSR_LAST, CSR_MONO, CSR_RANGE, CSR_ORDER}) {
    if (hbad[kind] == ~0ull) continue;
    const int64_t g = (int64_t)hbad[kind];
    const int k = (int)(std::upper_bound(r0.begin(), r0.end(), g) - r0.begin()) - 1;
    const std::string who = count > 1 ? "problem " + std::to_string(k) + ": " : std::string();
    const std::string row = std::to_string(g - r0[k]);
    static const char* what[CSR_KINDS] = {"rowptr[0] must be 0", "rowptr[m] != nnz",
                                          "rowptr is not monotone (or exceeds nnz) at row ",
                                          "column index out of range in row ",
                                          "columns not strictly increasing in row "};
    set_error(who + what[kind] + (kind >= CSR_MONO ? row : std::string()));
    return LSQ2L_EINVAL;
  }
  // global part numbers, checked, in parallel over column ranges
  {
    const unsigned nth = N < (1 << 16) ? 1u : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<int64_t> bad(nth, -1);
    std::vector<std::thread> pool;
    auto work = [&](unsigned t) {
      const int64_t g0 = N * t / nth, g1 = N * (t + 1) / nth;
      int k = (int)(std::upper_bound(c0.begin(), c0.end(), g0) - c0.begin()) - 1;
      for (int64_t g = g0; g < g1; ++g) {
        while (g >= c0[k + 1]) ++k;
        const int32_t* part = pdev[k].p ? pdev[k].p : probs[k].part;
        const int32_t v = part[g - c0[k]];
        if (v < 0 || v >= probs[k].nparts) { bad[t] = g; return; }
        pt[g] = (int32_t)(p0[k] + v);
      }
    };
    if (nth == 1) work(0);
    else {
      for (unsigned t = 0; t < nth; ++t) pool.emplace_back(work, t);
      for (auto& th : pool) th.join();
    }
    for (unsigned t = 0; t < nth; ++t)
      if (bad[t] >= 0) {
        const int k = (int)(std::upper_bound(c0.begin(), c0.end(), bad[t]) - c0.begin()) - 1;
        set_error(count == 1 ? "part[" + std::to_string(bad[t]) + "] out of range"
                             : "part out of range in problem " + std::to_string(k));
        return LSQ2L_EINVAL;
      }
  }
  for (int k = 0; k < count; ++k)
    for (int32_t q = 0; q < probs[k].nparts; ++q) seg_of_part[p0[k] + q] = k;
  c->info.t_prepare_ms = ms_since(t_prep);
  return setup_core(c, rp.p, ci.p, pt, (int32_t)NP, seg_of_part,
                    [&chunks](int64_t e) { chunks.wait(e); });
}

lsq2l_ctx* new_handle(double tau, const lsq2l_options* opt, void* hip_stream) {
  lsq2l_ctx* c = new lsq2l_ctx();
  c->st = (hipStream_t)hip_stream;
  lsq2l_default_options(&c->opt);
  if (opt) c->opt = *opt;
  c->tau = tau;
  return c;
}

lsq2l_status autotune_spmv(lsq2l_ctx* c, int reps) {
  hipEvent_t e0, e1;
  LSQ2L_HIP_TRY(hipEventCreate(&e0));
  LSQ2L_HIP_TRY(hipEventCreate(&e1));
  struct Ev { hipEvent_t a, b; ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } ev{e0, e1};
  launch_fill(c->st, c->M.n, 1.0, c->p);
  launch_fill(c->st, c->M.m, 1.0, c->tm);
  DevMatrix& M = c->row_perm ? c->Mi : c->M;
  for (int which = 0; which < 2; ++which) {
    int best = 0;
    float best_ms = 1e30f;
    for (int g = SPMV_ROWS_STREAM; g <= 64; g = g < 1 ? g + 1 + (g == -1) : 2 * g) {
      auto once = [&]() {
        if (which == 0) launch_spmv(c->st, M.m, M.rowptr, M.colind, M.vals, c->p, c->tm2, g, M.nnz, M.blk);
        else launch_spmv(c->st, M.n, M.trowptr, M.trow, M.tvals, c->tm, c->q, g, M.nnz, M.tblk);
      };
      once();
      LSQ2L_HIP_TRY(hipEventRecord(e0, c->st));
      for (int k = 0; k < reps; ++k) once();
      LSQ2L_HIP_TRY(hipEventRecord(e1, c->st));
      LSQ2L_HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      LSQ2L_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) { best_ms = ms; best = g; }
    }
    if (which == 0) { c->M.spmv_group = best; c->Mi.spmv_group = best; }
    else { c->M.spmvt_group = best; c->Mi.spmvt_group = best; }
  }
  c->info.spmv_lanes_A = c->M.spmv_group;
  c->info.spmv_lanes_AT = c->M.spmvt_group;
  return LSQ2L_OK;
}

lsq2l_status solve_dispatch(lsq2l_ctx* c, double* x, bool adjoint, lsq2l_solve_info* info) {
  auto t0 = clk::now();
  KrylovResult res;
  lsq2l_status s;
  const double tol = adjoint && c->opt.adjoint_tol > 0.0 ? c->opt.adjoint_tol : c->opt.tol;
  if (adjoint) TRY(norm_C(c));
  if (c->opt.krylov == LSQ2L_GMRES) s = gmres(c, x, adjoint, tol, res);
  else if (c->opt.krylov == LSQ2L_LSQR && !adjoint) s = lsqr(c, c->bsave, x, tol, res);
  else s = pcg(c, x, adjoint, tol, res);    // CG, and the adjoint of LSQR (M is symmetric)
  if (s != LSQ2L_OK && s != LSQ2L_NOT_CONVERGED) return s;
  const double ms = ms_since(t0);
  if (info)
    for (int k = 0; k < c->S; ++k) {
      info[k].iterations = k < (int)res.its.size() ? res.its[k] : res.total_its;
      info[k].restarts = res.restarts;
      info[k].relres = k < (int)res.relres.size() ? res.relres[k] : 0.0;
      info[k].relres_rec = k < (int)res.relres_rec.size() ? res.relres_rec[k] : 0.0;
      info[k].solve_ms = ms;
      info[k].backward_err = adjoint && k < (int)res.backward_err.size() ? res.backward_err[k] : 0.0;
    }
  return s;
}

}  // namespace
}  // namespace lsq2l

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
  opt->krylov = LSQ2L_PCG;
  opt->restart = 100;
  opt->diag_shift_rel = 0.0;
  opt->adjoint_tol = 0.0;
  opt->autotune = 0;
  opt->solve_order = LSQ2L_ORDER_AUTO;
  opt->local_factor = LSQ2L_FACTOR_CHOLESKY;
}

const char* lsq2l_last_error(void) { return g_err.c_str(); }

lsq2l_status lsq2l_setup(int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                         const int32_t* colind, const double* vals, const int32_t* part,
                         int32_t nparts, int32_t overlap, double tau, const lsq2l_options* opt,
                         void* hip_stream, lsq2l_handle* out) {
  g_err.clear();
  if (!out) { set_error("out is NULL"); return LSQ2L_EINVAL; }
  *out = nullptr;
  if (overlap != 1) { set_error("only overlap = 1 (one layer, Section 3) is supported"); return LSQ2L_EINVAL; }
  TRY(check_common(tau, opt));
  lsq2l_problem pr{};
  pr.m = m; pr.n = n; pr.nnz = nnz;
  pr.rowptr = rowptr; pr.colind = colind; pr.vals = vals; pr.part = part; pr.nparts = nparts;
  lsq2l_ctx* c = new_handle(tau, opt, hip_stream);
  const lsq2l_status s = setup_instances(c, 1, &pr);
  if (s != LSQ2L_OK) { delete c; return s; }
  *out = c;
  return LSQ2L_OK;
}

lsq2l_status lsq2l_setup_batched(int32_t count, const lsq2l_problem* probs, double tau,
                                 const lsq2l_options* opt, void* hip_stream, lsq2l_handle* out) {
  g_err.clear();
  if (!out || !probs || count < 1) { set_error("bad arguments"); return LSQ2L_EINVAL; }
  *out = nullptr;
  TRY(check_common(tau, opt));
  lsq2l_ctx* c = new_handle(tau, opt, hip_stream);
  const lsq2l_status s = setup_instances(c, count, probs);
  if (s != LSQ2L_OK) { delete c; return s; }
  *out = c;
  return LSQ2L_OK;
}

lsq2l_status lsq2l_solve(lsq2l_handle c, const double* b, double* x, lsq2l_solve_info* info) {
  g_err.clear();
  if (!c || !b || !x) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  c->have_solution = false;
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->bsave, b, c->M.m * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  spmv_AT(c, b, c->rhs);
  const lsq2l_status s = solve_dispatch(c, x, false, info);
  if (s != LSQ2L_OK && s != LSQ2L_NOT_CONVERGED) return s;
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->xsave, x, c->M.n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  c->have_solution = true;
  return s;
}

lsq2l_status lsq2l_solve_batched(lsq2l_handle c, const double* const* b, double* const* x,
                                 lsq2l_solve_info* info) {
  g_err.clear();
  if (!c || !b || !x) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  for (int k = 0; k < c->S; ++k)
    if (!b[k] || !x[k]) { set_error("NULL right-hand side or solution of instance " + std::to_string(k)); return LSQ2L_EINVAL; }
  c->have_solution = false;
  for (int k = 0; k < c->S; ++k) {
    const int64_t r0 = c->seg_row_h[k], mk = c->seg_row_h[k + 1] - r0;
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->bsave + r0, b[k], mk * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  }
  spmv_AT(c, c->bsave, c->rhs);
  const lsq2l_status s = solve_dispatch(c, c->xsave, false, info);
  if (s != LSQ2L_OK && s != LSQ2L_NOT_CONVERGED) return s;
  for (int k = 0; k < c->S; ++k) {
    const int64_t c0 = c->seg_col_h[k], nk = c->seg_col_h[k + 1] - c0;
    LSQ2L_HIP_TRY(hipMemcpyAsync(x[k], c->xsave + c0, nk * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  }
  LSQ2L_HIP_TRY(hipStreamSynchronize(c->st));
  c->have_solution = true;
  return s;
}

lsq2l_status lsq2l_backward(lsq2l_handle c, const double* g, double* dLdb, double* dLdvals,
                            lsq2l_solve_info* info) {
  g_err.clear();
  if (!c || !g) { set_error("NULL argument"); return LSQ2L_EINVAL; }
  if (!c->have_solution) { set_error("backward needs a previous solve"); return LSQ2L_EINVAL; }
  LSQ2L_HIP_TRY(hipMemcpyAsync(c->rhs, g, c->M.n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  const lsq2l_status s = solve_dispatch(c, c->xwork, true, info);       // lambda = C^{-1} g
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
  out->factor_nnz_min = c->fac_nnz_min;
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
  if (kernel < 0 || kernel > 4 || (kernel == 3 && !c->coarse)) { set_error("unknown or unused kernel"); return LSQ2L_EINVAL; }
  const double m = c->M.m, n = c->M.n, nnz = (double)c->M.nnz;
  const double eb = (c->opt.precision == LSQ2L_MIXED) ? 4.0 : 8.0;
  if (kernel == 4) TRY(factor_nnz_min(c));
  switch (kernel) {
    case 0: *bytes = 12.0 * nnz + 4.0 * (m + 1) + 8.0 * n + 8.0 * m; break;
    case 1: *bytes = 12.0 * nnz + 4.0 * (n + 1) + 8.0 * m + 8.0 * n; break;
    // each sweep reads every stored off-diagonal tile and every diagonal
    // inverse once (as many elements as the stored factor), plus y in and out
    case 2:
      *bytes = c->solve_plan
                   ? 2.0 * eb * (double)c->s_total_fac + (16.0 + 8.0) * (double)c->s_total_np
                   : 2.0 * eb * (double)c->H.total_fac + 16.0 * (double)c->H.total_loc;
      break;
    // the algorithmic minimum: each sweep reads the nnz(L_i) entries of the
    // factors under a fill-reducing order, y in and out per local unknown
    case 4: {
      double nloc = 0;
      for (const SubDesc& d : c->H.subs) nloc += d.nI + d.nG;
      *bytes = 2.0 * eb * (double)c->fac_nnz_min + 16.0 * nloc;
      break;
    }
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
      case 4: local_solves(c); break;
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

lsq2l_status lsq2l_autotune(lsq2l_handle c, int32_t reps, int32_t* lanes) {
  g_err.clear();
  if (!c || reps < 0 || (reps == 0 && !lanes)) { set_error("bad arguments"); return LSQ2L_EINVAL; }
  if (reps == 0) {
    auto valid = [](int g) {
      return (g >= SPMV_ROWS_STREAM && g <= 0) || (g >= 1 && g <= 64 && (g & (g - 1)) == 0);
    };
    if (!valid(lanes[0]) || !valid(lanes[1])) {
      set_error("SpMV shape must be -2, -1, 0 or a power of two up to 64");
      return LSQ2L_EINVAL;
    }
    c->M.spmv_group = c->Mi.spmv_group = lanes[0];
    c->M.spmvt_group = c->Mi.spmvt_group = lanes[1];
    c->info.spmv_lanes_A = lanes[0];
    c->info.spmv_lanes_AT = lanes[1];
    return LSQ2L_OK;
  }
  TRY(autotune_spmv(c, reps));
  if (lanes) { lanes[0] = c->M.spmv_group; lanes[1] = c->M.spmvt_group; }
  return LSQ2L_OK;
}

lsq2l_status lsq2l_transpose(int32_t m, int32_t n, int32_t nnz, const int32_t* rowptr,
                             const int32_t* colind, const double* vals, int32_t* trowptr,
                             int32_t* trow, double* tvals, int32_t* tperm, void* hip_stream) {
  g_err.clear();
  if (m < 0 || n < 0 || nnz < 0 || !rowptr || !trowptr || (nnz > 0 && (!colind || !trow)) ||
      (nnz > 0 && tvals && !vals)) {
    set_error("bad sizes or NULL required pointer");
    return LSQ2L_EINVAL;
  }
  const hipStream_t st = (hipStream_t)hip_stream;
  const size_t tb = transpose_temp_bytes(nnz, n);
  // the sort carries the permutation; a caller that does not want it gets
  // a temporary one.  The last 256 bytes hold the column check flag.
  const size_t perm_bytes = tperm ? 0 : ((size_t)nnz * sizeof(int32_t) + 255) / 256 * 256;
  void* temp = nullptr;
  LSQ2L_HIP_TRY(hipMalloc(&temp, tb + perm_bytes + 256));
  int32_t* perm = tperm ? tperm : (int32_t*)((char*)temp + tb);
  int32_t* flag = (int32_t*)((char*)temp + tb + perm_bytes);
  int32_t hflag = 0;
  launch_check_cols(st, nnz, colind, n, flag);
  hipError_t e = hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && hflag == 0)
    e = launch_transpose(st, m, n, nnz, rowptr, colind, vals, trowptr, trow, tvals, perm, temp, tb);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(temp);
  if (e != hipSuccess) {
    set_error(std::string("transpose: ") + hipGetErrorString(e));
    return LSQ2L_EHIP;
  }
  if (hflag) {
    set_error("transpose: a column index lies outside [0, n)");
    return LSQ2L_EINVAL;
  }
  return LSQ2L_OK;
}

void lsq2l_destroy(lsq2l_handle c) { delete c; }

void lsq2l_release_cache(void) {
  cache_release();
  pinned_release();
}

}  // extern "C"
