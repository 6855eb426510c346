// The handle of the C ABI: device copies of A, the plan, the factors, the
// coarse operator and the work vectors of the Krylov methods, plus the
// memory pools it draws from.  Shared by the setup (api.cpp) and the Krylov
// drivers (krylov.cpp).
#pragma once

#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace lsq2l {

using clk = std::chrono::steady_clock;
inline double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// Device blocks of destroyed handles, kept for later handles on the same
// device (api.cpp).
void* cache_take(size_t bytes, int dev, size_t* got);
void cache_give(void* p, size_t bytes, int dev);
void cache_release();

// Pinned host buffers kept for later setups (api.cpp).
void* pinned_take(size_t bytes, size_t* got);
void pinned_give(void* p, size_t bytes);
void pinned_release();

// A pinned host array of count elements from the pool, returned to it when
// the owner goes out of scope (the work that used it has been synchronized).
template <typename T>
struct PinnedArray {
  T* p = nullptr;
  size_t bytes = 0;
  lsq2l_status alloc(int64_t count) {
    const size_t want = (((size_t)std::max<int64_t>(count, 1) * sizeof(T)) + ((1 << 20) - 1)) >> 20 << 20;
    p = (T*)pinned_take(want, &bytes);
    if (!p) {
      set_error("pinned host allocation of " + std::to_string(want) + " bytes failed");
      return LSQ2L_ENOMEM;
    }
    return LSQ2L_OK;
  }
  ~PinnedArray() {
    if (p) pinned_give(p, bytes);
  }
};

// Work vectors of LSQR (per instance scalars live in LsqrScalars).
struct LsqrWork {
  double *u = nullptr, *Av = nullptr;        // m
  double *v = nullptr, *zh = nullptr, *w = nullptr, *q = nullptr, *s = nullptr;   // n
  double* sc = nullptr;                      // LSQR_NSC scalars per instance
};

// Work of restarted GMRES: the Krylov basis V (n x (restart + 1)), the
// products of a step and the per-instance coefficients.
struct GmresWork {
  int restart = 0;
  double* V = nullptr;                       // column j at V + j n
  double *w = nullptr, *z = nullptr, *t = nullptr;   // n
  double* part = nullptr;                    // multi-dot partials
  double* h = nullptr;                       // (restart + 1) per instance, reduced
  double* y = nullptr;                       // (restart + 1) per instance
  double* nrm = nullptr;                     // per instance
  double* h_h = nullptr;                     // pinned copies
  double* h_y = nullptr;
};

}  // namespace lsq2l

struct lsq2l_ctx {
  hipStream_t st = nullptr;
  hipStream_t gst = nullptr;   // stream the PCG iteration graph is captured on
  // second stream of the setup: the solve factors are computed on it while
  // the selection and the coarse operator run on st (joined by ev_join)
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  lsq2l_options opt{};
  double tau = 0.0;
  int S = 1;
  int nsub = 0;
  std::vector<lsq2l::SegDesc> segs_h;
  std::vector<int64_t> seg_row_h, seg_col_h;
  int64_t* d_seg_row = nullptr;
  int64_t* d_seg_col = nullptr;
  lsq2l::DevMatrix M;
  lsq2l::DevMatrix Mi;      // row-permuted copy of A and its transpose for C p = A^T (A p)
  bool row_perm = false;    // Mi is in use
  lsq2l::DevPlan P;
  lsq2l::DevCoarse Cc;
  lsq2l::HostPlan H;
  lsq2l::CoarsePlan CP;
  bool coarse = false;
  int64_t n0tot = 0;        // padded coarse size over all instances
  int64_t n0 = 0;           // true coarse size
  int64_t etiles = 0;
  double shift = 0.0;       // diagonal shift of C used by the preconditioner
  double *fac = nullptr, *dinv = nullptr, *scale = nullptr, *ctg = nullptr;
  // Factors of the local solves (see solve_layout in api.cpp).  With
  // solve_plan unset they are fac / dinv in the layout P; otherwise they are
  // in the layout Ps: sfac / sdinv (FP64 path), fac32 / dinv32 (mixed path).
  bool solve_plan = false;
  lsq2l::DevPlan Ps;
  int64_t s_total_fac = 0, s_total_dinv = 0, s_total_np = 0, s_total_tiles = 0;
  // candidate global-order layouts of the setup (solve_layout_begin): host
  // copy, device copy, position map and the tile envelope the assembly finds
  std::vector<lsq2l::SubDesc> sl_g;
  lsq2l::SubDesc* sl_dg = nullptr;
  int32_t *sl_inv = nullptr, *sl_Fg = nullptr;
  int64_t sl_tiles = 0, sl_loc = 0;
  double *sfac = nullptr, *sdinv = nullptr;
  float *fac32 = nullptr, *dinv32 = nullptr;
  float* X32 = nullptr;      // MIXED: FP32 copy of X for the restriction and prolongation
  double *X = nullptr, *W = nullptr, *efac = nullptr, *edinv = nullptr, *einv = nullptr;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *rhs = nullptr, *rold = nullptr;
  double *tm = nullptr, *tm2 = nullptr, *loc = nullptr, *cvec = nullptr, *dvec = nullptr;
  double *partial = nullptr, *partial2 = nullptr, *xwork = nullptr;
  double *bsave = nullptr, *xsave = nullptr;
  double *bal_u = nullptr, *bal_w = nullptr;   // balanced / deflated forms: two n-vectors
  bool have_solution = false;
  lsq2l::Scalars sc{};
  int32_t* status = nullptr;
  int32_t* h_done = nullptr;      // pinned
  int32_t* h_its = nullptr;       // pinned
  double* h_rn2 = nullptr;        // pinned
  double* h_r0n2 = nullptr;       // pinned
  double* h_part = nullptr;       // pinned, S * RED_BLOCKS
  std::vector<double> normC;      // ||C||_2 per instance (power iteration), empty until needed
  lsq2l::LsqrWork lsqr;
  lsq2l::GmresWork gmres;
  std::vector<int32_t> p_h;
  int max_p = 0;
  int64_t fac_nnz_min = -1;       // symbolic nnz(L) under a fill-reducing order (lazy)
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
  lsq2l_status raw_alloc(void** v, size_t bytes);
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
    if (e != hipSuccess) { lsq2l::set_error("pinned host allocation failed"); return LSQ2L_ENOMEM; }
    host_allocs.push_back(v);
    *ptr = (T*)v;
    return LSQ2L_OK;
  }
  // Upload of a host vector through a pinned staging buffer of the pool: the
  // copy never reads pageable memory, and the staging buffers go back to the
  // pool only after a stream synchronization (release_staged, destructor).
  std::vector<std::pair<void*, size_t>> staged;
  template <typename T>
  lsq2l_status upload(T** dst, const std::vector<T>& src) {
    lsq2l_status s = dalloc(dst, (int64_t)src.size());
    if (s != LSQ2L_OK) return s;
    if (src.empty()) return LSQ2L_OK;
    const size_t bytes = src.size() * sizeof(T);
    size_t got = 0;
    void* p = lsq2l::pinned_take((bytes + ((1 << 20) - 1)) >> 20 << 20, &got);
    if (!p) { lsq2l::set_error("pinned staging allocation failed"); return LSQ2L_ENOMEM; }
    staged.push_back({p, got});
    std::copy(src.begin(), src.end(), (T*)p);
    LSQ2L_HIP_TRY(hipMemcpyAsync(*dst, p, bytes, hipMemcpyHostToDevice, st));
    return LSQ2L_OK;
  }
  // the caller has synchronized the stream
  // a planner array: its block is page-locked (or small), so it is copied
  // directly; it outlives the copy (kept in the handle or synchronized)
  template <typename T>
  lsq2l_status upload(T** dst, const lsq2l::HostVec<T>& src) {
    lsq2l_status s = dalloc(dst, (int64_t)src.size());
    if (s != LSQ2L_OK) return s;
    if (src.empty()) return LSQ2L_OK;
    LSQ2L_HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return LSQ2L_OK;
  }
  void release_staged() {
    for (auto& b : staged) lsq2l::pinned_give(b.first, b.second);
    staged.clear();
  }
  ~lsq2l_ctx();
};

#define TRY(expr)                             \
  do {                                        \
    lsq2l_status _s = (expr);                 \
    if (_s != LSQ2L_OK) return _s;            \
  } while (0)
