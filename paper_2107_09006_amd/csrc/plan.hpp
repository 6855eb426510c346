// Host setup planner (integer work on the sparsity pattern).
#pragma once

#include <algorithm>
#include <cstring>
#include <string>
#include <functional>
#include <vector>

#include "internal.hpp"

namespace lsq2l {

// Storage of the planner's large host arrays.  The library hands out
// page-locked blocks it keeps for later setups (no page faults when a setup
// is repeated, uploads without a staging copy); a host-only build supplies
// malloc and free.
void* host_block_take(size_t bytes, size_t* got);
void host_block_give(void* p, size_t bytes);

// A host array in such a block.  resize() leaves the contents undefined.
template <typename T>
class HostVec {
 public:
  HostVec() = default;
  HostVec(const HostVec& o) { copy_from(o); }
  HostVec(HostVec&& o) noexcept { take_from(o); }
  HostVec& operator=(const HostVec& o) {
    if (this != &o) { reset(); copy_from(o); }
    return *this;
  }
  HostVec& operator=(HostVec&& o) noexcept {
    if (this != &o) { reset(); take_from(o); }
    return *this;
  }
  ~HostVec() { reset(); }
  bool resize(size_t n) {
    if (n * sizeof(T) > bytes_) {
      reset();
      size_t got = 0;
      p_ = (T*)host_block_take(std::max<size_t>(n, 1) * sizeof(T), &got);
      if (!p_) return false;
      bytes_ = got;
    }
    n_ = n;
    return true;
  }
  bool assign(size_t n, const T& v) {
    if (!resize(n)) return false;
    std::fill(p_, p_ + n, v);
    return true;
  }
  void reset() {
    if (p_) host_block_give(p_, bytes_);
    p_ = nullptr;
    n_ = bytes_ = 0;
  }
  T* data() { return p_; }
  const T* data() const { return p_; }
  size_t size() const { return n_; }
  bool empty() const { return n_ == 0; }
  T& operator[](size_t i) { return p_[i]; }
  const T& operator[](size_t i) const { return p_[i]; }
  T* begin() { return p_; }
  T* end() { return p_ + n_; }
  const T* begin() const { return p_; }
  const T* end() const { return p_ + n_; }
  T& back() { return p_[n_ - 1]; }

 private:
  void copy_from(const HostVec& o) {
    if (o.n_ && resize(o.n_)) std::memcpy(p_, o.p_, o.n_ * sizeof(T));
  }
  void take_from(HostVec& o) {
    p_ = o.p_; n_ = o.n_; bytes_ = o.bytes_;
    o.p_ = nullptr; o.n_ = o.bytes_ = 0;
  }
  T* p_ = nullptr;
  size_t n_ = 0, bytes_ = 0;
};

struct HostPlan {
  int32_t nparts = 0;
  std::vector<SubDesc> subs;
  HostVec<int32_t> omega;        // per subdomain: Omega_Ii then Omega_Gamma_i
  HostVec<int32_t> xi;           // per subdomain: Xi_i
  HostVec<int32_t> tileF;        // first stored tile of each tile row
  HostVec<int64_t> tileOff;      // tile index of (I, F(I)) relative to fac_off / TT
  HostVec<int32_t> locown;       // position of each column inside its own interior
  HostVec<int32_t> own_ptr;      // inverse overlap map (n + 1)
  HostVec<int32_t> own_pos;      // local-buffer positions holding each column
  // rows of Xi_i shared with Xi_j (i < j), as (i, j, pos in Xi_i, pos in Xi_j)
  // in row order, one list per row range of the planner (consumed by plan_maps)
  std::vector<std::vector<int32_t>> shared_rows;
  // pairs i < j of subdomains whose Xi share rows, in order of first
  // occurrence (by row, then by position in the row's list), with the shared
  // rows of pair k at cpair_rows[2 cpair_ptr[k] ..] as (pos in Xi_i, pos in Xi_j)
  std::vector<int32_t> cpair_ij, cpair_rows;
  std::vector<int64_t> cpair_ptr;
  int64_t total_loc = 0, total_tiles = 0, total_fac = 0, total_dinv = 0, total_g = 0;
};

// CSR pattern transpose (counting sort, rows ascending inside each column);
// tperm[k] is the index in A of the k-th entry of A^T.
bool plan_transpose(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* colind,
                    std::vector<int32_t>& trowptr, std::vector<int32_t>& tcol,
                    std::vector<int32_t>& tperm);

// Index sets, local layouts and envelopes of every subdomain.  colind may
// still be arriving: wait_nnz(e), if given, returns once colind[0 .. e) is
// in place, and every read of colind comes after such a call.
bool plan_build(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* colind,
                const int32_t* part, int32_t nparts, const std::vector<int32_t>& seg_of_part,
                HostPlan& P, std::string& err,
                const std::function<void(int64_t)>& wait_nnz = std::function<void(int64_t)>());

// Overlap maps of a built plan: for every column the local positions holding
// it (own_ptr / own_pos), and the pairs of subdomains sharing rows (cpair_*,
// from shared_rows, which it empties).  Reads the rest of P only, so it may
// run while the device works on the built part.
bool plan_maps(int32_t n, HostPlan& P, std::string& err);

// Coarse numbering (per instance, subdomains in order, padded to 32), the
// pairs of subdomains whose rows overlap (blocks of E), the tile envelope of
// E and the row lists of its right-looking Cholesky.
struct CoarsePlan {
  std::vector<SegDesc> segs;
  int64_t n0 = 0, n0tot = 0, etiles = 0, efac_tiles = 0;
  int64_t xtot = 0, wtot = 0, einv_tot = 0;
  std::vector<PairDesc> pairs;
  std::vector<int32_t> pair_rows;     // (pos in Xi_i, pos in Xi_j) per shared row
  std::vector<int32_t> eF, seg_of_tile;
  std::vector<int64_t> eOff;
  std::vector<int64_t> pad_idx;       // efac offsets of the diagonal of padding rows
  std::vector<int32_t> erows;         // envelope rows of every tile column
  std::vector<int64_t> eptr;
  std::vector<int32_t> items;         // E assembly work items: (pair, row block, column block, 0)
};

// Fills p, x_off, w_off, c_off, cg_off of every subdomain of H and the plan of E.
void plan_coarse(HostPlan& H, int S, int32_t m, const std::vector<int32_t>& p, CoarsePlan& C);

// When consecutive rows of A start at unrelated columns (more than one drop
// of the first column by more than 256 columns per 16 rows, at least 65,536
// rows), the rows sorted stably by their first column (counting sort):
// perm[i] is the row of A placed at i, prp the row starts of the permuted copy.  The x gathers of A p
// and the (A p) gathers of A^T (A p) then stay local.
struct RowOrder {
  bool use = false;
  std::vector<int32_t> perm, prp;
};

void row_order(int32_t m, int32_t n, const int32_t* rp, const int32_t* ci, RowOrder& ro);

}  // namespace lsq2l
