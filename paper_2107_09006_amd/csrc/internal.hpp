// Internal declarations of the lsq2l library (HIP, gfx950).
//
// Data layout in HBM (all per handle):
//   * A in CSR (int32 row pointers and columns, double values) and its
//     transpose in CSR with the permutation into A's value array;
//   * per subdomain i a local, zero-padded index space of size np_i:
//       [0, nI)           interior columns Omega_Ii (ascending)
//       [nI, nIp)         padding (identity rows), nIp = roundup(nI, 32)
//       [nIp, nIp + nG)   interface columns Omega_Gamma_i (ascending)
//       [nIp + nG, np)    padding, np = nIp + roundup(nG, 32)
//   * local factors in a tile-envelope layout: the lower triangle is cut in
//     32 x 32 tiles; tile row I keeps the tiles J = F(I) .. I contiguously
//     (column-major inside a tile), where F(I) is the first tile column any
//     row of the tile couples to.  Cholesky creates no fill outside the row
//     envelope, so the factor overwrites the matrix in place;
//   * the inverse of every diagonal factor tile (used by the blocked
//     triangular solves);
//   * coarse basis X_i (nIp x p_i, column-major), W_i = A(Xi_i, Omega_Ii) X_i,
//     the coarse matrix E in the same tile-envelope layout, and dense
//     per-instance inverses of E.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/lsq2l.h"

namespace lsq2l {

constexpr int TS = 32;        // tile edge
constexpr int TT = TS * TS;   // elements per tile
constexpr int LDT = TS + 1;   // padded leading dimension of tiles staged in LDS

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct SubDesc {
  int32_t nI, nG, nIp, np;    // interior, interface, padded interior, padded total
  int32_t ntiles, ntI;        // tiles per side, interior tiles (nIp / 32)
  int32_t nXi, p;             // |Xi_i| and number of coarse vectors
  int32_t seg, nGp;           // instance index, padded interface size
  int32_t id, spare;          // subdomain index (kernels may run subdomains in another order)
  int64_t omega_off;          // int32 offset: Omega_i (nI interior then nG interface)
  int64_t xi_off;             // int32 offset: Xi_i
  int64_t loc_off;            // double offset: local vectors (np entries)
  int64_t tile_base;          // offset into tile envelope tables (ntiles entries)
  int64_t fac_off;            // element offset of the first factor tile
  int64_t dinv_off;           // element offset of the diagonal inverse tiles
  int64_t g_off;              // element offset of interface work matrices (nGp * nGp)
  int64_t x_off;              // element offset of X_i (nIp * p)
  int64_t c_off;              // first coarse index of this subdomain (within its instance)
  int64_t cg_off;             // first coarse index in the global coarse numbering
  int64_t w_off;              // element offset of W_i (nXi * p)
};

// Pair of subdomains that share rows of A (for the blocks of E).
struct PairDesc {
  int32_t i, j;               // i <= j
  int32_t nrows;              // shared rows
  int32_t pad;
  int64_t rows_off;           // offset into pair row lists (pos in Xi_i, pos in Xi_j)
};

struct SegDesc {              // one least-squares instance of a batch
  int64_t row0, m, col0, n;
  int64_t n0, c0;             // coarse size and first global coarse index
  int64_t einv_off;           // element offset of the dense inverse of E (n0 x n0)
  int64_t etile0, etiles;     // first tile row of E and number of tile rows
};

// -------------------------------------------------------------------------
// tile addressing
// -------------------------------------------------------------------------
__host__ __device__ inline int64_t tile_pos(const int32_t* F, const int64_t* off, int I, int J) {
  return off[I] + (J - F[I]);
}

// -------------------------------------------------------------------------
// MFMA helpers: one wave computes a 32 x 32 tile as 2 x 2 blocks of 16 x 16.
// Operand lane maps (gfx950 v_mfma_*_16x16x4): lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  The accumulator maps are given by acc_row/acc_col.
// -------------------------------------------------------------------------
template <typename T> struct Mfma;

template <> struct Mfma<double> {
  typedef double4_t acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // element v of lane l holds D[acc_row(l, v)][acc_col(l, v)]; the f64 form
  // interleaves rows (measured on gfx950), the f32 form keeps them in blocks of 4
  __device__ static inline int acc_row(int l, int v) { return l / 16 + 4 * v; }
  __device__ static inline int acc_col(int l, int v) { return l % 16; }
};

template <> struct Mfma<float> {
  typedef float4_t acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int acc_row(int l, int v) { return 4 * (l / 16) + v; }
  __device__ static inline int acc_col(int l, int v) { return l % 16; }
};

// acc[bi * 2 + bj] covers rows 16 bi .. 16 bi + 15, columns 16 bj .. 16 bj + 15.
template <typename T>
__device__ inline void tile_acc_load(typename Mfma<T>::acc_t acc[4], const T* C, int ldc, int lane) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = 16 * bi + Mfma<T>::acc_row(lane, v), c = 16 * bj + Mfma<T>::acc_col(lane, v);
        acc[bi * 2 + bj][v] = C[(int64_t)c * ldc + r];
      }
}

template <typename T>
__device__ inline void tile_acc_store(const typename Mfma<T>::acc_t acc[4], T* C, int ldc, int lane) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = 16 * bi + Mfma<T>::acc_row(lane, v), c = 16 * bj + Mfma<T>::acc_col(lane, v);
        C[(int64_t)c * ldc + r] = acc[bi * 2 + bj][v];
      }
}

template <typename T>
__device__ inline void tile_acc_zero(typename Mfma<T>::acc_t acc[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = Mfma<T>::zero();
}

// acc += sign * A * B^T with A, B 32 x 32 column-major (leading dims lda, ldb).
template <typename T, bool NEG>
__device__ inline void tile_mma_nt(typename Mfma<T>::acc_t acc[4], const T* A, int lda,
                                   const T* B, int ldb, int lane) {
  const int li = lane % 16, lk = lane / 16;
  // all operand fragments load first (32 independent loads per lane), then
  // the MFMAs run
  T a0[8], a1[8], b0[8], b1[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kk = 4 * q;
    a0[q] = A[(int64_t)(kk + lk) * lda + li];
    a1[q] = A[(int64_t)(kk + lk) * lda + 16 + li];
    b0[q] = B[(int64_t)(kk + lk) * ldb + li];
    b1[q] = B[(int64_t)(kk + lk) * ldb + 16 + li];
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const T x0 = NEG ? -a0[q] : a0[q], x1 = NEG ? -a1[q] : a1[q];
    acc[0] = Mfma<T>::mma(x0, b0[q], acc[0]);
    acc[1] = Mfma<T>::mma(x0, b1[q], acc[1]);
    acc[2] = Mfma<T>::mma(x1, b0[q], acc[2]);
    acc[3] = Mfma<T>::mma(x1, b1[q], acc[3]);
  }
}

// Orders the LDS accesses of the lanes of one wave: a wave's LDS operations
// complete in issue order, so wavefront-scope fences around a code-motion
// barrier suffice.
// x + x of lane (l xor 32), the same value in both halves of the wave, by
// two v_permlane32_swap (gfx950): with both operands x, the first result of
// every lane is x of lane l % 32 and the second x of lane l % 32 + 32.  All
// lanes of the wave must be active.
__device__ inline double half_pair_sum(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const auto rlo = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rhi = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(rhi[0], rlo[0]) + __hiloint2double(rhi[1], rlo[1]);
}

// The same for a float (one swap).
__device__ inline float half_pair_sum(float x) {
  const int v = __float_as_int(x);
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// x + x of the lane whose index differs by the DPP pattern CTRL
template <int CTRL>
__device__ inline double dpp_pair_sum(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return x + __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, the same value in every lane: lane pairs within
// quads (DPP quad permutations 1032 and 2301), the two quads of each group of
// eight (row half mirror), the two halves of each row of 16 (row mirror),
// rows 0, 1 and 2, 3 (one cross-lane read), then the halves of the wave.
// Each step adds two values that the partner lane adds in the other order,
// so every lane ends with the same bits.
__device__ inline double wave_allsum(double x) {
  x = dpp_pair_sum<0xB1>(x);
  x = dpp_pair_sum<0x4E>(x);
  x = dpp_pair_sum<0x141>(x);
  x = dpp_pair_sum<0x140>(x);
  x += __shfl_xor(x, 16, 64);
  return half_pair_sum(x);
}

// Orders this wave's global stores before its later loads by other lanes
// (workgroup-scope release and acquire).
__device__ inline void wg_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// -------------------------------------------------------------------------
// Cholesky factor and inverse of one 32 x 32 diagonal tile
// -------------------------------------------------------------------------
// Broadcast of lane l's value (l wave-uniform) through a scalar register.
__device__ inline double lane_bcast(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ inline float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 1 / sqrt(d) from the hardware estimate, refined by Newton-Raphson steps
// r <- r + r (1 - d r^2) / 2 (the error roughly squares each step): two in
// double, one in float
__device__ inline double rsqrt_refined(double d) {
  double rs = __builtin_amdgcn_rsq(d);
  rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
  return fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
}

__device__ inline float rsqrt_refined(float d) {
  const float rs = __builtin_amdgcn_rsqf(d);
  return fmaf(0.5f * rs, fmaf(-d * rs, rs, 1.0f), rs);
}

// L L^T = W and Inv = L^{-1} for one SPD tile W (column-major in LDS, leading
// dimension LDT, lower part read), by the 64 lanes of one wave with the tile in
// registers: lane j < 32 holds column j of the symmetric tile, lane 32 + j
// column j of the running inverse Z.  Step k eliminates column k (trailing
// update of columns j > k) and applies the same elementary operation to Z
// (rows i > k: Z(i, :) -= W(i, k) / d_k Z(k, :), then row k scaled by
// 1 / sqrt(d_k)).  Column k is broadcast by lane reads, so the 32 steps need no
// LDS traffic and no barrier.  L and Inv are written to LDS (L may be null).
// Returns false if a pivot is not positive and finite (it is then replaced by
// 1, so the caller can continue and report).  T is double or float (the
// arithmetic of the whole tile).
template <typename T>
__device__ inline bool tile_potrf_inv_reg(const T* W, T* L, T* Inv, int lane) {
  const int j = lane % TS;
  const bool fac = lane < TS;
  T v[TS];
#pragma unroll
  for (int i = 0; i < TS; ++i)
    v[i] = fac ? ((i >= j) ? W[j * LDT + i] : W[i * LDT + j]) : ((i == j) ? T(1) : T(0));
  bool ok = true;
  T colscale = T(1);
  // Every lane runs the same instructions: the lane reads happen in uniform
  // control flow and the per-lane roles are selects, never branches (a lane
  // read inside a divergent branch may see another version of the value).
#pragma unroll
  for (int k = 0; k < TS; ++k) {
    T d = lane_bcast(v[k], k);
    if (!(d > T(0)) || !(d < T(INFINITY))) { ok = false; d = T(1); }
    const T rs = rsqrt_refined(d);
    const T invd = rs * rs, inv_sd = rs;
    // factor lanes j > k: W(i, j) -= W(i, k) W(k, j) / d; inverse lanes j <= k:
    // Z(i, j) -= W(i, k) Z(k, j) / d; other lanes unchanged
    const bool upd = fac ? (j > k) : (j <= k);
    const T coef = upd ? v[k] * invd : T(0);
#pragma unroll
    for (int i = k + 1; i < TS; ++i) v[i] -= lane_bcast(v[i], k) * coef;
    if (!fac && j <= k) v[k] *= inv_sd;
    if (fac && j == k) colscale = inv_sd;
  }
#pragma unroll
  for (int i = 0; i < TS; ++i) {
    if (fac) { if (L) L[j * LDT + i] = (i >= j) ? v[i] * colscale : T(0); }
    else Inv[j * LDT + i] = v[i];
  }
  return ok;
}

// -------------------------------------------------------------------------
// subdomain addressing shared by the setup kernels
// -------------------------------------------------------------------------
// Local position of global column c in subdomain i (or -1): interior columns
// are found through the owner table, interface columns by binary search in
// the sorted Omega_Gamma_i.
__device__ inline int local_pos(int i, int c, const int32_t* __restrict__ part,
                                const int32_t* __restrict__ locown, const int32_t* __restrict__ G,
                                int nG, int nIp) {
  if (part[c] == i) return locown[c];
  int lo = 0, hi = nG;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (G[mid] < c) lo = mid + 1; else hi = mid;
  }
  return (lo < nG && G[lo] == c) ? nIp + lo : -1;
}

// Rows I > J of the tile envelope whose envelope reaches column J, in
// ascending order (ballot compaction by wave 0).  Returns the count.
__device__ inline int envelope_rows(const int32_t* F, int J, int ntiles, int32_t* list, int cap,
                                    int* s_count) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int cnt = 0;
    for (int base = J + 1; base < ntiles; base += 64) {
      const int I = base + lane;
      const bool fl = I < ntiles && F[I] <= J;
      const unsigned long long mask = __ballot(fl);
      const int before = __popcll(mask & ((1ull << lane) - 1ull));
      if (fl && cnt + before < cap) list[cnt + before] = I;
      cnt += __popcll(mask);
    }
    if (lane == 0) *s_count = cnt;
  }
  __syncthreads();
  return *s_count;
}

// -------------------------------------------------------------------------
// host-side helpers shared by the translation units
// -------------------------------------------------------------------------
void set_error(const std::string& msg);

#define LSQ2L_HIP_TRY(expr)                                                              \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      ::lsq2l::set_error(std::string("HIP error ") + hipGetErrorString(_e) + " at " +   \
                         __FILE__ + ":" + std::to_string(__LINE__) + " in " #expr);      \
      return LSQ2L_EHIP;                                                                 \
    }                                                                                    \
  } while (0)

}  // namespace lsq2l
