// CSR transpose of A's pattern on the device (the Aᵀ used by the assembly,
// the adjoint and Aᵀy, and read back by the host planner).  The entries are
// sorted by column with a stable radix sort keyed on the column index, so
// inside every column the rows stay in ascending order; tperm[k] is the
// index in A of the k-th entry of Aᵀ.
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"

namespace lsq2l {

__global__ void k_iota(int64_t n, int32_t* __restrict__ v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) v[k] = (int32_t)k;
}

__global__ void k_row_ids(int32_t m, const int32_t* __restrict__ rowptr, int32_t* __restrict__ rowid) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) rowid[e] = r;
}

// trowptr[c] = first position of column c among the sorted keys
__global__ void k_col_ptr(int64_t nnz, int32_t n, const int32_t* __restrict__ keys,
                          int32_t* __restrict__ trowptr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int32_t cur = keys[k], prev = (k == 0) ? -1 : keys[k - 1];
  for (int32_t c = prev + 1; c <= cur; ++c) trowptr[c] = (int32_t)k;
  if (k == nnz - 1)
    for (int32_t c = cur + 1; c <= n; ++c) trowptr[c] = (int32_t)nnz;
}

__global__ void k_gather_i32(int64_t n, const int32_t* __restrict__ idx, const int32_t* __restrict__ src,
                             int32_t* __restrict__ dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[idx[k]];
}

// Row i of the row-permuted copy is row perm[i] of A (one thread per row;
// prowptr holds the permuted row starts).
__global__ void k_permute_rows(int32_t m, const int32_t* __restrict__ perm,
                               const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                               const double* __restrict__ vals, const int32_t* __restrict__ prowptr,
                               int32_t* __restrict__ pcolind, double* __restrict__ pvals) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t r = perm[i];
  int32_t d = prowptr[i];
  for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k, ++d) {
    pcolind[d] = colind[k];
    pvals[d] = vals[k];
  }
}

void launch_permute_rows(hipStream_t st, int32_t m, const int32_t* perm, const int32_t* rowptr,
                         const int32_t* colind, const double* vals, const int32_t* prowptr,
                         int32_t* pcolind, double* pvals) {
  if (m == 0) return;
  k_permute_rows<<<(m + 255) / 256, 256, 0, st>>>(m, perm, rowptr, colind, vals, prowptr, pcolind, pvals);
}

static int key_bits(int32_t n) {
  int b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

size_t transpose_temp_bytes(int64_t nnz, int32_t n) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const int32_t*)nullptr, (int32_t*)nullptr,
                                          (const int32_t*)nullptr, (int32_t*)nullptr, (int)nnz, 0,
                                          key_bits(n));
  return bytes;
}

hipError_t launch_transpose(hipStream_t st, int32_t m, int32_t n, int64_t nnz, const int32_t* rowptr,
                            const int32_t* colind, int32_t* trowptr, int32_t* trow, int32_t* tperm,
                            int32_t* work_keys, int32_t* work_vals, int32_t* work_rows, void* temp,
                            size_t temp_bytes) {
  if (nnz == 0) return hipMemsetAsync(trowptr, 0, (size_t)(n + 1) * sizeof(int32_t), st);
  const unsigned gb = (unsigned)((nnz + 255) / 256);
  k_iota<<<gb, 256, 0, st>>>(nnz, work_vals);
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, colind, work_keys, work_vals,
                                                    tperm, (int)nnz, 0, key_bits(n), st);
  if (e != hipSuccess) return e;
  k_col_ptr<<<gb, 256, 0, st>>>(nnz, n, work_keys, trowptr);
  k_row_ids<<<(m + 255) / 256, 256, 0, st>>>(m, rowptr, work_rows);
  k_gather_i32<<<gb, 256, 0, st>>>(nnz, tperm, work_rows, trow);
  return hipGetLastError();
}

}  // namespace lsq2l
