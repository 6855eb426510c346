// Sparse products and the vector work of preconditioned CG on C = A^T A
// (eq. normal): C p is applied as A^T (A p), never formed.
//
// Reductions are deterministic: every segment (instance) of a vector is cut
// into RED_BLOCKS fixed chunks, each reduced by a fixed tree; the partial
// sums are added in index order by the scalar kernel.  Repeated runs give
// bitwise-identical results.
#include "kernels.hpp"

namespace lsq2l {

// y = A x, G lanes per row (G in {1, 2, 4, 8, 16, 32, 64}); rows are short
// (1 - 64 stored entries), so a sub-wave per row keeps lanes busy and the
// column/value reads coalesced inside the group.
template <int G>
__global__ void __launch_bounds__(256)
k_spmv(int32_t nrows, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
       const double* __restrict__ vals, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = t / G;
  const int sub = (int)(t % G);
  double s = 0.0;
  if (row < nrows) {
    const int e1 = rowptr[row + 1];
    for (int e = rowptr[row] + sub; e < e1; e += G) s += vals[e] * x[colind[e]];
  }
#pragma unroll
  for (int w = G / 2; w > 0; w /= 2) s += __shfl_down(s, w, G);
  if (row < nrows && sub == 0) y[row] = s;
}

void launch_spmv(hipStream_t st, int32_t nrows, const int32_t* rowptr, const int32_t* colind,
                 const double* vals, const double* x, double* y, int group) {
  if (nrows == 0) return;
  const int64_t threads = (int64_t)nrows * group;
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  switch (group) {
    case 1: k_spmv<1><<<blocks, 256, 0, st>>>(nrows, rowptr, colind, vals, x, y); break;
    case 2: k_spmv<2><<<blocks, 256, 0, st>>>(nrows, rowptr, colind, vals, x, y); break;
    case 4: k_spmv<4><<<blocks, 256, 0, st>>>(nrows, rowptr, colind, vals, x, y); break;
    case 8: k_spmv<8><<<blocks, 256, 0, st>>>(nrows, rowptr, colind, vals, x, y); break;
    case 16: k_spmv<16><<<blocks, 256, 0, st>>>(nrows, rowptr, colind, vals, x, y); break;
    case 32: k_spmv<32><<<blocks, 256, 0, st>>>(nrows, rowptr, colind, vals, x, y); break;
    default: k_spmv<64><<<blocks, 256, 0, st>>>(nrows, rowptr, colind, vals, x, y); break;
  }
}

// dL/dA_ij = r_i lam_j - (A lam)_i x_j on the stored pattern, CSR order.
__global__ void k_grad_vals(int32_t m, const int32_t* __restrict__ rowptr,
                            const int32_t* __restrict__ colind, const double* __restrict__ r,
                            const double* __restrict__ lam, const double* __restrict__ Alam,
                            const double* __restrict__ x, double* __restrict__ out) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= m) return;
  const double ri = r[row], ai = Alam[row];
  for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) {
    const int j = colind[e];
    out[e] = ri * lam[j] - ai * x[j];
  }
}

void launch_grad_vals(hipStream_t st, int32_t m, const int32_t* rowptr, const int32_t* colind,
                      const double* r, const double* lam, const double* Alam, const double* x,
                      double* out) {
  if (m == 0) return;
  k_grad_vals<<<(m + 255) / 256, 256, 0, st>>>(m, rowptr, colind, r, lam, Alam, x, out);
}

// Sum over a block of 256 threads: a sum in every wave, then the four wave
// sums in order (the result is returned to every thread)
__device__ inline double block_reduce_256(double v, double* sh) {
  v = wave_allsum(v);
  const int wave = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) sh[wave] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// partial[s * RED_BLOCKS + b] = sum over chunk b of segment s of a .* b
__global__ void __launch_bounds__(256)
k_dot(const int64_t* __restrict__ seg_ptr, const double* __restrict__ a,
      const double* __restrict__ b, double* __restrict__ partial) {
  __shared__ double sh[256];
  const int s = blockIdx.y, blk = blockIdx.x;
  const int64_t lo = seg_ptr[s], hi = seg_ptr[s + 1];
  const int64_t len = hi - lo;
  const int64_t chunk = (len + RED_BLOCKS - 1) / RED_BLOCKS;
  const int64_t c0 = lo + blk * chunk, c1 = min(hi, c0 + chunk);
  double v = 0.0;
  for (int64_t k = c0 + threadIdx.x; k < c1; k += blockDim.x) v += a[k] * b[k];
  v = block_reduce_256(v, sh);
  if (threadIdx.x == 0) partial[(int64_t)s * RED_BLOCKS + blk] = v;
}

void launch_dot(hipStream_t st, int S, const int64_t* seg_ptr, const double* a, const double* b,
                double* partial) {
  k_dot<<<dim3(RED_BLOCKS, S), 256, 0, st>>>(seg_ptr, a, b, partial);
}

__global__ void k_scalar(int op, int S, const double* __restrict__ partial,
                         const double* __restrict__ partial2, Scalars sc, double tol2,
                         int flexible) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double v = 0.0, v2 = 0.0;
  for (int b = 0; b < RED_BLOCKS; ++b) v += partial[(int64_t)s * RED_BLOCKS + b];
  if (partial2)
    for (int b = 0; b < RED_BLOCKS; ++b) v2 += partial2[(int64_t)s * RED_BLOCKS + b];
  switch (op) {
    case OP_R0:
      sc.r0n2[s] = v;
      sc.rn2[s] = v;
      sc.done[s] = (v == 0.0) ? 1 : 0;
      break;
    case OP_RHO_INIT:
      sc.rho[s] = v;
      if (sc.done[s] == 0 && !isfinite(v)) sc.done[s] = 2;
      break;
    case OP_ALPHA:
      sc.pq[s] = v;
      if (sc.done[s] != 0) {
        sc.alpha[s] = 0.0;
      } else if (!(v > 0.0) || !isfinite(v) || !isfinite(sc.rho[s])) {
        sc.alpha[s] = 0.0;
        sc.done[s] = 2;
      } else {
        sc.alpha[s] = sc.rho[s] / v;
      }
      break;
    case OP_RNORM:
      sc.rn2[s] = v;
      if (sc.done[s] == 0) {
        if (!isfinite(v)) sc.done[s] = 2;
        else if (v <= tol2 * sc.r0n2[s]) sc.done[s] = 1;
      }
      break;
    case OP_BETA: {
      // partial: z^T r_new; partial2 (flexible only): z^T r_old
      const double num = flexible ? (v - v2) : v;
      if (sc.done[s] != 0) sc.beta[s] = 0.0;
      else sc.beta[s] = num / sc.rho[s];
      sc.rho[s] = v;
      break;
    }
  }
}

void launch_scalar(hipStream_t st, int op, int S, const double* partial, const double* partial2,
                   Scalars sc, double tol2, int flexible) {
  k_scalar<<<(S + 63) / 64, 64, 0, st>>>(op, S, partial, partial2, sc, tol2, flexible);
}

__device__ inline int seg_of(int64_t k, int S, const int64_t* seg_ptr) {
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (seg_ptr[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_axpy_xr(int64_t n, int S, const int64_t* __restrict__ seg_ptr,
                          const double* __restrict__ alpha, const double* __restrict__ p,
                          const double* __restrict__ q, double* __restrict__ x,
                          double* __restrict__ r) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double a = alpha[S == 1 ? 0 : seg_of(k, S, seg_ptr)];
  x[k] += a * p[k];
  r[k] -= a * q[k];
}

void launch_axpy_xr(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr, const double* alpha,
                    const double* p, const double* q, double* x, double* r) {
  if (n == 0) return;
  k_axpy_xr<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, S, seg_ptr, alpha, p, q, x, r);
}

__global__ void k_xpby(int64_t n, int S, const int64_t* __restrict__ seg_ptr,
                       const double* __restrict__ beta, const double* __restrict__ z,
                       double* __restrict__ p) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double b = beta[S == 1 ? 0 : seg_of(k, S, seg_ptr)];
  p[k] = z[k] + b * p[k];
}

void launch_xpby(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr, const double* beta,
                 const double* z, double* p) {
  if (n == 0) return;
  k_xpby<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, S, seg_ptr, beta, z, p);
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = a[k] - b[k];
}

void launch_sub(hipStream_t st, int64_t n, const double* a, const double* b, double* out) {
  if (n == 0) return;
  k_sub<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, b, out);
}

__global__ void k_add(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

void launch_add(hipStream_t st, int64_t n, const double* a, const double* b, double* out) {
  if (n == 0) return;
  k_add<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, b, out);
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = v;
}

__global__ void k_copy(int64_t n, const double* __restrict__ a, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i];
}

void launch_copy(hipStream_t st, int64_t n, const double* a, double* out) {
  if (n == 0) return;
  k_copy<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, a, out);
}

void launch_fill(hipStream_t st, int64_t n, double v, double* out) {
  if (n == 0) return;
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, v, out);
}

}  // namespace lsq2l
