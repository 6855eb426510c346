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

// y = A x for short, uneven rows, staged through LDS.  Workgroup b owns the
// rows whose first entry lies in [b SPMV_NB, (b + 1) SPMV_NB): rows
// tab[2b] .. tab[2b + 2] - 1, whose entries start at tab[2b + 1] (a table
// made once per matrix, k_row_blocks), so that one 8-byte load gives the
// block's extent.  Its entries are read once, coalesced, four per thread in
// flight, as vals[e] x[colind[e]] into LDS; then every thread sums its rows
// from LDS in entry order and writes y coalesced.  A block whose rows hold
// more than SPMV_CAP entries (a long last row) sums each row with a
// wavefront instead.  Every row is summed in one fixed order, so runs are
// bitwise reproducible.  With STREAM the matrix arrays are read with
// non-temporal loads, which keeps the caches for x when the matrix is
// larger than the last-level cache.
constexpr int SPMV_NB = 1024, SPMV_CAP = 2048, SPMV_THREADS = 256, SPMV_U = 4;
constexpr int64_t SPMV_STREAM_BYTES = (int64_t)256 << 20;   // MI355X last-level cache

int64_t spmv_blocks(int64_t nnz) { return std::max<int64_t>(1, (nnz + SPMV_NB - 1) / SPMV_NB); }
int64_t spmv_table_len(int64_t nnz) { return 2 * (spmv_blocks(nnz) + 1); }

// tab[2b] = first row whose start is >= b SPMV_NB (b < nblk), tab[2b + 1] =
// its start; tab[2 nblk] = nrows, tab[2 nblk + 1] = nnz
__global__ void k_row_blocks(int32_t nrows, const int32_t* __restrict__ rowptr, int64_t nblk,
                             int32_t* __restrict__ tab) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblk) return;
  int32_t lo = nrows;
  if (b < nblk) {
    const int64_t v = b * SPMV_NB;
    lo = 0;
    int32_t hi = nrows;
    while (lo < hi) {
      const int32_t mid = (int32_t)(((int64_t)lo + hi) >> 1);
      if (rowptr[mid] < v) lo = mid + 1;
      else hi = mid;
    }
  }
  tab[2 * b] = lo;
  tab[2 * b + 1] = rowptr[lo];
}

void launch_row_blocks(hipStream_t st, int32_t nrows, const int32_t* rowptr, int64_t nnz, int32_t* tab) {
  const int64_t nblk = spmv_blocks(nnz);
  k_row_blocks<<<(unsigned)((nblk + 1 + 255) / 256), 256, 0, st>>>(nrows, rowptr, nblk, tab);
}

template <bool STREAM, typename V>
__device__ inline V spmv_load(const V* p) {
  if constexpr (STREAM) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool STREAM>
__global__ void __launch_bounds__(SPMV_THREADS)
k_spmv_stream(const int32_t* __restrict__ tab, const int32_t* __restrict__ rowptr,
              const int32_t* __restrict__ colind, const double* __restrict__ vals,
              const double* __restrict__ x, double* __restrict__ y) {
  __shared__ double prod[SPMV_CAP];
  const int tid = threadIdx.x;
  typedef int32_t i2 __attribute__((ext_vector_type(2)));
  const i2 lo = reinterpret_cast<const i2*>(tab)[blockIdx.x];
  const i2 hi = reinterpret_cast<const i2*>(tab)[blockIdx.x + 1];
  const int32_t r0 = lo.x, e0 = lo.y, r1 = hi.x, e1 = hi.y;
  if (r0 >= r1) return;
  if (e1 - e0 <= SPMV_CAP) {
    for (int32_t e = e0 + tid; e < e1; e += SPMV_U * SPMV_THREADS) {
      int32_t c[SPMV_U];
      double v[SPMV_U];
#pragma unroll
      for (int u = 0; u < SPMV_U; ++u) {
        const int32_t q = e + u * SPMV_THREADS;
        c[u] = q < e1 ? spmv_load<STREAM>(colind + q) : 0;
        v[u] = q < e1 ? spmv_load<STREAM>(vals + q) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < SPMV_U; ++u) {
        const int32_t q = e + u * SPMV_THREADS;
        if (q < e1) prod[q - e0] = v[u] * x[c[u]];
      }
    }
    __syncthreads();
    for (int32_t r = r0 + tid; r < r1; r += SPMV_THREADS) {
      const int32_t a = rowptr[r] - e0, b = rowptr[r + 1] - e0;
      double s = 0.0;
      for (int32_t k = a; k < b; ++k) s += prod[k];
      y[r] = s;
    }
    return;
  }
  // long rows: one wavefront per row, lanes strided over the row
  const int lane = tid & 63, wave = tid >> 6;
  for (int32_t r = r0 + wave; r < r1; r += SPMV_THREADS / 64) {
    double s = 0.0;
    for (int32_t e = rowptr[r] + lane; e < rowptr[r + 1]; e += 64) s += vals[e] * x[colind[e]];
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) s += __shfl_down(s, w, 64);
    if (lane == 0) y[r] = s;
  }
}

// group 0: row blocks, streaming loads if the matrix arrays (12 bytes per
// entry) exceed the last-level cache; -1 / -2: row blocks with cached /
// streaming loads; 1 .. 64: that many lanes per row
void launch_spmv(hipStream_t st, int32_t nrows, const int32_t* rowptr, const int32_t* colind,
                 const double* vals, const double* x, double* y, int group, int64_t nnz,
                 const int32_t* blk) {
  if (nrows == 0) return;
  if (group == 0) group = 12 * nnz > SPMV_STREAM_BYTES ? SPMV_ROWS_STREAM : SPMV_ROWS_CACHED;
  if (group < 0 && blk) {
    if (group == SPMV_ROWS_STREAM)
      k_spmv_stream<true><<<(unsigned)spmv_blocks(nnz), SPMV_THREADS, 0, st>>>(blk, rowptr, colind, vals, x, y);
    else
      k_spmv_stream<false><<<(unsigned)spmv_blocks(nnz), SPMV_THREADS, 0, st>>>(blk, rowptr, colind, vals, x, y);
    return;
  }
  if (group < 0) group = 1;
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
        sc.its[s] += 1;
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

__global__ void k_fill_i32(int64_t n, int32_t v, int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = v;
}

void launch_fill_i32(hipStream_t st, int64_t n, int32_t v, int32_t* out) {
  if (n == 0) return;
  k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, v, out);
}

__global__ void k_hash_fill(int64_t n, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint64_t h = (uint64_t)k * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  h ^= h >> 31;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 29;
  out[k] = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

void launch_hash_fill(hipStream_t st, int64_t n, double* out) {
  if (n == 0) return;
  k_hash_fill<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, out);
}

__global__ void k_scale_seg(int64_t n, int S, const int64_t* __restrict__ seg_ptr,
                            const double* __restrict__ f, const double* __restrict__ a,
                            double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  out[k] = a[k] * f[S == 1 ? 0 : seg_of(k, S, seg_ptr)];
}

void launch_scale_seg(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr, const double* f,
                      const double* a, double* out) {
  if (n == 0) return;
  k_scale_seg<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, S, seg_ptr, f, a, out);
}

// ---------------------------------------------------------------------------
// LSQR (Section 4.1, "Solution phase"): Golub-Kahan bidiagonalization of
// A W^{-1}, M = W^{-1} W^{-T}, carried in x-space.  With v the unit vector of
// the bidiagonalization, the iteration keeps vt = W^{-1} v and zh = W^T v:
//   u <- (A vt - alpha u) / beta,
//   q  = A^T u - beta zh,  s = M q,  alpha = sqrt(q^T s),
//   zh <- q / alpha,  vt <- s / alpha,
// so alpha = ||W^{-T} A^T u - beta v|| needs products with M only.  The
// plane rotations, the step x += (phi / rho) wt, wt <- vt - (theta / rho) wt
// and the estimates ||A W^{-1}||_F^2 = sum (alpha^2 + beta^2),
// ||(A W^{-1})^T r|| = alpha |c phibar|-style follow Paige and Saunders.
// done: 0 active, 1 converged, 2 breakdown, 3 converged by this step (its
// update still applies).
// ---------------------------------------------------------------------------
__global__ void k_lsqr_scalar(int op, int S, const double* __restrict__ partial,
                              double* __restrict__ scb, int32_t* __restrict__ done,
                              int32_t* __restrict__ its, double tol) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double v = 0.0;
  for (int b = 0; b < RED_BLOCKS; ++b) v += partial[(int64_t)s * RED_BLOCKS + b];
  double* sc = scb + (int64_t)s * LSQR_NSC;
  switch (op) {
    case LSQR_INIT_BETA: {
      const double beta = sqrt(v);
      sc[LS_BETA] = beta;
      sc[LS_PHIBAR] = beta;
      sc[LS_ANORM2] = 0.0;
      sc[LS_RNORM0] = beta;
      sc[LS_TEST] = 1.0;
      its[s] = 0;
      done[s] = !isfinite(v) ? 2 : (beta == 0.0 ? 1 : 0);
      break;
    }
    case LSQR_INIT_ALPHA: {
      if (done[s] != 0) { sc[LS_ALPHA] = 0.0; break; }
      if (!isfinite(v) || v < 0.0) { done[s] = 2; sc[LS_ALPHA] = 0.0; break; }
      const double alpha = sqrt(v);
      sc[LS_ALPHA] = alpha;
      sc[LS_RHOBAR] = alpha;
      if (alpha == 0.0) { done[s] = 1; sc[LS_TEST] = 0.0; }
      break;
    }
    case LSQR_BETA: {
      if (done[s] == 3) done[s] = 1;
      if (done[s] != 0) break;
      if (!isfinite(v)) { done[s] = 2; break; }
      const double beta = sqrt(v);
      const double a = sc[LS_ALPHA];
      sc[LS_ANORM2] += a * a + beta * beta;
      sc[LS_BETA] = beta;
      break;
    }
    case LSQR_ALPHA: {
      if (done[s] != 0) break;
      if (!isfinite(v) || v < 0.0) { done[s] = 2; break; }
      const double alpha = sqrt(v);
      const double rhobar = sc[LS_RHOBAR], beta = sc[LS_BETA], phibar = sc[LS_PHIBAR];
      const double rho = hypot(rhobar, beta);
      const double c = rhobar / rho, sn = beta / rho;
      const double theta = sn * alpha;
      const double phi = c * phibar;
      const double phibar_new = sn * phibar;
      const double tau = sn * phi;
      sc[LS_RHOBAR] = -c * alpha;
      sc[LS_PHIBAR] = phibar_new;
      sc[LS_T1] = phi / rho;
      sc[LS_T2] = -theta / rho;
      sc[LS_ALPHA] = alpha;
      const double anorm = sqrt(sc[LS_ANORM2]);
      const double test = (phibar_new == 0.0) ? 0.0 : alpha * fabs(tau) / (anorm * phibar_new);
      sc[LS_TEST] = test;
      its[s] += 1;
      if (!isfinite(test) || !isfinite(sc[LS_T1])) done[s] = 2;
      else if (test <= tol || alpha == 0.0) done[s] = 3;
      break;
    }
  }
}

void launch_lsqr_scalar(hipStream_t st, int op, int S, const double* partial, double* sc,
                        int32_t* done, int32_t* its, double tol) {
  k_lsqr_scalar<<<(S + 63) / 64, 64, 0, st>>>(op, S, partial, sc, done, its, tol);
}

__global__ void k_lsqr_u(int64_t m, int S, const int64_t* __restrict__ seg_ptr,
                         const double* __restrict__ sc, const int32_t* __restrict__ done,
                         const double* __restrict__ a, double* __restrict__ u, int first) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int s = S == 1 ? 0 : seg_of(k, S, seg_ptr);
  if (done[s] != 0) return;
  u[k] = first ? a[k] : a[k] - sc[(int64_t)s * LSQR_NSC + LS_ALPHA] * u[k];
}

void launch_lsqr_u(hipStream_t st, int64_t m, int S, const int64_t* seg_row, const double* sc,
                   const int32_t* done, const double* a, double* u, int first) {
  if (m == 0) return;
  k_lsqr_u<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(m, S, seg_row, sc, done, a, u, first);
}

__global__ void k_lsqr_unorm(int64_t m, int S, const int64_t* __restrict__ seg_ptr,
                             const double* __restrict__ sc, const int32_t* __restrict__ done,
                             double* __restrict__ u) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int s = S == 1 ? 0 : seg_of(k, S, seg_ptr);
  if (done[s] != 0) return;
  const double beta = sc[(int64_t)s * LSQR_NSC + LS_BETA];
  u[k] = beta > 0.0 ? u[k] / beta : 0.0;
}

void launch_lsqr_unorm(hipStream_t st, int64_t m, int S, const int64_t* seg_row, const double* sc,
                       const int32_t* done, double* u) {
  if (m == 0) return;
  k_lsqr_unorm<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(m, S, seg_row, sc, done, u);
}

__global__ void k_lsqr_q(int64_t n, int S, const int64_t* __restrict__ seg_ptr,
                         const double* __restrict__ sc, const int32_t* __restrict__ done,
                         const double* __restrict__ zh, double* __restrict__ q, int first) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int s = S == 1 ? 0 : seg_of(k, S, seg_ptr);
  if (done[s] != 0) { q[k] = 0.0; return; }
  if (!first) q[k] -= sc[(int64_t)s * LSQR_NSC + LS_BETA] * zh[k];
}

void launch_lsqr_q(hipStream_t st, int64_t n, int S, const int64_t* seg_col, const double* sc,
                   const int32_t* done, const double* zh, double* q, int first) {
  if (n == 0) return;
  k_lsqr_q<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, S, seg_col, sc, done, zh, q, first);
}

__global__ void k_lsqr_update(int64_t n, int S, const int64_t* __restrict__ seg_ptr,
                              const double* __restrict__ scb, const int32_t* __restrict__ done,
                              const double* __restrict__ q, const double* __restrict__ sv,
                              double* __restrict__ zh, double* __restrict__ v,
                              double* __restrict__ w, double* __restrict__ x, int first) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int s = S == 1 ? 0 : seg_of(k, S, seg_ptr);
  const int dn = done[s];
  if (!(dn == 0 || dn == 3)) return;
  const double* sc = scb + (int64_t)s * LSQR_NSC;
  const double alpha = sc[LS_ALPHA];
  const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
  const double vn = sv[k] * ia;
  zh[k] = q[k] * ia;
  v[k] = vn;
  if (first) {
    w[k] = vn;
  } else {
    const double wo = w[k];
    x[k] += sc[LS_T1] * wo;
    w[k] = vn + sc[LS_T2] * wo;
  }
}

void launch_lsqr_update(hipStream_t st, int64_t n, int S, const int64_t* seg_col, const double* sc,
                        const int32_t* done, const double* q, const double* s, double* zh,
                        double* v, double* w, double* x, int first) {
  if (n == 0) return;
  k_lsqr_update<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, S, seg_col, sc, done, q, s, zh, v,
                                                             w, x, first);
}

// ---------------------------------------------------------------------------
// GMRES building blocks: Gram-Schmidt against the stored basis V, with
// per-instance coefficients and fixed-order reductions
// ---------------------------------------------------------------------------
__device__ inline double block_sum_256_sync(double v, double* sh) {
  v = wave_allsum(v);
  const int wave = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) sh[wave] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256)
k_multidot(const int64_t* __restrict__ seg_ptr, int64_t n, int kv, const double* __restrict__ V,
           const double* __restrict__ w, double* __restrict__ partial, int ld) {
  __shared__ double sh[4];
  const int s = blockIdx.y, blk = blockIdx.x;
  const int64_t lo = seg_ptr[s], hi = seg_ptr[s + 1];
  const int64_t chunk = (hi - lo + RED_BLOCKS - 1) / RED_BLOCKS;
  const int64_t c0 = lo + blk * chunk, c1 = min(hi, c0 + chunk);
  for (int i = 0; i < kv; ++i) {
    const double* vi = V + (int64_t)i * n;
    double acc = 0.0;
    for (int64_t k = c0 + threadIdx.x; k < c1; k += blockDim.x) acc += vi[k] * w[k];
    acc = block_sum_256_sync(acc, sh);
    if (threadIdx.x == 0) partial[((int64_t)s * RED_BLOCKS + blk) * ld + i] = acc;
  }
}

void launch_multidot(hipStream_t st, int S, const int64_t* seg_ptr, int64_t n, int k,
                     const double* V, const double* w, double* partial, int ld) {
  if (k == 0) return;
  k_multidot<<<dim3(RED_BLOCKS, S), 256, 0, st>>>(seg_ptr, n, k, V, w, partial, ld);
}

__global__ void k_multidot_reduce(int S, int kv, const double* __restrict__ partial, int ld,
                                  double* __restrict__ h, int accumulate) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S * kv) return;
  const int s = t / kv, i = t % kv;
  double v = 0.0;
  for (int b = 0; b < RED_BLOCKS; ++b) v += partial[((int64_t)s * RED_BLOCKS + b) * ld + i];
  if (accumulate) h[(int64_t)s * ld + i] += v;
  else h[(int64_t)s * ld + i] = v;
}

void launch_multidot_reduce(hipStream_t st, int S, int k, const double* partial, int ld,
                            double* h, int accumulate) {
  if (k == 0) return;
  k_multidot_reduce<<<(S * k + 63) / 64, 64, 0, st>>>(S, k, partial, ld, h, accumulate);
}

// out_k (-)= sum_i V_i[k] c[seg(k) * ld + i]
template <bool SUB>
__global__ void k_multi_comb(int S, const int64_t* __restrict__ seg_ptr, int64_t n, int kv,
                             const double* __restrict__ V, const double* __restrict__ c, int ld,
                             double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int s = S == 1 ? 0 : seg_of(k, S, seg_ptr);
  const double* cs = c + (int64_t)s * ld;
  double acc = 0.0;
  for (int i = 0; i < kv; ++i) acc += V[(int64_t)i * n + k] * cs[i];
  out[k] = SUB ? out[k] - acc : acc;
}

void launch_multi_axpy(hipStream_t st, int S, const int64_t* seg_ptr, int64_t n, int k,
                       const double* V, const double* h, int ld, double* w) {
  if (n == 0 || k == 0) return;
  k_multi_comb<true><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(S, seg_ptr, n, k, V, h, ld, w);
}

void launch_multi_gemv(hipStream_t st, int S, const int64_t* seg_ptr, int64_t n, int k,
                       const double* V, const double* y, int ld, double* out) {
  if (n == 0) return;
  k_multi_comb<false><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(S, seg_ptr, n, k, V, y, ld, out);
}

__global__ void k_normalize_seg(int64_t n, int S, const int64_t* __restrict__ seg_ptr,
                                const double* __restrict__ nrm2, const int32_t* __restrict__ done,
                                const double* __restrict__ a, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int s = S == 1 ? 0 : seg_of(k, S, seg_ptr);
  const double q = nrm2[s];
  const bool ok = q > 0.0 && isfinite(q) && (done == nullptr || done[s] == 0);
  out[k] = ok ? a[k] / sqrt(q) : 0.0;
}

void launch_normalize_seg(hipStream_t st, int64_t n, int S, const int64_t* seg_ptr,
                          const double* nrm2, const int32_t* done, const double* a, double* out) {
  if (n == 0) return;
  k_normalize_seg<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, S, seg_ptr, nrm2, done, a, out);
}

__global__ void k_seg_sum(int S, const double* __restrict__ partial, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double v = 0.0;
  for (int b = 0; b < RED_BLOCKS; ++b) v += partial[(int64_t)s * RED_BLOCKS + b];
  out[s] = v;
}

void launch_seg_sum(hipStream_t st, int S, const double* partial, double* out) {
  k_seg_sum<<<(S + 63) / 64, 64, 0, st>>>(S, partial, out);
}

}  // namespace lsq2l
