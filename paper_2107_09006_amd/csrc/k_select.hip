// Coarse-space selection per subdomain (Lemma 2.4 / eq. gevp, reduced to the
// interface pencil; see k_coarse.hip for the reduction).
//
// With T = L_GI L_GI^T and Ct = Ct_GG (both diagonally scaled by the
// equilibration of C_ii), the selected directions are the eigenvectors of
//     K = W^T T W,   W^T Ct W = I,  range(W) = range(Ct),
// with eigenvalue sigma^2 > 1 - tau.  One workgroup per subdomain:
//   1. W: if Ct is diagonal, W = diag(Ct)^{-1/2}.  Otherwise a pivoted
//      Cholesky P^T Ct P = R^T R of the unit-diagonal scaled Ct, stopped when
//      the largest remaining diagonal falls below n eps (rank r), and
//      W = P [R11^{-1}; 0].  R W = I gives W^T Ct W = I; range(W) differs from
//      range(Ct) by null(Ct) only, which T annihilates (T <= Ct_GG because the
//      splitting matrix Ct_ii is positive semidefinite with C_I as its
//      interior block), so K is the same as on range(Ct);
//   2. K = W^T T W with MFMA tile products; if (1 - tau) I - K has a
//      Cholesky factor (tiled, on MFMA), no eigenvalue reaches the threshold
//      and the subdomain selects nothing (steps 3-6 are skipped);
//   3. Householder tridiagonalization of K;
//   4. p = number of eigenvalues above 1 - tau (one Sturm count), then the
//      p largest eigenvalues by multisection (one wave each);
//   5. eigenvectors of the tridiagonal matrix by inverse iteration (one
//      thread per vector), clusters of close eigenvalues re-orthonormalised,
//      and back-transformation through the Householder reflectors;
//   6. Y = W U (interface coefficients of the selected vectors), sigma.
// With qr_range (the QR route of Remarks 3.1 / 3.2), ctg holds instead the
// upper triangle R_G of a QR of A(Xi_i, Omega_Gamma_i) S (R_G^T R_G = Ct),
// and step 1 takes W from a QR with column pivoting of R_G with unit
// columns, stopped when the largest remaining column norm is at most n eps:
// no Gram matrix of A is formed on the way to W.  With T from the QR factor
// of A(Xi_i, Omega_i), K = W^T T W is the Gram matrix of Q_I^T Q_G and its
// eigenvalues are the squared cosines of the principal angles between
// range(A(Xi_i, Omega_Ii)) and range(A(Xi_i, Omega_Gamma_i)).
// Work matrices (ld = nGp, five per subdomain at 5 g_off): M0 scaled Ct and
// the pivoted factor, then K and the Householder vectors, then Y; M1 the
// permuted T, then U; M2 R11^{-T}; M3 products, then with M4 the scratch of
// the inverse iteration (3 r doubles per vector, the vector index fastest).
#include "kernels.hpp"

namespace lsq2l {

constexpr int SEL_THREADS = 1024;
constexpr int SEL_MAXN = 1024;
constexpr int SEL_NBP = 24;        // rows of the pivoted Cholesky per panel (interfaces above 128)
constexpr int TRD_U = 8;           // loads in flight per thread in the tridiagonalization
constexpr int TRD_NB = 16;         // reflectors per panel of the tridiagonalization
constexpr double SEL_EPS = 2.220446049250313e-16;

// ----------------------------------------------------------------------------
// block-wide reductions (a wave sum, one LDS round across waves)
// ----------------------------------------------------------------------------
__device__ inline double wg_sum(double v, double* red) {
  v = wave_allsum(v);
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, nw = blockDim.x / 64;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += red[q];   // every thread, fixed order
  return s;
}

// argmax of v over the block (ties: smallest index); returns (value, index)
__device__ inline void wg_argmax(double v, int idx, double* redv, int* redi, double* outv, int* outi) {
  for (int w = 32; w > 0; w >>= 1) {
    const double ov = __shfl_down(v, w, 64);
    const int oi = __shfl_down(idx, w, 64);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, nw = blockDim.x / 64;
  __syncthreads();
  if (lane == 0) { redv[wave] = v; redi[wave] = idx; }
  __syncthreads();
  double bv = redv[0];
  int bi = redi[0];
  for (int q = 1; q < nw; ++q)
    if (redv[q] > bv || (redv[q] == bv && redi[q] < bi)) { bv = redv[q]; bi = redi[q]; }
  *outv = bv;
  *outi = bi;
}

// ----------------------------------------------------------------------------
// tridiagonal helpers (single thread)
// ----------------------------------------------------------------------------
// 1 / x for |x| in the normal range: hardware estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r) (the error roughly squares each
// step); a few units in the last place from the rounded quotient, in a
// third of the dependent latency of a division
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Sturm count with the reciprocal above, for the bisection steps (the count
// that decides how many eigenvalues are selected uses sturm_below)
__device__ inline int sturm_below_fast(const double* d, const double* e, int n, double x,
                                       double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] * rcp_nr(q);
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__device__ inline int sturm_below(const double* d, const double* e, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Solve (T - lam I) x = sc b (b overwritten by x) with Gaussian elimination
// and row interchanges; a, up, u2 are scratch of length n.  The elimination
// carries the entries of rows i and i + 1 it updates in registers and only
// stores the finished row i, so no step reads back what the previous one
// wrote; the back substitution reads the stored rows.  Both sweeps load
// their operands TRI_CH rows at a time ahead of the dependent steps.
constexpr int TRI_CH = 4;
__device__ void tri_solve(const double* __restrict__ d, const double* __restrict__ e, int n,
                          double lam, double tiny, double sc, double* __restrict__ b,
                          double* __restrict__ a, double* __restrict__ up,
                          double* __restrict__ u2, int sst) {
  // row i: diagonal ai, superdiagonal upi, right-hand side bi; row i + 1:
  // diagonal an, superdiagonal upn, right-hand side bn
  double ai = d[0] - lam, upi = n > 1 ? e[0] : 0.0, bi = b[0] * sc;
  for (int i0 = 0; i0 + 1 < n; i0 += TRI_CH) {
    double bq[TRI_CH];
#pragma unroll
    for (int u = 0; u < TRI_CH; ++u) bq[u] = i0 + 1 + u < n ? b[i0 + 1 + u] * sc : 0.0;
#pragma unroll
    for (int u = 0; u < TRI_CH; ++u) {
      const int i = i0 + u;
      if (i + 1 >= n) break;
      const double lo = e[i];
      double an = d[i + 1] - lam, upn = i + 2 < n ? e[i + 1] : 0.0, bn = bq[u];
      double u2i = 0.0;
      if (fabs(ai) >= fabs(lo)) {
        if (ai == 0.0) ai = tiny;
        const double mlt = lo * rcp_nr(ai);
        an -= mlt * upi;
        bn -= mlt * bi;
      } else {
        const double mlt = ai * rcp_nr(lo);
        ai = lo;
        const double t = an;
        an = upi - mlt * t;
        if (i + 2 < n) { u2i = upn; upn = -mlt * u2i; }
        upi = t;
        const double bo = bi;
        bi = bn;
        bn = bo - mlt * bn;
      }
      a[i * sst] = ai;
      up[i * sst] = upi;
      u2[i * sst] = u2i;
      b[i] = bi;
      ai = an;
      upi = upn;
      bi = bn;
    }
  }
  if (ai == 0.0) ai = tiny;
  double x1 = bi * rcp_nr(ai), x2 = 0.0;     // x(i + 1), x(i + 2)
  b[n - 1] = x1;
  if (n >= 2) {
    x2 = x1;
    x1 = (b[n - 2] - up[(n - 2) * sst] * x2) * rcp_nr(a[(n - 2) * sst]);
    b[n - 2] = x1;
  }
  for (int i0 = n - 3; i0 >= 0; i0 -= TRI_CH) {
    double aq[TRI_CH], uq[TRI_CH], vq[TRI_CH], bq[TRI_CH];
#pragma unroll
    for (int u = 0; u < TRI_CH; ++u) {
      const int i = i0 - u;
      aq[u] = i >= 0 ? a[i * sst] : 1.0;
      uq[u] = i >= 0 ? up[i * sst] : 0.0;
      vq[u] = i >= 0 ? u2[i * sst] : 0.0;
      bq[u] = i >= 0 ? b[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < TRI_CH; ++u) {
      const int i = i0 - u;
      if (i < 0) break;
      const double x = (bq[u] - uq[u] * x1 - vq[u] * x2) * rcp_nr(aq[u]);
      b[i] = x;
      x2 = x1;
      x1 = x;
    }
  }
}

// ----------------------------------------------------------------------------
// the selection kernel
// ----------------------------------------------------------------------------
// acc += sign * A * B with A, B 32 x 32 column-major (leading dims lda, ldb).
template <bool NEG>
__device__ inline void tile_mma_nn(double4_t acc[4], const double* A, int lda, const double* B,
                                   int ldb, int lane) {
  const int li = lane % 16, lk = lane / 16;
#pragma unroll 2
  for (int kk = 0; kk < TS; kk += 4) {
    double a0 = A[(int64_t)(kk + lk) * lda + li];
    double a1 = A[(int64_t)(kk + lk) * lda + 16 + li];
    const double b0 = B[(int64_t)li * ldb + kk + lk];
    const double b1 = B[(int64_t)(16 + li) * ldb + kk + lk];
    if (NEG) { a0 = -a0; a1 = -a1; }
    acc[0] = Mfma<double>::mma(a0, b0, acc[0]);
    acc[1] = Mfma<double>::mma(a0, b1, acc[1]);
    acc[2] = Mfma<double>::mma(a1, b0, acc[2]);
    acc[3] = Mfma<double>::mma(a1, b1, acc[3]);
  }
}

// X = R^{-1} for the upper triangle R of a 32 x 32 tile (column-major, ld):
// lane c < 32 forms column c by back substitution, X(a, c) = -(sum_{b =
// a+1..c} R(a, b) X(b, c)) / R(a, a) from X(c, c) = 1 / R(c, c), the lower
// part set to zero.  Each lane reads only what it wrote itself.
__device__ inline void tri_inv_upper_tile(const double* R, int ld, double* X, int lane) {
  if (lane < TS) {
    const int c = lane;
    double* xc = X + (int64_t)c * ld;
    for (int a = c + 1; a < TS; ++a) xc[a] = 0.0;
    xc[c] = 1.0 / R[(int64_t)c * ld + c];
    for (int a = c - 1; a >= 0; --a) {
      double t = 0.0;
      for (int b = a + 1; b <= c; ++b) t += R[(int64_t)b * ld + a] * xc[b];
      xc[a] = -t / R[(int64_t)a * ld + a];
    }
  }
  wg_fence();
}

// The same by one wave with the tile staged in LDS (sR, sX: TS x LDT), X
// formed there and copied out: the dependent reads of the back substitution
// then go to LDS instead of global memory.
__device__ inline void tri_inv_upper_tile_lds(const double* R, int ld, double* X, double* sR,
                                              double* sX, int lane) {
  for (int e = lane; e < TT; e += 64) {
    const int a = e % TS, c = e / TS;
    sR[c * LDT + a] = R[(int64_t)c * ld + a];
  }
  wave_sync();
  if (lane < TS) {
    const int c = lane;
    double* xc = sX + c * LDT;
    for (int a = c + 1; a < TS; ++a) xc[a] = 0.0;
    xc[c] = 1.0 / sR[c * LDT + c];
    for (int a = c - 1; a >= 0; --a) {
      double t = 0.0;
      for (int b = a + 1; b <= c; ++b) t += sR[b * LDT + a] * xc[b];
      xc[a] = -t / sR[a * LDT + a];
    }
  }
  wave_sync();
  for (int e = lane; e < TT; e += 64) {
    const int a = e % TS, c = e / TS;
    X[(int64_t)c * ld + a] = sX[c * LDT + a];
  }
  wg_fence();
}

// acc += sign * A * B^T (32 x 32 tiles, column-major), operands loaded one
// contraction step of four at a time (fewer registers than tile_mma_nt)
template <bool NEG>
__device__ inline void tile_mma_nt_lean(double4_t acc[4], const double* A, int lda, const double* B,
                                        int ldb, int lane) {
  const int li = lane % 16, lk = lane / 16;
#pragma unroll 2
  for (int kk = 0; kk < TS; kk += 4) {
    double a0 = A[(int64_t)(kk + lk) * lda + li];
    double a1 = A[(int64_t)(kk + lk) * lda + 16 + li];
    const double b0 = B[(int64_t)(kk + lk) * ldb + li];
    const double b1 = B[(int64_t)(kk + lk) * ldb + 16 + li];
    if (NEG) { a0 = -a0; a1 = -a1; }
    acc[0] = Mfma<double>::mma(a0, b0, acc[0]);
    acc[1] = Mfma<double>::mma(a0, b1, acc[1]);
    acc[2] = Mfma<double>::mma(a1, b0, acc[2]);
    acc[3] = Mfma<double>::mma(a1, b1, acc[3]);
  }
}

// Cholesky factor L (lower triangle, in place) and Inv = L^{-1} of a 32 x 32
// tile W in LDS (leading dimension LDT, lower part read) by one wave.  Step k
// scales column k and updates the trailing lower triangle, lanes over rows
// and two interleaved column sets; then lane c < 32 forms column c of the
// inverse by forward substitution (only if want_inv).  Returns false if a
// pivot is not positive and finite (it is then taken as 1).
__device__ inline bool tile_chol_inv_lds(double* W, double* Inv, int lane, bool want_inv) {
  bool ok = true;
  const int i = lane % TS, h = lane / TS;
  for (int k = 0; k < TS; ++k) {
    double d = W[k * LDT + k];
    if (!(d > 0.0) || !(d < INFINITY)) { ok = false; d = 1.0; }
    const double sd = sqrt(d), rs = 1.0 / sd;
    wave_sync();
    if (h == 0 && i > k) W[k * LDT + i] *= rs;
    if (lane == k) W[k * LDT + k] = sd;
    wave_sync();
    if (i > k) {
      const double lik = W[k * LDT + i];
      for (int j = k + 1 + h; j <= i; j += 2) W[j * LDT + i] -= lik * W[k * LDT + j];
    }
    wave_sync();
  }
  if (want_inv && h == 0) {
    double* xc = Inv + i * LDT;
    for (int a = 0; a < i; ++a) xc[a] = 0.0;
    xc[i] = 1.0 / W[i * LDT + i];
    for (int a = i + 1; a < TS; ++a) {
      double t = 0.0;
      for (int b = i; b < a; ++b) t += W[b * LDT + a] * xc[b];
      xc[a] = -t / W[a * LDT + a];
    }
  }
  wave_sync();
  return ok;
}

// True if S = sh I - K is positive definite for the symmetric K (r x r,
// column-major, leading dimension ld): a right-looking Cholesky of S by
// 32 x 32 tiles in M (its lower triangle, identity on the padding to whole
// tiles; ld >= the padded size), the diagonal tile by one wave in LDS, the
// tiles below it and the trailing tiles on MFMA; a pivot that is not
// positive ends it.  Called by the whole workgroup; sW, sI are LDS tiles.
__device__ __forceinline__ bool below_shift(const double* K, double* M, int r, int ld, double sh,
                                         double* sW, double* sI, int* s_ok) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nb = (r + TS - 1) / TS, np = nb * TS;
  const int wv = tid / 64, ln = tid % 64, nwv = nthr / 64;
  for (int64_t q = tid; q < (int64_t)np * np; q += nthr) {
    const int a = (int)(q % np), c = (int)(q / np);
    if (a < c) continue;
    double v = a == c ? 1.0 : 0.0;
    if (a < r) v = (a == c ? sh : 0.0) - K[(int64_t)c * ld + a];
    M[(int64_t)c * ld + a] = v;
  }
  __syncthreads();
  for (int J = 0; J < nb; ++J) {
    if (wv == 0) {
      const double* Sjj = M + (int64_t)(J * TS) * ld + J * TS;
      for (int e = ln; e < TT; e += 64) {
        const int a = e % TS, c = e / TS;
        sW[c * LDT + a] = a >= c ? Sjj[(int64_t)c * ld + a] : 0.0;
      }
      wave_sync();
      const bool ok = tile_chol_inv_lds(sW, sI, ln, J + 1 < nb);
      if (ln == 0) *s_ok = ok;
    }
    __syncthreads();
    if (!*s_ok) return false;
    // S_IJ <- S_IJ L_JJ^{-T} below the diagonal tile
    for (int I = J + 1 + wv; I < nb; I += nwv) {
      double* Sij = M + (int64_t)(J * TS) * ld + I * TS;
      double4_t acc[4];
      tile_acc_zero<double>(acc);
      tile_mma_nt_lean<false>(acc, Sij, ld, sI, LDT, ln);
      tile_acc_store<double>(acc, Sij, ld, ln);
    }
    __syncthreads();
    // S_ab -= S_aJ S_bJ^T for J < b <= a
    const int m = nb - J - 1;
    for (int it = wv; it < m * (m + 1) / 2; it += nwv) {
      int a = (int)((sqrt(8.0 * it + 1.0) - 1.0) / 2.0);
      while (a * (a + 1) / 2 > it) --a;
      while ((a + 1) * (a + 2) / 2 <= it) ++a;
      const int b = it - a * (a + 1) / 2;
      const int ta = J + 1 + a, tb = J + 1 + b;
      double* Sab = M + (int64_t)(tb * TS) * ld + ta * TS;
      double4_t acc[4];
      tile_acc_load<double>(acc, Sab, ld, ln);
      tile_mma_nt_lean<true>(acc, M + (int64_t)(J * TS) * ld + ta * TS, ld,
                             M + (int64_t)(J * TS) * ld + tb * TS, ld, ln);
      tile_acc_store<double>(acc, Sab, ld, ln);
    }
    __syncthreads();
  }
  return true;
}

// Interfaces of up to MAXN columns (and more than MINN) with THREADS threads:
// the LDS arrays scale with MAXN, so small interfaces run many workgroups
// per CU.  Workgroups of other sizes return at once.
template <int THREADS, int MINN, int MAXN>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(4)))
k_select(const SubDesc* __restrict__ subs, const double* __restrict__ ctg,
         const double* __restrict__ Tg, double* __restrict__ work, double tau, int nev_max,
         int32_t* __restrict__ p_out, double* __restrict__ sig_out, int32_t* __restrict__ fail,
         int qr_range) {
  constexpr int NG = THREADS / 256;   // thread groups splitting the columns of A22 v
  static_assert(NG >= 1 && THREADS % 256 == 0, "whole groups of 256 threads");
  __shared__ double sd[MAXN], se[MAXN], stau[MAXN], sv[MAXN], sw[MAXN], sD2[MAXN], slam[MAXN];
  __shared__ int sperm[MAXN], scl[MAXN + 1];
  __shared__ double spart[NG][MAXN];
  __shared__ double svp[MAXN], swp[MAXN];   // the previous reflector's v and w
  __shared__ double sred[16];
  __shared__ int sredi[16];
  __shared__ double sPW[TS * LDT], sPI[TS * LDT];   // diagonal tile of the test of step 2b
  __shared__ double sc1[TRD_NB], sc2[TRD_NB];   // dot products of the tridiagonalization's panel
  __shared__ int s_r, s_p, s_nclus, s_diag, s_pd;
  __shared__ double s_anorm;
  const SubDesc dsc = subs[blockIdx.x];
  const int i = dsc.id;
  const int n = dsc.nG, ld = dsc.nGp, tid = threadIdx.x, nthr = blockDim.x;
  if (n <= MINN) {
    if (n == 0 && MINN == 0 && tid == 0) p_out[i] = 0;
    return;
  }
  if (n > MAXN) {
    if (MAXN == SEL_MAXN && tid == 0) { p_out[i] = 0; atomicExch(fail, 2); }
    return;
  }
  const int64_t mm = (int64_t)ld * ld;
  double* M0 = work + SEL_WORK_MATS * dsc.g_off;
  double* M1 = M0 + mm;
  double* M2 = M1 + mm;
  double* M3 = M2 + mm;
  const double* Ct = ctg + dsc.g_off;
  const double* T = Tg + dsc.g_off;

  // ---- 1. scaled Ct (unit diagonal) and the range basis W
  // a zero diagonal (stored zeros only) leaves its column out of range(Ct)
  int nz = 0;
  for (int a = tid; a < n; a += nthr) {
    double c = 0.0;
    if (qr_range) {                       // diagonal of Ct = squared column norm of R_G
      for (int b = 0; b <= a; ++b) { const double t = Ct[(int64_t)a * ld + b]; c += t * t; }
    } else {
      c = Ct[(int64_t)a * ld + a];
    }
    sD2[a] = c > 0.0 ? 1.0 / sqrt(c) : 0.0;
    nz += !(c > 0.0);
  }
  __syncthreads();
  double off = (double)nz;
  for (int64_t q = tid; q < mm; q += nthr) {
    const int r = (int)(q % ld), c = (int)(q / ld);
    double v = 0.0;
    if (r < n && c < n) {
      if (qr_range) {
        // R_G D2, upper triangle; Ct is diagonal iff R_G is
        v = r <= c ? Ct[(int64_t)c * ld + r] * sD2[c] : 0.0;
      } else {
        v = (r >= c) ? Ct[(int64_t)c * ld + r] : Ct[(int64_t)r * ld + c];
        v *= sD2[r] * sD2[c];
      }
      if (r != c) off += fabs(v);   // exact zero test: any coupling needs the general route
    }
    M0[q] = v;
  }
  off = wg_sum(off, sred);
  if (tid == 0) s_diag = (off == 0.0);
  __syncthreads();
  int r;
  if (s_diag) {
    // W = D2 (diagonal): K = D2 T D2 elementwise
    r = n;
    for (int64_t q = tid; q < mm; q += nthr) {
      const int a = (int)(q % ld), c = (int)(q / ld);
      M0[q] = (a < n && c < n) ? sD2[a] * T[(int64_t)c * ld + a] * sD2[c] : 0.0;
    }
    __syncthreads();
  } else {
   if (qr_range) {
    // QR with column pivoting of M0 = R_G D2 (unit columns): step k takes the
    // remaining column of largest norm (ties: the first), reflects it onto
    // row k and applies the reflector to the columns right of it, one thread
    // per column.  Column norms over rows k.. are downdated and recomputed
    // when the downdate has cancelled below 1e-4 of the last exact value.  R
    // ends in the upper triangle, sperm holds the column order.
    double* snrm = sd;                    // sd / se are free until step 3
    double* sref = se;
    for (int a = tid; a < n; a += nthr) {
      sperm[a] = a;
      double t = 0.0;
      for (int b = 0; b < n; ++b) { const double x = M0[(int64_t)a * ld + b]; t += x * x; }
      snrm[a] = t;
      sref[a] = t;
    }
    __syncthreads();
    const double tol = (double)n * SEL_EPS;
    int k = 0;
    for (; k < n; ++k) {
      double bv = -1.0;
      int bi = n;
      for (int j = k + tid; j < n; j += nthr)
        if (snrm[j] > bv) { bv = snrm[j]; bi = j; }
      double mv;
      int mj;
      wg_argmax(bv, bi, sred, sredi, &mv, &mj);
      if (!(mv > tol * tol)) break;
      if (mj != k) {
        for (int a = tid; a < n; a += nthr) {
          const double t = M0[(int64_t)k * ld + a];
          M0[(int64_t)k * ld + a] = M0[(int64_t)mj * ld + a];
          M0[(int64_t)mj * ld + a] = t;
        }
        __syncthreads();
        if (tid == 0) {
          int t = sperm[k]; sperm[k] = sperm[mj]; sperm[mj] = t;
          double u = snrm[k]; snrm[k] = snrm[mj]; snrm[mj] = u;
          u = sref[k]; sref[k] = sref[mj]; sref[mj] = u;
        }
        __syncthreads();
      }
      // alpha is read before the barriers of the sum: (k, k) is overwritten below
      const double alpha = M0[(int64_t)k * ld + k];
      double part = 0.0;
      for (int a = k + 1 + tid; a < n; a += nthr) { const double t = M0[(int64_t)k * ld + a]; part += t * t; }
      const double xn2 = wg_sum(part, sred);
      double tk = 0.0, beta = alpha, scl = 0.0;
      if (xn2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tk = (beta - alpha) / beta;
        scl = 1.0 / (alpha - beta);
      }
      for (int a = k + tid; a < n; a += nthr) {
        sv[a] = a == k ? 1.0 : M0[(int64_t)k * ld + a] * scl;
        M0[(int64_t)k * ld + a] = a == k ? beta : 0.0;
      }
      __syncthreads();
      // one wave per column, lanes over its rows (each lane rereads only
      // the entries it wrote)
      {
        const int wv = tid / 64, ln = tid % 64, nwv = nthr / 64;
        for (int j = k + 1 + wv; j < n; j += nwv) {
          double* cj = M0 + (int64_t)j * ld;
          const double ck = cj[k];
          double w = 0.0;
          if (tk != 0.0) {
            for (int a = k + ln; a < n; a += 64) w += sv[a] * cj[a];
            w = wave_allsum(w) * tk;
            for (int a = k + ln; a < n; a += 64) cj[a] -= w * sv[a];
          }
          const double ckn = ck - w;          // the new entry (k, j): sv[k] = 1
          double t = snrm[j] - ckn * ckn;
          if (!(t > 1e-4 * sref[j])) {
            double part = 0.0;
            for (int a = k + ln; a < n; a += 64)
              if (a > k) part += cj[a] * cj[a];
            t = wave_allsum(part);
            if (ln == 0) sref[j] = t;
          }
          if (ln == 0) snrm[j] = t;
        }
      }
      __syncthreads();
    }
    r = k;
   } else {
    // pivoted Cholesky of M0 (both triangles) without moving entries: thread
    // c owns column c and its updated diagonal d_c.  Step k takes the
    // unpivoted column c* of largest d (ties: the smallest index); row k of R
    // in the original column order is
    //   R(k, c) = (M0(c*, c) - sum_{s in panel, s < k} R(s, c*) R(s, c)) / sqrt(d_c*)
    // (zero on columns pivoted earlier), and d_c -= R(k, c)^2.  Rows are
    // formed NBP at a time in registers; M0 (its upper triangle, the only
    // part read) takes the panel's update R_P^T R_P once per panel, on MFMA.
    // R goes to M3 (entry (k, c) at c ld + k) and, for the panel update, to
    // M2 (at k ld + c); R11 in pivot order goes back to the upper triangle of
    // M0 at the end.  sperm holds the pivot order, then the unpivoted columns
    // in ascending order.
    constexpr int NBP = MAXN <= 128 ? 16 : SEL_NBP;
    const double tol = n * SEL_EPS;     // the scaled matrix has unit diagonal
    const int wv = tid / 64, ln = tid % 64, nwv = nthr / 64;
    double dc = tid < n ? M0[(int64_t)tid * ld + tid] : 0.0;
    bool piv = tid >= n;                  // pivoted (or not a column)
    int k = 0;
    bool stop = n == 0;
    while (!stop) {
      const int k0 = k;
      double P[NBP];
#pragma unroll
      for (int jj = 0; jj < NBP; ++jj) {
        P[jj] = 0.0;
        if (stop) continue;               // uniform
        double mv;
        int mj;
        wg_argmax(piv ? -1.0 : dc, piv ? n : tid, sred, sredi, &mv, &mj);
        if (!(mv > tol)) { stop = true; continue; }
        if (tid == mj) {
#pragma unroll
          for (int q = 0; q < jj; ++q) sv[q] = P[q];
          sperm[k] = mj;
        }
        __syncthreads();
        if (tid < n) {
          // M0(c*, c) from the upper triangle
          double u = tid <= mj ? M0[(int64_t)mj * ld + tid] : M0[(int64_t)tid * ld + mj];
#pragma unroll
          for (int q = 0; q < jj; ++q) u -= sv[q] * P[q];
          const double sk = sqrt(mv);
          if (tid == mj) {
            P[jj] = sk;
            piv = true;
          } else if (!piv) {
            P[jj] = u / sk;
            dc -= P[jj] * P[jj];
          }
        }
        ++k;
        if (k == n) stop = true;
      }
      const int nr = k - k0;
      if (tid < n)
#pragma unroll
        for (int q = 0; q < NBP; ++q)
          if (q < nr) {
            M3[(int64_t)tid * ld + k0 + q] = P[q];     // column c of R, for R11 below
            M2[(int64_t)(k0 + q) * ld + tid] = P[q];   // row k of R, for the panel update
          }
      __syncthreads();
      if (stop) break;
      // M0 -= R_P^T R_P on the 32 x 32 tiles (I, J), I <= J, of the upper
      // triangle, one wave per tile
      const int nbt = (n + TS - 1) / TS;
      const int li = ln % 16, lk = ln / 16;
      for (int t = wv; t < nbt * (nbt + 1) / 2; t += nwv) {
        int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) / 2.0);
        while (J * (J + 1) / 2 > t) --J;
        while ((J + 1) * (J + 2) / 2 <= t) ++J;
        const int I = t - J * (J + 1) / 2;
        double* Cij = M0 + (int64_t)(J * TS) * ld + I * TS;
        double4_t acc[4];
        tile_acc_load<double>(acc, Cij, ld, ln);
        const double* RI = M2 + (int64_t)k0 * ld + I * TS;
        const double* RJ = M2 + (int64_t)k0 * ld + J * TS;
#pragma unroll
        for (int s0 = 0; s0 < NBP; s0 += 4) {
          const double a0 = -RI[(int64_t)(s0 + lk) * ld + li];
          const double a1 = -RI[(int64_t)(s0 + lk) * ld + 16 + li];
          const double b0 = RJ[(int64_t)(s0 + lk) * ld + li];
          const double b1 = RJ[(int64_t)(s0 + lk) * ld + 16 + li];
          acc[0] = Mfma<double>::mma(a0, b0, acc[0]);
          acc[1] = Mfma<double>::mma(a0, b1, acc[1]);
          acc[2] = Mfma<double>::mma(a1, b0, acc[2]);
          acc[3] = Mfma<double>::mma(a1, b1, acc[3]);
        }
        tile_acc_store<double>(acc, Cij, ld, ln);
      }
      __syncthreads();
    }
    // the unpivoted columns after the r pivots, ascending
    {
      const bool up = tid < n && !piv;
      const unsigned long long bal = __ballot(up);
      if (ln == 0) sredi[wv] = __popcll(bal);
      __syncthreads();
      int base = k;
      for (int w = 0; w < wv; ++w) base += sredi[w];
      if (up) sperm[base + __popcll(bal & ((1ull << ln) - 1ull))] = tid;
      __syncthreads();
    }
    // R11 (r x r, pivot order) into the upper triangle of M0, zero elsewhere
    for (int64_t q = tid; q < mm; q += nthr) {
      const int a = (int)(q % ld), c = (int)(q / ld);
      M0[q] = (a <= c && c < k) ? M3[(int64_t)sperm[c] * ld + a] : 0.0;
    }
    __syncthreads();
    r = k;
   }
    if (r == 0) {
      if (tid == 0) p_out[i] = 0;
      return;
    }
    // M2 = Q = R11^{-T} from X = R11^{-1}, formed in M3 by 32 x 32 tiles.
    // The factor is padded to nb tiles with an identity block, so X is too.
    // Phase 1: each diagonal tile's inverse D_I (one wave per tile); phase
    // 2: column block J, from I = J - 1 up to 0,
    //   X_IJ = -D_I (sum_{K = I+1..J} R_IK X_KJ),
    // one wave per column block, on MFMA; phase 3: Q = X^T.
    {
      const int nb = (r + TS - 1) / TS, np = nb * TS;
      const int wv = tid / 64, ln = tid % 64, nwv = nthr / 64;
      for (int64_t q = tid; q < (int64_t)np * np; q += nthr) {
        const int a = (int)(q % np), c = (int)(q / np);
        if (a <= c && c >= r) M0[(int64_t)c * ld + a] = (a == c) ? 1.0 : 0.0;
      }
      __syncthreads();
      // (up to four tiles one after another by wave 0 through LDS, more in
      // parallel, one wave each, in global memory)
      if (nb <= 4) {
        if (wv == 0)
          for (int I = 0; I < nb; ++I)
            tri_inv_upper_tile_lds(M0 + (int64_t)(I * TS) * ld + I * TS, ld,
                                   M3 + (int64_t)(I * TS) * ld + I * TS, sPW, sPI, ln);
      } else {
        for (int I = wv; I < nb; I += nwv)
          tri_inv_upper_tile(M0 + (int64_t)(I * TS) * ld + I * TS, ld,
                             M3 + (int64_t)(I * TS) * ld + I * TS, ln);
      }
      __syncthreads();
      for (int J = wv; J < nb; J += nwv)
        for (int I = J - 1; I >= 0; --I) {
          double4_t acc[4];
          tile_acc_zero<double>(acc);
          for (int K = I + 1; K <= J; ++K)
            tile_mma_nn<false>(acc, M0 + (int64_t)(K * TS) * ld + I * TS, ld,
                               M3 + (int64_t)(J * TS) * ld + K * TS, ld, ln);
          double* Xij = M3 + (int64_t)(J * TS) * ld + I * TS;   // the sum, then X_IJ
          tile_acc_store<double>(acc, Xij, ld, ln);
          wg_fence();
          tile_acc_zero<double>(acc);
          tile_mma_nn<true>(acc, M3 + (int64_t)(I * TS) * ld + I * TS, ld, Xij, ld, ln);
          wg_fence();
          tile_acc_store<double>(acc, Xij, ld, ln);
          wg_fence();
        }
      __syncthreads();
      for (int64_t q = tid; q < mm; q += nthr) {
        const int a = (int)(q % ld), c = (int)(q / ld);
        M2[q] = (a < r && c <= a) ? M3[(int64_t)a * ld + c] : 0.0;
      }
      __syncthreads();
    }
    // M1 = T11 = D2 T D2 in pivot order (r x r, zero padded)
    for (int64_t q = tid; q < mm; q += nthr) {
      const int a = (int)(q % ld), c = (int)(q / ld);
      double v = 0.0;
      if (a < r && c < r) {
        const int pa = sperm[a], pc = sperm[c];
        v = sD2[pa] * T[(int64_t)pc * ld + pa] * sD2[pc];
      }
      M1[q] = v;
    }
    __syncthreads();
    // K = Q T11 Q^T by 32 x 32 tiles, one wave per output tile, with Q lower
    // triangular: M3 = Q T11 (tile (I, J) sums K <= I), then the lower tiles
    // of M0 = M3 Q^T (tile (I, J), I >= J, sums K <= J), mirrored to the
    // upper triangle
    {
      const int nb = (r + TS - 1) / TS;
      const int wv = tid / 64, ln = tid % 64, nwv = nthr / 64;
      for (int t = wv; t < nb * nb; t += nwv) {
        const int I = t % nb, J = t / nb;
        double4_t acc[4];
        tile_acc_zero<double>(acc);
        for (int K = 0; K <= I; ++K)
          tile_mma_nn<false>(acc, M2 + (int64_t)(K * TS) * ld + I * TS, ld,
                             M1 + (int64_t)(J * TS) * ld + K * TS, ld, ln);
        tile_acc_store<double>(acc, M3 + (int64_t)(J * TS) * ld + I * TS, ld, ln);
      }
      __syncthreads();
      for (int t = wv; t < nb * (nb + 1) / 2; t += nwv) {
        int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) / 2.0);
        while (I * (I + 1) / 2 > t) --I;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        const int J = t - I * (I + 1) / 2;        // J <= I
        double4_t acc[4];
        tile_acc_zero<double>(acc);
        for (int K = 0; K <= J; ++K)
          tile_mma_nt_lean<false>(acc, M3 + (int64_t)(K * TS) * ld + I * TS, ld,
                                  M2 + (int64_t)(K * TS) * ld + J * TS, ld, ln);
        tile_acc_store<double>(acc, M0 + (int64_t)(J * TS) * ld + I * TS, ld, ln);
      }
      __syncthreads();
      for (int64_t q = tid; q < (int64_t)r * r; q += nthr) {
        const int a = (int)(q % r), c = (int)(q / r);
        if (a < c) M0[(int64_t)c * ld + a] = M0[(int64_t)a * ld + c];
      }
      __syncthreads();
    }
  }

  // ---- 2b. nothing to select: if S = (1 - tau) I - K is positive definite,
  // every eigenvalue of K lies below 1 - tau, the least value the threshold
  // of step 4 takes, and p = 0 without the eigen-decomposition.
  if (1.0 - tau > 0.0 && below_shift(M0, M1, r, ld, 1.0 - tau, sPW, sPI, &s_pd)) {
    if (tid == 0) p_out[i] = 0;
    return;
  }

  // ---- 3. tridiagonalization of K (r x r) in M0: for interfaces up to 128
  // columns step by step (below), larger ones by panels (further below).
  if constexpr (MAXN <= 128) {
  // Step k reflects column k
  // (v, tk) and updates the trailing block, A22 -= v w^T + w v^T with
  // w = tk A22 v - (tk^2 / 2) (v^T A22 v) v.  The update of step k is applied
  // during the pass of step k + 1 that forms A22 v there, so each step reads
  // and writes the trailing block once; column k + 1, which the next reflector
  // needs first, takes the pending update on its own.  Every entry receives
  // the same operations in the same order as with the update as a pass of its
  // own.
  bool pend = false;                      // svp, swp hold an update not yet applied
  for (int k = 0; k + 2 < r; ++k) {
    const int m = r - k - 1;
    // column k (rows k .. r-1) with the pending update of step k - 1, whose
    // block starts at row k (local index i - k), into sw
    for (int a = tid; a <= m; a += nthr) {
      double x = M0[(int64_t)k * ld + k + a];
      if (pend) x -= svp[a] * swp[0] + swp[a] * svp[0];
      sw[a] = x;
    }
    __syncthreads();
    double part = 0.0;
    for (int a = 1 + tid; a < m; a += nthr) { const double t = sw[1 + a]; part += t * t; }
    const double xn2 = wg_sum(part, sred);
    const double alpha = sw[1];
    double tk = 0.0, beta = alpha;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tk = (beta - alpha) / beta;
      const double sc = 1.0 / (alpha - beta);
      for (int a = tid; a < m; a += nthr) sv[a] = (a == 0) ? 1.0 : sw[1 + a] * sc;
    } else {
      for (int a = tid; a < m; a += nthr) sv[a] = (a == 0) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) { se[k] = beta; sd[k] = sw[0]; stau[k] = tk; }
    for (int a = 1 + tid; a < m; a += nthr) M0[(int64_t)k * ld + k + 1 + a] = sv[a];
    if (tk != 0.0 || pend) {
      // one pass over A22 (rows and columns k + 1 ..): the pending update,
      // then w = tk A22 v from NG thread groups splitting the columns,
      // their partial sums added in a fixed order
      const int g = tid / 256, t256 = tid % 256;
      for (int a0 = 0; a0 < m; a0 += 256) {
        const int a = a0 + t256;
        double acc = 0.0;
        if (a < m) {
          // row a of the block, columns b = g, g + NG, ...: TRD_U loads in
          // flight before their updates are stored
          double* rowa = M0 + (int64_t)(k + 1) * ld + k + 1 + a;
          const double va = svp[a + 1], wa = swp[a + 1];
          int b = g;
          for (; b + (TRD_U - 1) * NG < m; b += TRD_U * NG) {
            double x[TRD_U];
#pragma unroll
            for (int u = 0; u < TRD_U; ++u) x[u] = rowa[(int64_t)(b + u * NG) * ld];
#pragma unroll
            for (int u = 0; u < TRD_U; ++u) {
              const int bu = b + u * NG;
              if (pend) {
                x[u] -= va * swp[bu + 1] + wa * svp[bu + 1];
                rowa[(int64_t)bu * ld] = x[u];
              }
              acc += x[u] * sv[bu];
            }
          }
          for (; b < m; b += NG) {
            double x = rowa[(int64_t)b * ld];
            if (pend) {
              x -= va * swp[b + 1] + wa * svp[b + 1];
              rowa[(int64_t)b * ld] = x;
            }
            acc += x * sv[b];
          }
          spart[g][a] = acc;
        }
      }
    }
    __syncthreads();
    if (tk != 0.0) {
      double pp = 0.0;
      for (int a = tid; a < m; a += nthr) {
        double sp = spart[0][a];
#pragma unroll
        for (int q = 1; q < NG; ++q) sp += spart[q][a];
        sw[a] = tk * sp;
        pp += sw[a] * sv[a];
      }
      const double wv = wg_sum(pp, sred);
      const double a2 = -0.5 * tk * wv;
      for (int a = tid; a < m; a += nthr) {
        swp[a] = sw[a] + a2 * sv[a];
        svp[a] = sv[a];
      }
    }
    pend = tk != 0.0;
    __syncthreads();
  }
  if (pend && tid == 0) {                 // the last update reaches rows r-2, r-1
    for (int b = 0; b < 2; ++b)
      for (int a = b; a < 2; ++a)
        M0[(int64_t)(r - 2 + b) * ld + r - 2 + a] -= svp[a] * swp[b] + swp[a] * svp[b];
  }
  } else {
  // TRD_NB reflectors per panel.  Step k reflects column k (v, tk); the trailing block's update
  // A22 -= v w^T + w v^T, w = tk A22 v - (tk^2 / 2) (v^T A22 v) v, is held
  // back as the panel's columns of V and Wm (in M3) and applied once per
  // panel on MFMA tiles, so the steps only read the block: inside a panel,
  // column k and A22 v are formed from the matrix at the panel's start
  // minus V Wm^T + Wm V^T of the earlier steps.
  {
    double* VV = M3;                      // panel reflectors, column q at q ld (rows k + 1 ..)
    double* WW = M3 + (int64_t)TRD_NB * ld;
    const int wave = tid / 64, lane = tid % 64, nwv = nthr / 64;
    int k = 0;
    while (k + 2 < r) {
      const int k0 = k;
      int jj = 0;
      for (; jj < TRD_NB && k + 2 < r; ++jj, ++k) {
        const int m = r - k - 1;
        // row k of the panel's V and Wm
        if (tid < jj) { svp[tid] = VV[(int64_t)tid * ld + k]; swp[tid] = WW[(int64_t)tid * ld + k]; }
        __syncthreads();
        // column k (rows k .. r-1) of the current matrix into sw
        for (int a = tid; a <= m; a += nthr) {
          double x = M0[(int64_t)k * ld + k + a];
          for (int q = 0; q < jj; ++q)
            x -= VV[(int64_t)q * ld + k + a] * swp[q] + WW[(int64_t)q * ld + k + a] * svp[q];
          sw[a] = x;
        }
        __syncthreads();
        double part = 0.0;
        for (int a = 1 + tid; a < m; a += nthr) { const double t = sw[1 + a]; part += t * t; }
        const double xn2 = wg_sum(part, sred);
        const double alpha = sw[1];
        double tk = 0.0, beta = alpha;
        if (xn2 > 0.0) {
          beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
          tk = (beta - alpha) / beta;
          const double sc = 1.0 / (alpha - beta);
          for (int a = tid; a < m; a += nthr) sv[a] = (a == 0) ? 1.0 : sw[1 + a] * sc;
        } else {
          for (int a = tid; a < m; a += nthr) sv[a] = (a == 0) ? 1.0 : 0.0;
        }
        __syncthreads();
        if (tid == 0) { se[k] = beta; sd[k] = sw[0]; stau[k] = tk; }
        for (int a = tid; a < m; a += nthr) {
          if (a >= 1) M0[(int64_t)k * ld + k + 1 + a] = sv[a];
          VV[(int64_t)jj * ld + k + 1 + a] = sv[a];
        }
        if (tk == 0.0) {
          for (int a = tid; a < m; a += nthr) WW[(int64_t)jj * ld + k + 1 + a] = 0.0;
          __syncthreads();
          continue;
        }
        // Wm^T v and V^T v over the earlier steps of the panel, one wave each
        for (int t = wave; t < 2 * jj; t += nwv) {
          const double* col = (t < jj ? WW + (int64_t)t * ld : VV + (int64_t)(t - jj) * ld) + k + 1;
          double d = 0.0;
          for (int a = lane; a < m; a += 64) d += col[a] * sv[a];
          d = wave_allsum(d);
          if (lane == 0) { if (t < jj) sc1[t] = d; else sc2[t - jj] = d; }
        }
        // A22 v from the matrix at the panel's start, NG thread groups
        // splitting the columns, TRD_U loads in flight
        {
          const int g = tid / 256, t256 = tid % 256;
          for (int a0 = 0; a0 < m; a0 += 256) {
            const int a = a0 + t256;
            if (a >= m) continue;
            const double* rowa = M0 + (int64_t)(k + 1) * ld + k + 1 + a;
            double acc = 0.0;
            int b = g;
            for (; b + (TRD_U - 1) * NG < m; b += TRD_U * NG) {
              double x[TRD_U];
#pragma unroll
              for (int u = 0; u < TRD_U; ++u) x[u] = rowa[(int64_t)(b + u * NG) * ld];
#pragma unroll
              for (int u = 0; u < TRD_U; ++u) acc += x[u] * sv[b + u * NG];
            }
            for (; b < m; b += NG) acc += rowa[(int64_t)b * ld] * sv[b];
            spart[g][a] = acc;
          }
        }
        __syncthreads();
        // y = A22 v - V (Wm^T v) - Wm (V^T v), w = tk y - (tk / 2)(tk y^T v) v
        double pp = 0.0;
        for (int a = tid; a < m; a += nthr) {
          double y = spart[0][a];
#pragma unroll
          for (int q = 1; q < NG; ++q) y += spart[q][a];
          for (int q = 0; q < jj; ++q)
            y -= VV[(int64_t)q * ld + k + 1 + a] * sc1[q] + WW[(int64_t)q * ld + k + 1 + a] * sc2[q];
          sw[a] = tk * y;
          pp += sw[a] * sv[a];
        }
        const double wv = wg_sum(pp, sred);
        const double a2 = -0.5 * tk * wv;
        for (int a = tid; a < m; a += nthr) WW[(int64_t)jj * ld + k + 1 + a] = sw[a] + a2 * sv[a];
        __syncthreads();
      }
      // the panel's update of rows and columns from k on (the next panel's
      // first column and everything after it): A -= V Wm^T + Wm V^T on
      // 32 x 32 tiles, entries before k left as they are
      const int nq = jj, kn = k;
      const int tlo = kn / TS, nbt = (r + TS - 1) / TS, nt = nbt - tlo;
      for (int t = wave; t < nt * nt; t += nwv) {
        const int I = tlo + t % nt, J = tlo + t / nt;
        double4_t acc[4];
        double* C = M0 + (int64_t)(J * TS) * ld + I * TS;
        tile_acc_load<double>(acc, C, ld, lane);
        const int li = lane % 16, lk = lane / 16;
        for (int q0 = 0; q0 < nq; q0 += 4) {
          const int q = q0 + lk;
          const bool in = q < nq;
          const double* vq = VV + (int64_t)q * ld;
          const double* wq = WW + (int64_t)q * ld;
          const double av0 = in ? -vq[I * TS + li] : 0.0, av1 = in ? -vq[I * TS + 16 + li] : 0.0;
          const double aw0 = in ? -wq[I * TS + li] : 0.0, aw1 = in ? -wq[I * TS + 16 + li] : 0.0;
          const double bw0 = in ? wq[J * TS + li] : 0.0, bw1 = in ? wq[J * TS + 16 + li] : 0.0;
          const double bv0 = in ? vq[J * TS + li] : 0.0, bv1 = in ? vq[J * TS + 16 + li] : 0.0;
          acc[0] = Mfma<double>::mma(av0, bw0, acc[0]);
          acc[1] = Mfma<double>::mma(av0, bw1, acc[1]);
          acc[2] = Mfma<double>::mma(av1, bw0, acc[2]);
          acc[3] = Mfma<double>::mma(av1, bw1, acc[3]);
          acc[0] = Mfma<double>::mma(aw0, bv0, acc[0]);
          acc[1] = Mfma<double>::mma(aw0, bv1, acc[1]);
          acc[2] = Mfma<double>::mma(aw1, bv0, acc[2]);
          acc[3] = Mfma<double>::mma(aw1, bv1, acc[3]);
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = I * TS + 16 * bi + Mfma<double>::acc_row(lane, v);
              const int col = J * TS + 16 * bj + Mfma<double>::acc_col(lane, v);
              if (row >= kn && col >= kn && row < r && col < r) C[(int64_t)(16 * bj + Mfma<double>::acc_col(lane, v)) * ld + 16 * bi + Mfma<double>::acc_row(lane, v)] = acc[bi * 2 + bj][v];
            }
      }
      __syncthreads();
      (void)k0;
    }
  }
  }
  __syncthreads();
  if (tid == 0) {
    if (r >= 2) { se[r - 2] = M0[(int64_t)(r - 2) * ld + r - 1]; sd[r - 2] = M0[(int64_t)(r - 2) * ld + r - 2]; }
    sd[r - 1] = M0[(int64_t)(r - 1) * ld + r - 1];
    se[r - 1] = 0.0;
    for (int k = (r >= 2 ? r - 2 : 0); k < r; ++k) stau[k] = 0.0;
    double an = 0.0;
    for (int a = 0; a < r; ++a) an = fmax(an, fabs(sd[a]) + fabs(se[a]) + (a > 0 ? fabs(se[a - 1]) : 0.0));
    s_anorm = an;
  }
  __syncthreads();
  const double anorm = s_anorm;
  if (!(anorm < INFINITY)) {            // NaN or Inf in K: report, select nothing
    if (tid == 0) { p_out[i] = 0; atomicExch(fail, 3); }
    return;
  }
  const double pivmin = fmax(SEL_EPS * anorm * 1e-2, 1e-300);

  // ---- 4. count above 1 - tau, multisection for the p largest eigenvalues.  A
  // selected sigma^2 must also be numerically positive (it divides X).
  const double thr = fmax(1.0 - tau, r * SEL_EPS * anorm);
  if (tid == 0) {
    int p = r - sturm_below(sd, se, r, thr, pivmin);
    if (nev_max > 0 && p > nev_max) p = nev_max;
    s_p = p;
  }
  __syncthreads();
  const int p = s_p;
  if (p == 0) {
    if (tid == 0) p_out[i] = 0;
    return;
  }
  // the j-th largest is the (r-1-j)-th smallest; all p lie above thr.  One
  // wave per eigenvalue, multisection: each round the 64 lanes count at 64
  // points splitting [lo, hi] into 65 equal parts, and the first point with
  // more than r-1-j eigenvalues below it bounds the interval (the invariant
  // count(lo) <= r-1-j < count(hi) of bisection, shrinking 65-fold a round)
  {
    const int wave = tid / 64, lane = tid % 64, nw = nthr / 64;
    for (int j = wave; j < p; j += nw) {
      const int kidx = r - 1 - j;
      double lo = thr, hi = anorm * (1.0 + 4.0 * SEL_EPS) + pivmin;
      for (int it = 0; it < 64; ++it) {
        if (hi - lo <= 2.0 * SEL_EPS * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        const double h = (hi - lo) / 65.0;
        const bool above = sturm_below_fast(sd, se, r, lo + (lane + 1) * h, pivmin) > kidx;
        const unsigned long long bal = __ballot(above);
        const int first = bal ? __ffsll((long long)bal) - 1 : 64;
        const double nlo = first == 0 ? lo : lo + first * h;
        const double nhi = first == 64 ? hi : lo + (first + 1) * h;
        lo = nlo;
        hi = nhi;
      }
      if (lane == 0) slam[j] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();
  // clusters of close eigenvalues (descending order); separate equal ones.
  // Inverse iteration with a shift accurate to rounding leaves a vector off
  // its eigenvector by about eps ||T|| / gap, so vectors whose eigenvalues
  // are more than 1e-6 ||T|| apart come out orthogonal to about 1e-10
  // without re-orthogonalisation; only closer ones form a cluster.
  if (tid == 0) {
    const double ortol = 1e-6 * anorm, sep = 10.0 * SEL_EPS * anorm;
    int nc = 0;
    for (int j = 0; j < p; ++j) {
      if (j > 0 && fabs(slam[j - 1] - slam[j]) < sep) slam[j] = slam[j - 1] - sep;
      if (j == 0 || slam[j - 1] - slam[j] > ortol) scl[nc++] = j;
    }
    scl[nc] = p;
    s_nclus = nc;
  }
  __syncthreads();

  // ---- 5. inverse iteration, one thread per vector (scratch of 3 r doubles
  // per vector, in LDS or in M3 / M4).  Shifts are accurate to rounding, so
  // after a few sweeps every vector lies in the invariant subspace of its
  // cluster; only clusters of (numerically) multiple eigenvalues need
  // orthonormalising, which is done after the independent sweeps and again
  // after one cleaning sweep.  Vectors in M1 (r x p).
  const double tiny = SEL_EPS * anorm;
  // The scratch sits in LDS (svp, swp, spart[0], free now: MAXN doubles each)
  // when every vector fits in one round there, else in M3 / M4.
  const bool lds_scr = p <= MAXN / r;
  const int slots = lds_scr ? p : (int)min<int64_t>(2 * mm / (3 * r), nthr);
  const int wave = tid / 64, lane = tid % 64, nw = nthr / 64;
  for (int64_t q = tid; q < (int64_t)ld * p; q += nthr) {
    const int row = (int)(q % ld), j = (int)(q / ld);
    M1[q] = row < r ? sin((row + 1.0) * (j + 1.0)) : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 4; ++sweep) {
    for (int j0 = 0; j0 < p; j0 += slots) {
      const int j = j0 + tid;
      if (tid >= slots || j >= p) continue;
      double* x = M1 + (int64_t)j * ld;
      double* scr = M3 + tid;                // row q of array k at (k r + q) slots
      double* s0 = lds_scr ? svp + tid : scr;
      double* s1 = lds_scr ? swp + tid : scr + (int64_t)r * slots;
      double* s2 = lds_scr ? spart[0] + tid : scr + (int64_t)2 * r * slots;
      double nr = 0.0;
      for (int q0 = 0; q0 < r; q0 += TRI_CH) {
        double xq[TRI_CH];
#pragma unroll
        for (int u = 0; u < TRI_CH; ++u) xq[u] = q0 + u < r ? x[q0 + u] : 0.0;
#pragma unroll
        for (int u = 0; u < TRI_CH; ++u)
          if (q0 + u < r) nr += xq[u] * xq[u];
      }
      nr = 1.0 / sqrt(nr);
      // the solve scales its right-hand side by nr as it reads it
      tri_solve(sd, se, r, slam[j], tiny, nr, x, s0, s1, s2, slots);
    }
    __syncthreads();
    if (sweep < 2) continue;
    // normalise every vector (one wave per vector)
    for (int j = wave; j < p; j += nw) {
      double* x = M1 + (int64_t)j * ld;
      double nr = 0.0;
      for (int q = lane; q < r; q += 64) nr += x[q] * x[q];
      nr = wave_allsum(nr);
      nr = 1.0 / sqrt(nr);
      for (int q = lane; q < r; q += 64) x[q] *= nr;
    }
    __syncthreads();
    // classical Gram-Schmidt, twice, inside every cluster of two or more
    for (int c = 0; c < s_nclus; ++c) {
      const int j0 = scl[c], j1 = scl[c + 1];
      for (int j = j0 + 1; j < j1; ++j) {
        double* x = M1 + (int64_t)j * ld;
        for (int pass = 0; pass < 2; ++pass) {
          for (int jj = j0 + wave; jj < j; jj += nw) {
            const double* y = M1 + (int64_t)jj * ld;
            double dp = 0.0;
            for (int q = lane; q < r; q += 64) dp += y[q] * x[q];
            dp = wave_allsum(dp);
            if (lane == 0) sw[jj - j0] = dp;
          }
          __syncthreads();
          for (int q = tid; q < r; q += nthr) {
            double v = x[q];
            for (int jj = j0; jj < j; ++jj) v -= sw[jj - j0] * M1[(int64_t)jj * ld + q];
            x[q] = v;
          }
          __syncthreads();
        }
        double nr = 0.0;
        for (int q = tid; q < r; q += nthr) nr += x[q] * x[q];
        nr = 1.0 / sqrt(wg_sum(nr, sred));
        for (int q = tid; q < r; q += nthr) x[q] *= nr;
        __syncthreads();
      }
    }
  }
  for (int64_t q = tid; q < (int64_t)(ld - r) * p; q += nthr) {
    const int row = r + (int)(q % (ld - r)), j = (int)(q / (ld - r));
    M1[(int64_t)j * ld + row] = 0.0;
  }
  __syncthreads();
  // back-transformation U = H_0 ... H_{r-3} Z.  The vectors are independent,
  // so each wave takes its own (j = wave, wave + nw, ...) through all the
  // reflectors without block barriers; a reflector (v(0) = 1, the rest stored
  // in column k of M0) is read straight from memory.  With r <= 256 a wave
  // holds BT_REG_V of its vectors in registers (lane l: rows l, l + 64, ...)
  // for a whole sweep over the reflectors; otherwise each reflector updates
  // them in memory, BT_VEC at a time.
  {
    constexpr int BT_REG_V = 4, BT_VEC = 4;
    if (r <= 256) {
      for (int jb = wave; jb < p; jb += nw * BT_REG_V) {
        const int nv = min(BT_REG_V, (p - jb + nw - 1) / nw);   // vectors jb + g nw, g < nv
        double z[BT_REG_V][4];
#pragma unroll
        for (int g = 0; g < BT_REG_V; ++g)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = lane + 64 * i;
            z[g][i] = 0.0;
            if (g < nv && q < r) z[g][i] = M1[(int64_t)(jb + g * nw) * ld + q];
          }
        // reflector k in v, the next one (k - 1) loading under the products
        auto load_v = [&](int k, double (&v)[4]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = lane + 64 * i;
            v[i] = q == k + 1 ? 1.0 : 0.0;
            if (q > k + 1 && q < r) v[i] = M0[(int64_t)k * ld + q];
          }
        };
        double v[4];
        if (r >= 3) load_v(r - 3, v);
        for (int k = r - 3; k >= 0; --k) {
          double vn[4] = {0.0, 0.0, 0.0, 0.0};
          if (k > 0) load_v(k - 1, vn);
          const double tk = stau[k];
          if (tk == 0.0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = vn[i];
            continue;
          }
          double sg[BT_REG_V];
#pragma unroll
          for (int g = 0; g < BT_REG_V; ++g) {
            sg[g] = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) sg[g] += v[i] * z[g][i];
          }
#pragma unroll
          for (int g = 0; g < BT_REG_V; ++g)
            sg[g] = wave_allsum(sg[g]);
#pragma unroll
          for (int g = 0; g < BT_REG_V; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) z[g][i] -= tk * sg[g] * v[i];
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = vn[i];
        }
#pragma unroll
        for (int g = 0; g < BT_REG_V; ++g)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = lane + 64 * i;
            if (g < nv && q < r) M1[(int64_t)(jb + g * nw) * ld + q] = z[g][i];
          }
      }
    } else {
      for (int jb = wave; jb < p; jb += nw * BT_VEC) {
        const int ng = min(BT_VEC, (p - jb + nw - 1) / nw);   // vectors jb + g nw, g < ng
        double* x0 = M1 + (int64_t)jb * ld;
        const int64_t js = (int64_t)nw * ld;
        for (int k = r - 3; k >= 0; --k) {
          const double tk = stau[k];
          if (tk == 0.0) continue;
          const int m = r - k - 1;
          const double* vk = M0 + (int64_t)k * ld + k + 1;
          double* xk = x0 + k + 1;
          double sg[BT_VEC];
#pragma unroll
          for (int g = 0; g < BT_VEC; ++g) sg[g] = 0.0;
#pragma unroll 1
          for (int a = lane; a < m; a += 64) {
            const double va = a == 0 ? 1.0 : vk[a];
#pragma unroll
            for (int g = 0; g < BT_VEC; ++g)
              if (g < ng) sg[g] += va * xk[g * js + a];
          }
#pragma unroll
          for (int g = 0; g < BT_VEC; ++g)
            sg[g] = wave_allsum(sg[g]);
#pragma unroll 1
          for (int a = lane; a < m; a += 64) {
            const double va = a == 0 ? 1.0 : vk[a];
#pragma unroll
            for (int g = 0; g < BT_VEC; ++g)
              if (g < ng) xk[g * js + a] -= tk * sg[g] * va;
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- 6. Y = W U into M0 (n x p, padding rows zero), sigma
  // (general case: row sperm[a] of Y is D2 (R11^{-1} U)(a, :) for a < r, else 0)
  for (int64_t q = tid; q < (int64_t)ld * p; q += nthr) {
    const int a = (int)(q % ld), c = (int)(q / ld);
    double s = 0.0;
    int row = a;
    if (s_diag) {
      if (a < n) s = sD2[a] * M1[(int64_t)c * ld + a];
    } else if (a < n) {
      row = sperm[a];
      if (a < r) {
        for (int b = a; b < r; ++b) s += M2[(int64_t)a * ld + b] * M1[(int64_t)c * ld + b];
        s *= sD2[row];
      }
    }
    M0[(int64_t)c * ld + row] = s;
  }
  for (int c = tid; c < p; c += nthr) sig_out[dsc.loc_off + c] = sqrt(slam[c]);
  if (tid == 0) p_out[i] = p;
}

void launch_select(hipStream_t st, int nsub, const DevPlan& P, const double* ctg, const double* Tg,
                   double* work, double tau, int nev_max, int32_t* p_out, double* sig_out,
                   int qr_range) {
  // size classes of the interface: up to 128, 512 and SEL_MAXN columns (the
  // last also reports larger ones); a class is launched only when some
  // interface size may fall in it, so that idle workgroups of the larger
  // classes do not wait for CUs held by kernels on the other stream
  if (P.min_nG <= 128)
    k_select<256, 0, 128><<<nsub, 256, 0, st>>>(P.heavy(), ctg, Tg, work, tau, nev_max, p_out,
                                                sig_out, p_out + nsub, qr_range);
  if (P.max_nG > 128 && P.min_nG <= 512)
    k_select<512, 128, 512><<<nsub, 512, 0, st>>>(P.heavy(), ctg, Tg, work, tau, nev_max, p_out,
                                                  sig_out, p_out + nsub, qr_range);
  if (P.max_nG > 512)
    k_select<SEL_THREADS, 512, SEL_MAXN><<<nsub, SEL_THREADS, 0, st>>>(
        P.heavy(), ctg, Tg, work, tau, nev_max, p_out, sig_out, p_out + nsub, qr_range);
}

}  // namespace lsq2l
