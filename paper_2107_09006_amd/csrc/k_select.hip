// Coarse-space selection per subdomain (Lemma 2.4 / eq. gevp, reduced to the
// interface pencil; see k_coarse.hip for the reduction).
//
// With T = L_GI L_GI^T and Ct = Ct_GG (both diagonally scaled by the
// equilibration of C_ii), the selected directions are the eigenvectors of
//     K = W^T T W,   W^T Ct W = I,  range(W) = range(Ct),
// with eigenvalue sigma^2 > 1 - tau.  One workgroup per subdomain:
//   1. W: if Ct is diagonal, W = diag(Ct)^{-1/2}; otherwise a pivoted
//      Cholesky Ct = R^T R (rank r: stop when the largest remaining diagonal
//      of the unit-diagonal scaled matrix falls below n eps) and
//      W = R^T (R R^T)^{-1};
//   2. K = W^T (T W) with MFMA tile products;
//   3. Householder tridiagonalization of K;
//   4. p = number of eigenvalues above 1 - tau (one Sturm count), then the
//      p largest eigenvalues by bisection (one thread each);
//   5. eigenvectors of the tridiagonal matrix by inverse iteration (one thread
//      per cluster of close eigenvalues, re-orthogonalised inside the cluster)
//      and back-transformation through the Householder reflectors;
//   6. Y = W U (interface coefficients of the selected vectors), sigma.
// Work matrices (ld = nGp, four per subdomain at 4 g_off): M0 scaled Ct, then
// K and the Householder vectors, then Y; M1 R^T, then U; M2 the Cholesky
// factor of R R^T, then W; M3 scratch, T W, then scratch of the inverse
// iteration (3 r doubles per cluster).
#include "kernels.hpp"

namespace lsq2l {

constexpr int SEL_THREADS = 1024;
constexpr int SEL_MAXN = 1024;
constexpr double SEL_EPS = 2.220446049250313e-16;

// ----------------------------------------------------------------------------
// block-wide reductions (shuffles inside a wave, one LDS round across waves)
// ----------------------------------------------------------------------------
__device__ inline double wg_sum(double v, double* red) {
  for (int w = 32; w > 0; w >>= 1) v += __shfl_down(v, w, 64);
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

// C (M x N) = op(A) B with M, N, Kd multiples of 16 (zero padded operands),
// all column-major with leading dimension ld; one 16 x 16 quadrant of the
// output per wave at a time.
// Only the first Kv entries of the contraction are read (the rest count as 0).
template <bool TA>
__device__ void wg_gemm(double* C, const double* A, const double* B, int M, int N, int Kd, int Kv,
                        int ld) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
  const int li = lane % 16, lk = lane / 16;
  const int mq = M / 16, nq = N / 16;
  for (int q = wave; q < mq * nq; q += nw) {
    const int qi = q % mq, qj = q / mq;
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < Kd; k0 += 4) {
      const int k = k0 + lk;
      double a = 0.0, b = 0.0;
      if (k < Kv) {
        a = TA ? A[(int64_t)(16 * qi + li) * ld + k] : A[(int64_t)k * ld + 16 * qi + li];
        b = B[(int64_t)(16 * qj + li) * ld + k];
      }
      acc = Mfma<double>::mma(a, b, acc);
    }
    for (int v = 0; v < 4; ++v)
      C[(int64_t)(16 * qj + Mfma<double>::acc_col(lane, v)) * ld + 16 * qi + Mfma<double>::acc_row(lane, v)] = acc[v];
  }
}

// ----------------------------------------------------------------------------
// tridiagonal helpers (single thread)
// ----------------------------------------------------------------------------
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

// Solve (T - lam I) x = b (b overwritten by x) with Gaussian elimination and
// row interchanges; a, up, u2 are scratch of length n.
__device__ void tri_solve(const double* d, const double* e, int n, double lam, double tiny, double* b,
                          double* a, double* up, double* u2) {
  for (int i = 0; i < n; ++i) { a[i] = d[i] - lam; u2[i] = 0.0; }
  for (int i = 0; i + 1 < n; ++i) up[i] = e[i];
  for (int i = 0; i + 1 < n; ++i) {
    const double lo = e[i];
    if (fabs(a[i]) >= fabs(lo)) {
      if (a[i] == 0.0) a[i] = tiny;
      const double mlt = lo / a[i];
      a[i + 1] -= mlt * up[i];
      b[i + 1] -= mlt * b[i];
    } else {
      const double mlt = a[i] / lo;
      a[i] = lo;
      const double t = a[i + 1];
      a[i + 1] = up[i] - mlt * t;
      if (i + 2 < n) { u2[i] = up[i + 1]; up[i + 1] = -mlt * u2[i]; }
      up[i] = t;
      const double bi = b[i];
      b[i] = b[i + 1];
      b[i + 1] = bi - mlt * b[i + 1];
    }
  }
  if (a[n - 1] == 0.0) a[n - 1] = tiny;
  b[n - 1] = b[n - 1] / a[n - 1];
  if (n >= 2) b[n - 2] = (b[n - 2] - up[n - 2] * b[n - 1]) / a[n - 2];
  for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - up[i] * b[i + 1] - u2[i] * b[i + 2]) / a[i];
}

// ----------------------------------------------------------------------------
// the selection kernel
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(SEL_THREADS)
k_select(const SubDesc* __restrict__ subs, const double* __restrict__ ctg,
         const double* __restrict__ Tg, double* __restrict__ work, double tau, int nev_max,
         int32_t* __restrict__ p_out, double* __restrict__ sig_out, int32_t* __restrict__ fail) {
  __shared__ double sd[SEL_MAXN], se[SEL_MAXN], stau[SEL_MAXN], sv[SEL_MAXN], sw[SEL_MAXN],
      sD2[SEL_MAXN], slam[SEL_MAXN];
  __shared__ int sperm[SEL_MAXN], scl[SEL_MAXN + 1];
  __shared__ double sred[16];
  __shared__ int sredi[16];
  __shared__ int s_r, s_p, s_nclus, s_diag;
  __shared__ double s_anorm;
  const int i = blockIdx.x;
  const SubDesc dsc = subs[i];
  const int n = dsc.nG, ld = dsc.nGp, tid = threadIdx.x, nthr = blockDim.x;
  if (n == 0 || n > SEL_MAXN) {
    if (tid == 0) { p_out[i] = 0; if (n > SEL_MAXN) atomicExch(fail, 2); }
    return;
  }
  const int64_t mm = (int64_t)ld * ld;
  double* M0 = work + 4 * dsc.g_off;
  double* M1 = M0 + mm;
  double* M2 = M1 + mm;
  double* M3 = M2 + mm;
  const double* Ct = ctg + dsc.g_off;
  const double* T = Tg + dsc.g_off;

  // ---- 1. scaled Ct (unit diagonal) and the range basis W
  // a zero diagonal (stored zeros only) leaves its column out of range(Ct)
  int nz = 0;
  for (int a = tid; a < n; a += nthr) {
    const double c = Ct[(int64_t)a * ld + a];
    sD2[a] = c > 0.0 ? 1.0 / sqrt(c) : 0.0;
    nz += !(c > 0.0);
  }
  __syncthreads();
  double off = (double)nz;
  for (int64_t q = tid; q < mm; q += nthr) {
    const int r = (int)(q % ld), c = (int)(q / ld);
    double v = 0.0;
    if (r < n && c < n) {
      v = (r >= c) ? Ct[(int64_t)c * ld + r] : Ct[(int64_t)r * ld + c];
      v *= sD2[r] * sD2[c];
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
    // pivoted Cholesky of M0 (in place, original indexing); R^T kept in M1
    for (int a = tid; a < n; a += nthr) sperm[a] = a;
    for (int64_t q = tid; q < mm; q += nthr) M1[q] = 0.0;
    __syncthreads();
    const double tol = n * SEL_EPS;     // the scaled matrix has unit diagonal
    int k = 0;
    for (; k < n; ++k) {
      double bv = -1.0;
      int bi = n;
      for (int j = k + tid; j < n; j += nthr) {
        const int pj = sperm[j];
        const double v = M0[(int64_t)pj * ld + pj];
        if (v > bv || (v == bv && j < bi)) { bv = v; bi = j; }
      }
      double mv;
      int mj;
      wg_argmax(bv, bi, sred, sredi, &mv, &mj);
      if (!(mv > tol)) break;
      __syncthreads();
      if (tid == 0) { const int t = sperm[k]; sperm[k] = sperm[mj]; sperm[mj] = t; }
      __syncthreads();
      const int pk = sperm[k];
      const double s = sqrt(M0[(int64_t)pk * ld + pk]);
      for (int j = k + tid; j < n; j += nthr) {
        const int pj = sperm[j];
        M1[(int64_t)k * ld + pj] = (j == k) ? s : M0[(int64_t)pj * ld + pk] / s;
      }
      __syncthreads();
      const int rem = n - k - 1;
      for (int64_t q = tid; q < (int64_t)rem * rem; q += nthr) {
        const int pa = sperm[k + 1 + (int)(q % rem)], pb = sperm[k + 1 + (int)(q / rem)];
        M0[(int64_t)pb * ld + pa] -= M1[(int64_t)k * ld + pa] * M1[(int64_t)k * ld + pb];
      }
      __syncthreads();
    }
    r = k;
    if (r == 0) {
      if (tid == 0) p_out[i] = 0;
      return;
    }
    const int rp = (r + 15) / 16 * 16, np16 = (n + 15) / 16 * 16;
    // G = R R^T (r x r) in M2, its Cholesky in place
    wg_gemm<true>(M2, M1, M1, rp, rp, np16, n, ld);
    __syncthreads();
    for (int kk = 0; kk < r; ++kk) {
      const double dk = M2[(int64_t)kk * ld + kk];
      const double sk = sqrt(dk);
      __syncthreads();
      for (int a = kk + 1 + tid; a < r; a += nthr) M2[(int64_t)kk * ld + a] /= sk;
      if (tid == 0) M2[(int64_t)kk * ld + kk] = sk;
      __syncthreads();
      const int rem = r - kk - 1;
      for (int64_t q = tid; q < (int64_t)rem * rem; q += nthr) {
        const int a = kk + 1 + (int)(q % rem), b = kk + 1 + (int)(q / rem);
        if (b <= a) M2[(int64_t)b * ld + a] -= M2[(int64_t)kk * ld + a] * M2[(int64_t)kk * ld + b];
      }
      __syncthreads();
    }
    // W rows: w G = (R^T row) -> forward with Lg then backward with Lg^T;
    // W stored in M3 (n x r) temporarily, then D2-scaled into M2's place below
    for (int a = tid; a < n; a += nthr) {
      double* w = M3 + a;                       // row a of W, stride ld
      for (int c = 0; c < r; ++c) {             // forward: Lg y = rt
        double s = M1[(int64_t)c * ld + a];
        for (int b = 0; b < c; ++b) s -= M2[(int64_t)b * ld + c] * w[(int64_t)b * ld];
        w[(int64_t)c * ld] = s / M2[(int64_t)c * ld + c];
      }
      for (int c = r - 1; c >= 0; --c) {        // backward: Lg^T w = y
        double s = w[(int64_t)c * ld];
        for (int b = c + 1; b < r; ++b) s -= M2[(int64_t)c * ld + b] * w[(int64_t)b * ld];
        w[(int64_t)c * ld] = s / M2[(int64_t)c * ld + c];
      }
    }
    __syncthreads();
    // M2 = D2 W (n x r, zero padded)
    for (int64_t q = tid; q < mm; q += nthr) {
      const int a = (int)(q % ld), c = (int)(q / ld);
      M2[q] = (a < n && c < r) ? sD2[a] * M3[q] : 0.0;
    }
    __syncthreads();
    // K = W^T (T W): M3 = T M2, M0 = M2^T M3
    wg_gemm<false>(M3, T, M2, np16, rp, np16, n, ld);
    __syncthreads();
    wg_gemm<true>(M0, M2, M3, rp, rp, np16, n, ld);
    __syncthreads();
    for (int64_t q = tid; q < (int64_t)r * r; q += nthr) {     // symmetrise
      const int a = (int)(q % r), c = (int)(q / r);
      if (a > c) {
        const double v = 0.5 * (M0[(int64_t)c * ld + a] + M0[(int64_t)a * ld + c]);
        M0[(int64_t)c * ld + a] = v;
        M0[(int64_t)a * ld + c] = v;
      }
    }
    __syncthreads();
  }

  // ---- 3. tridiagonalization of K (r x r) in M0
  for (int k = 0; k + 2 < r; ++k) {
    const int m = r - k - 1;
    double part = 0.0;
    for (int a = 1 + tid; a < m; a += nthr) { const double t = M0[(int64_t)k * ld + k + 1 + a]; part += t * t; }
    const double xn2 = wg_sum(part, sred);
    const double alpha = M0[(int64_t)k * ld + k + 1];
    double tk = 0.0, beta = alpha;
    if (xn2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tk = (beta - alpha) / beta;
      const double sc = 1.0 / (alpha - beta);
      for (int a = tid; a < m; a += nthr) sv[a] = (a == 0) ? 1.0 : M0[(int64_t)k * ld + k + 1 + a] * sc;
    } else {
      for (int a = tid; a < m; a += nthr) sv[a] = (a == 0) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) { se[k] = beta; sd[k] = M0[(int64_t)k * ld + k]; stau[k] = tk; }
    for (int a = 1 + tid; a < m; a += nthr) M0[(int64_t)k * ld + k + 1 + a] = sv[a];
    if (tk != 0.0) {
      double pp = 0.0;
      for (int a = tid; a < m; a += nthr) {
        double s = 0.0;
        for (int b = 0; b < m; ++b) s += M0[(int64_t)(k + 1 + b) * ld + k + 1 + a] * sv[b];
        sw[a] = tk * s;
        pp += sw[a] * sv[a];
      }
      const double wv = wg_sum(pp, sred);
      const double a2 = -0.5 * tk * wv;
      for (int a = tid; a < m; a += nthr) sw[a] += a2 * sv[a];
      __syncthreads();
      for (int64_t q = tid; q < (int64_t)m * m; q += nthr) {
        const int a = (int)(q % m), b = (int)(q / m);
        M0[(int64_t)(k + 1 + b) * ld + k + 1 + a] -= sv[a] * sw[b] + sw[a] * sv[b];
      }
    }
    __syncthreads();
  }
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

  // ---- 4. count above 1 - tau, bisection for the p largest eigenvalues.  A
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
  // the j-th largest is the (r-1-j)-th smallest; all p lie above thr
  for (int j = tid; j < p; j += nthr) {
    const int kidx = r - 1 - j;
    double lo = thr, hi = anorm * (1.0 + 4.0 * SEL_EPS) + pivmin;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (hi - lo <= 2.0 * SEL_EPS * fmax(fabs(lo), fabs(hi)) + pivmin) break;
      if (sturm_below(sd, se, r, mid, pivmin) > kidx) hi = mid; else lo = mid;
    }
    slam[j] = 0.5 * (lo + hi);
  }
  __syncthreads();
  // clusters of close eigenvalues (descending order); separate equal ones
  if (tid == 0) {
    const double ortol = 1e-3 * anorm, sep = 10.0 * SEL_EPS * anorm;
    int nc = 0;
    for (int j = 0; j < p; ++j) {
      if (j > 0 && fabs(slam[j - 1] - slam[j]) < sep) slam[j] = slam[j - 1] - sep;
      if (j == 0 || slam[j - 1] - slam[j] > ortol) scl[nc++] = j;
    }
    scl[nc] = p;
    s_nclus = nc;
  }
  __syncthreads();

  // ---- 5. shifted block inverse iteration: every sweep solves all p systems
  // in parallel (one thread per vector, scratch of 3 r doubles in M3, free
  // now), then one wave per cluster re-orthonormalises that cluster
  // (Gram-Schmidt, two passes).  Vectors in M1 (r x p).
  const double tiny = SEL_EPS * anorm;
  const int slots = (int)min<int64_t>(mm / (3 * r), nthr);
  const int wave = tid / 64, lane = tid % 64, nw = nthr / 64;
  for (int64_t q = tid; q < (int64_t)ld * p; q += nthr) {
    const int row = (int)(q % ld), j = (int)(q / ld);
    M1[q] = row < r ? sin((row + 1.0) * (j + 1.0)) : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 5; ++sweep) {
    for (int j0 = 0; j0 < p; j0 += slots) {
      const int j = j0 + tid;
      if (tid >= slots || j >= p) continue;
      double* x = M1 + (int64_t)j * ld;
      double* scr = M3 + (int64_t)tid * 3 * r;
      double nr = 0.0;
      for (int q = 0; q < r; ++q) nr += x[q] * x[q];
      nr = 1.0 / sqrt(nr);
      for (int q = 0; q < r; ++q) x[q] *= nr;
      tri_solve(sd, se, r, slam[j], tiny, x, scr, scr + r, scr + 2 * r);
    }
    __syncthreads();
    for (int c = wave; c < s_nclus; c += nw) {
      for (int j = scl[c]; j < scl[c + 1]; ++j) {
        double* x = M1 + (int64_t)j * ld;
        for (int pass = 0; pass < 2; ++pass)
          for (int jj = scl[c]; jj < j; ++jj) {
            const double* y = M1 + (int64_t)jj * ld;
            double dp = 0.0;
            for (int q = lane; q < r; q += 64) dp += y[q] * x[q];
            for (int w = 32; w > 0; w >>= 1) dp += __shfl_xor(dp, w, 64);
            for (int q = lane; q < r; q += 64) x[q] -= dp * y[q];
          }
        double nr = 0.0;
        for (int q = lane; q < r; q += 64) nr += x[q] * x[q];
        for (int w = 32; w > 0; w >>= 1) nr += __shfl_xor(nr, w, 64);
        nr = 1.0 / sqrt(nr);
        for (int q = lane; q < r; q += 64) x[q] *= nr;
      }
    }
    __syncthreads();
  }
  // back-transformation U = H_0 ... H_{r-3} Z
  for (int k = r - 3; k >= 0; --k) {
    const double tk = stau[k];
    if (tk == 0.0) continue;
    const int m = r - k - 1;
    for (int a = tid; a < m; a += nthr) sv[a] = (a == 0) ? 1.0 : M0[(int64_t)k * ld + k + 1 + a];
    __syncthreads();
    for (int j = wave; j < p; j += nw) {
      double* x = M1 + (int64_t)j * ld + k + 1;
      double s = 0.0;
      for (int a = lane; a < m; a += 64) s += sv[a] * x[a];
      for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w, 64);
      for (int a = lane; a < m; a += 64) x[a] -= tk * s * sv[a];
    }
    __syncthreads();
  }

  // ---- 6. Y = W U into M0 (n x p, padding rows zero), sigma
  for (int64_t q = tid; q < (int64_t)ld * p; q += nthr) {
    const int a = (int)(q % ld), c = (int)(q / ld);
    double s = 0.0;
    if (a < n) {
      if (s_diag) s = sD2[a] * M1[(int64_t)c * ld + a];
      else for (int b = 0; b < r; ++b) s += M2[(int64_t)b * ld + a] * M1[(int64_t)c * ld + b];
    }
    M0[(int64_t)c * ld + a] = s;
  }
  for (int c = tid; c < p; c += nthr) sig_out[dsc.loc_off + c] = sqrt(slam[c]);
  if (tid == 0) p_out[i] = p;
}

void launch_select(hipStream_t st, int nsub, const DevPlan& P, const double* ctg, const double* Tg,
                   double* work, double tau, int nev_max, int32_t* p_out, double* sig_out) {
  k_select<<<nsub, SEL_THREADS, 0, st>>>(P.subs, ctg, Tg, work, tau, nev_max, p_out, sig_out,
                                         p_out + nsub);
}

}  // namespace lsq2l
