// Coarse space and coarse solve (Lemma 2.4, eq. gevp, Algorithm 1).
//
// Selection.  With the 0/1 partition of unity D_i of Section 3.3.1 and the
// splitting of eq. (spsd_normal_eq), a vector v = (x, y) of eq. (gevp),
// D C D v = lambda Ct v, has lambda = 0 when x = 0; for x != 0 the interface
// part can be eliminated, which leaves the interior pencil
//     S x = mu C_I x,  S = C_I - Ct_IG Ct_GG^+ Ct_GI,  mu = 1 / lambda,
// so lambda > 1/tau is mu < tau.  Its nonzero spectrum is that of the small
// interface pencil (size n_Gamma instead of n_I)
//     T y = sigma^2 Ct_GG y  on range(Ct_GG),  T = Ct_GI C_I^{-1} Ct_IG,
// with sigma^2 = 1 - mu, and the interior vectors are x = C_I^{-1} Ct_IG y.
// Because Ct_IG = C_IG, L_GI^T = L_I^{-1} C_IG in the Cholesky factor of
// C_ii, so T = L_GI L_GI^T comes straight from the local factor.
// Selected: sigma^2 > 1 - tau.  X_i = L_I^{-T} L_GI^T Y diag(1/sigma) is
// C_I-orthonormal (X^T C_I X = diag(sigma)^-1 Y^T T Y diag(sigma)^-1 = I).
//
// Coarse operator.  W = A R_0^T has block i = A(Xi_i, Omega_Ii) X_i; the
// Galerkin matrix E = W^T W (Algorithm 1, C_00 = (A R_0^T)^T (A R_0^T)) has a
// block for every pair of subdomains that share rows.  E is factored in the
// same tile-envelope layout as the local matrices and its dense inverse is
// formed for the per-iteration coarse solve.
#include "kernels.hpp"

namespace lsq2l {

// ---------------------------------------------------------------------------
// tile helpers for multi-right-hand-side products (one 16 x 16 quadrant per wave)
// ---------------------------------------------------------------------------
// acc += op(A) * B for the quadrant (bi, bj); op(A) = A or A^T; A, B are
// 32 x 32 column-major with leading dimensions lda, ldb.  The operand
// fragments of a whole 32-deep product are loaded first (16 independent
// loads), then the 8 MFMAs run.
struct QuadFrag { double a[8], b[8]; };

template <bool TA>
__device__ inline void quad_frag_load(QuadFrag& f, const double* A, int lda, const double* B, int ldb,
                                      int bi, int bj, int lane) {
  const int li = lane % 16, lk = lane / 16;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int k = 4 * q + lk;
    f.a[q] = TA ? A[(int64_t)(16 * bi + li) * lda + k] : A[(int64_t)k * lda + 16 * bi + li];
    f.b[q] = B[(int64_t)(16 * bj + li) * ldb + k];
  }
}

__device__ inline void quad_frag_mma(double4_t& acc, const QuadFrag& f, bool neg) {
#pragma unroll
  for (int q = 0; q < 8; ++q) acc = Mfma<double>::mma(neg ? -f.a[q] : f.a[q], f.b[q], acc);
}

template <bool TA>
__device__ inline void quad_mma(double4_t& acc, const double* A, int lda, const double* B, int ldb,
                                int bi, int bj, int lane, bool neg) {
  QuadFrag f;
  quad_frag_load<TA>(f, A, lda, B, ldb, bi, bj, lane);
  quad_frag_mma(acc, f, neg);
}

// the A fragments of quad_mma<false> (rows 16 bi .. 16 bi + 15 of A), for a
// product issued later with quad_mma_pre
__device__ inline void quad_afrag(double (&a)[8], const double* A, int lda, int bi, int lane) {
  const int li = lane % 16, lk = lane / 16;
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = A[(int64_t)(4 * q + lk) * lda + 16 * bi + li];
}

__device__ inline void quad_mma_pre(double4_t& acc, const double (&a)[8], const double* B, int ldb,
                                    int bj, int lane) {
  const int li = lane % 16, lk = lane / 16;
  double b[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) b[q] = B[(int64_t)(16 * bj + li) * ldb + 4 * q + lk];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc = Mfma<double>::mma(a[q], b[q], acc);
}

__device__ inline void quad_load(double4_t& acc, const double* C, int ldc, int bi, int bj, int lane) {
  for (int v = 0; v < 4; ++v)
    acc[v] = C[(int64_t)(16 * bj + Mfma<double>::acc_col(lane, v)) * ldc + 16 * bi +
               Mfma<double>::acc_row(lane, v)];
}

__device__ inline void quad_store(const double4_t& acc, double* C, int ldc, int bi, int bj, int lane) {
  for (int v = 0; v < 4; ++v)
    C[(int64_t)(16 * bj + Mfma<double>::acc_col(lane, v)) * ldc + 16 * bi +
      Mfma<double>::acc_row(lane, v)] = acc[v];
}

// ---------------------------------------------------------------------------
// T = L_GI L_GI^T (interface x interface, full symmetric, ld nGp)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_gamma_T(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
          const int64_t* __restrict__ tileOff, const double* __restrict__ fac,
          double* __restrict__ Tg) {
  const SubDesc d = subs[blockIdx.x];
  if (d.nG == 0) return;
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  const double* A = fac + d.fac_off;
  double* T = Tg + d.g_off;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
  const int ng = d.ntiles - d.ntI;
  int item = 0;
  for (int a = 0; a < ng; ++a)
    for (int b = 0; b <= a; ++b, ++item) {
      if (item % nwaves != wave) continue;
      const int Ia = d.ntI + a, Ib = d.ntI + b;
      double4_t acc[4];
      tile_acc_zero<double>(acc);
      const int K0 = max(F[Ia], F[Ib]);
      for (int K = K0; K < d.ntI; ++K)
        tile_mma_nt<double, false>(acc, A + tile_pos(F, off, Ia, K) * TT, TS,
                                   A + tile_pos(F, off, Ib, K) * TT, TS, lane);
      tile_acc_store<double>(acc, T + (int64_t)(b * TS) * d.nGp + a * TS, d.nGp, lane);
      if (a != b) {
        // transpose block
        for (int q = 0; q < 4; ++q)
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * (q / 2) + Mfma<double>::acc_row(lane, v);
            const int c = 16 * (q % 2) + Mfma<double>::acc_col(lane, v);
            T[(int64_t)(a * TS + r) * d.nGp + b * TS + c] = acc[q][v];
          }
      }
    }
}

// acc (32 x 32, acc[bi * 2 + bj] as in tile_acc_load) += op(A) B with K = 32;
// op(A) = A or A^T of a 32 x 32 column-major tile, B column-major (ldb) with
// its columns >= nb read as zero.
template <bool TA>
__device__ inline void tile_mma_cols(double4_t acc[4], const double* A, int lda, const double* B,
                                     int ldb, int nb, int lane, bool neg) {
  const int li = lane % 16, lk = lane / 16;
  // all operand fragments of the 32-deep product load first (32 independent
  // loads per lane), then the 32 MFMAs run
  double a0[8], a1[8], b0[8], b1[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int k = 4 * q + lk;
    a0[q] = TA ? A[(int64_t)li * lda + k] : A[(int64_t)k * lda + li];
    a1[q] = TA ? A[(int64_t)(16 + li) * lda + k] : A[(int64_t)k * lda + 16 + li];
    b0[q] = li < nb ? B[(int64_t)li * ldb + k] : 0.0;
    b1[q] = 16 + li < nb ? B[(int64_t)(16 + li) * ldb + k] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double x0 = neg ? -a0[q] : a0[q], x1 = neg ? -a1[q] : a1[q];
    acc[0] = Mfma<double>::mma(x0, b0[q], acc[0]);
    acc[1] = Mfma<double>::mma(x0, b1[q], acc[1]);
    acc[2] = Mfma<double>::mma(x1, b0[q], acc[2]);
    acc[3] = Mfma<double>::mma(x1, b1[q], acc[3]);
  }
}

__device__ inline void tile_io_cols(double4_t acc[4], double* C, int ldc, int nb, int lane, bool store) {
#pragma unroll
  for (int qd = 0; qd < 4; ++qd)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * (qd / 2) + Mfma<double>::acc_row(lane, v);
      const int c = 16 * (qd % 2) + Mfma<double>::acc_col(lane, v);
      if (c >= nb) { if (!store) acc[qd][v] = 0.0; continue; }
      if (store) C[(int64_t)c * ldc + r] = acc[qd][v];
      else acc[qd][v] = C[(int64_t)c * ldc + r];
    }
}

constexpr int XS_MAXROWS = 8192, XS_MAXP = 1024;   // LDS copies of S_I and sigma (p <= 1024 always)
// the backward substitution keeps F, the tile offsets and the last envelope
// row of every interior tile column in LDS (aliasing the copies of S_I)
constexpr int XS_TMAX = XS_MAXROWS * 2 / 3;
// X_i = S_I L_I^{-T} (L_GI^T Y) diag(1/sigma), written as nIp x p (column-major).
// H = L_GI^T Y by 32 x 32 output blocks (one per wave task), then the
// backward substitution with L_I^T by tile rows (left-looking, a wave per
// block of columns), all on MFMA.
__global__ void __launch_bounds__(512)
k_coarse_X(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
           const int64_t* __restrict__ tileOff, const double* __restrict__ fac,
           const double* __restrict__ dinv, const double* __restrict__ scale,
           const double* __restrict__ work, const double* __restrict__ sig, double* __restrict__ X) {
  __shared__ double sXs[XS_MAXROWS], sXg[XS_MAXP];
  const SubDesc d = subs[blockIdx.x];
  if (d.p == 0) return;
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  const double* A = fac + d.fac_off;
  const double* Di = dinv + d.dinv_off;
  const double* Y = work + SEL_WORK_MATS * d.g_off;   // nGp x p, ld nGp
  double* H = X + d.x_off;                 // nIp x p, ld nIp
  const int p = d.p, ldh = d.nIp, ldy = d.nGp, tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid / 64, lane = tid % 64, nw = nthr / 64;
  const int npb = (p + TS - 1) / TS;
  // H_J = sum over interface tile rows I with F(I) <= J of L(I,J)^T Y_I: a
  // wave task is tile row J of up to XG column blocks, so that each tile of
  // L is loaded once for all of them
  constexpr int XG = 4;
  const int ngrp = (npb + XG - 1) / XG;
  for (int t = wave; t < d.ntI * ngrp; t += nw) {
    const int J = t % d.ntI, g0 = (t / d.ntI) * XG;
    const int ng = min(XG, npb - g0);
    double4_t acc[XG][4];
#pragma unroll
    for (int g = 0; g < XG; ++g) tile_acc_zero<double>(acc[g]);
    const int li = lane % 16, lk = lane / 16;
    for (int I = d.ntI; I < d.ntiles; ++I) {
      if (F[I] > J) continue;
      const double* At = A + tile_pos(F, off, I, J) * TT;
      double a0[8], a1[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = 4 * q + lk;
        a0[q] = At[li * TS + k];
        a1[q] = At[(16 + li) * TS + k];
      }
#pragma unroll
      for (int g = 0; g < XG; ++g) {
        if (g >= ng) break;
        const int nb = min(TS, p - TS * (g0 + g));
        const double* Bt = Y + (int64_t)(TS * (g0 + g)) * ldy + (I - d.ntI) * TS;
        double b0[8], b1[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = 4 * q + lk;
          b0[q] = li < nb ? Bt[(int64_t)li * ldy + k] : 0.0;
          b1[q] = 16 + li < nb ? Bt[(int64_t)(16 + li) * ldy + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          acc[g][0] = Mfma<double>::mma(a0[q], b0[q], acc[g][0]);
          acc[g][1] = Mfma<double>::mma(a0[q], b1[q], acc[g][1]);
          acc[g][2] = Mfma<double>::mma(a1[q], b0[q], acc[g][2]);
          acc[g][3] = Mfma<double>::mma(a1[q], b1[q], acc[g][3]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < XG; ++g) {
      if (g >= ng) break;
      const int nb = min(TS, p - TS * (g0 + g));
      tile_io_cols(acc[g], H + (int64_t)(TS * (g0 + g)) * ldh + J * TS, ldh, nb, lane, true);
    }
  }
  __syncthreads();
  // envelope of the interior in LDS: F, the tile offsets and, per tile
  // column I, the last interior tile row K with F(K) <= I (the backward
  // substitution then visits only the rows that can hold a tile of column I)
  int32_t* sF = reinterpret_cast<int32_t*>(sXs);
  int32_t* sOff = sF + XS_TMAX;
  int32_t* sLast = sOff + XS_TMAX;
  const bool staged = d.ntI <= XS_TMAX;
  if (staged) {
    for (int K = tid; K < d.ntI; K += nthr) {
      sF[K] = F[K];
      sOff[K] = (int32_t)off[K];
      sLast[K] = K;
    }
    __syncthreads();
    for (int K = tid; K < d.ntI; K += nthr)
      for (int I = sF[K]; I < K; ++I) atomicMax(&sLast[I], K);
    __syncthreads();
  }
  // backward substitution with L_I^T, left-looking, one wave per block of 32
  // columns with no block barriers: for I from the last tile row down,
  // X_I = Dinv_I^T (H_I - sum over K > I with F(K) <= I of L(K,I)^T X_K)
  for (int pb = wave; pb < npb; pb += nw) {
    const int nb = min(TS, p - TS * pb);
    double* Hp = H + (int64_t)(TS * pb) * ldh;
    for (int I = d.ntI - 1; I >= 0; --I) {
      double4_t acc[4];
      tile_io_cols(acc, Hp + I * TS, ldh, nb, lane, false);
      const int kend = staged ? sLast[I] : d.ntI - 1;
      for (int K = I + 1; K <= kend; ++K) {
        const int fk = staged ? sF[K] : F[K];
        if (fk <= I) {
          const int64_t t = staged ? (int64_t)sOff[K] + (I - fk) : tile_pos(F, off, K, I);
          tile_mma_cols<true>(acc, A + t * TT, TS, Hp + K * TS, ldh, nb, lane, true);
        }
      }
      tile_io_cols(acc, Hp + I * TS, ldh, nb, lane, true);
      wg_fence();
      tile_acc_zero<double>(acc);
      tile_mma_cols<true>(acc, Di + (int64_t)I * TT, TS, Hp + I * TS, ldh, nb, lane, false);
      wg_fence();
      tile_io_cols(acc, Hp + I * TS, ldh, nb, lane, true);
      wg_fence();
    }
  }
  __syncthreads();
  // scale rows by S_I and columns by 1/sigma; zero the padding rows.  S_I
  // and sigma from LDS, pairs of entries as 16-byte accesses, eight in
  // flight per thread
  const double* s_loc = scale + d.loc_off;
  if (ldh > XS_MAXROWS) {                  // larger interiors: straight from memory
    for (int64_t q = tid; q < (int64_t)ldh * p; q += nthr) {
      const int a = (int)(q % ldh), k = (int)(q / ldh);
      H[q] = (a < d.nI) ? H[q] * s_loc[a] / sig[d.loc_off + k] : 0.0;
    }
    return;
  }
  for (int a = tid; a < ldh; a += nthr) sXs[a] = a < d.nI ? s_loc[a] : 0.0;
  for (int k = tid; k < p; k += nthr) sXg[k] = sig[d.loc_off + k];
  __syncthreads();
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2* H2 = reinterpret_cast<d2*>(H);       // ldh is even: a pair never spans two columns
  const int64_t n2 = (int64_t)ldh * p / 2;
  for (int64_t q0 = tid; q0 < n2; q0 += 8 * nthr) {
    d2 h[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) h[u] = q0 + u * nthr < n2 ? H2[q0 + u * nthr] : d2{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t q = q0 + u * nthr;
      if (q >= n2) break;
      const int k = (int)(2 * q / ldh), a = (int)(2 * q % ldh);
      const double g = sXg[k];
      d2 v;
      v.x = (a < d.nI) ? h[u].x * sXs[a] / g : 0.0;
      v.y = (a + 1 < d.nI) ? h[u].y * sXs[a + 1] / g : 0.0;
      H2[q] = v;
    }
  }
}

// W_i = A(Xi_i, Omega_Ii) X_i  (nXi x p, column-major)
__global__ void __launch_bounds__(256)
k_coarse_W(const SubDesc* __restrict__ subs, const int32_t* __restrict__ xi,
           const int32_t* __restrict__ part, const int32_t* __restrict__ locown,
           const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
           const double* __restrict__ vals, const double* __restrict__ X, double* __restrict__ W) {
  constexpr int ECAP = 8;
  const SubDesc d = subs[blockIdx.x];
  const int i = d.id;
  if (d.p == 0) return;
  const int32_t* rows = xi + d.xi_off;
  const double* Xi = X + d.x_off;
  double* Wi = W + d.w_off;
  // one thread per row of Xi_i (a subdomain's rows spread over gridDim.y
  // workgroups): its entries in Omega_Ii are read once and kept in registers
  // for all p columns, four columns at a time (rows with more than ECAP such
  // entries read them again per column)
  const int step = gridDim.y * blockDim.x;
  for (int rho = blockIdx.y * blockDim.x + threadIdx.x; rho < d.nXi; rho += step) {
    const int r = rows[rho];
    double ev[ECAP];
    int ep[ECAP];
    int ne = 0;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      const int c = colind[e];
      if (part[c] != i) continue;
      if (ne < ECAP) { ev[ne] = vals[e]; ep[ne] = locown[c]; }
      ++ne;
    }
    if (ne <= ECAP) {
      int k = 0;
      for (; k + 4 <= d.p; k += 4) {
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < ECAP; ++q)
          if (q < ne)
#pragma unroll
            for (int u = 0; u < 4; ++u) s4[u] += ev[q] * Xi[(int64_t)(k + u) * d.nIp + ep[q]];
#pragma unroll
        for (int u = 0; u < 4; ++u) Wi[(int64_t)(k + u) * d.nXi + rho] = s4[u];
      }
      for (; k < d.p; ++k) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < ECAP; ++q)
          if (q < ne) s += ev[q] * Xi[(int64_t)k * d.nIp + ep[q]];
        Wi[(int64_t)k * d.nXi + rho] = s;
      }
      continue;
    }
    for (int k = 0; k < d.p; ++k) {
      const double* xk = Xi + (int64_t)k * d.nIp;
      double s = 0.0;
      {
        for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          const int c = colind[e];
          if (part[c] == i) s += vals[e] * xk[locown[c]];
        }
      }
      Wi[(int64_t)k * d.nXi + rho] = s;
    }
  }
}

// Blocks of E = W^T W for every pair (i <= j) sharing rows; lower part only,
// in the tile-envelope layout of E (global coarse numbering).  One work item
// = (pair, 32 x 32 output block); each wave forms one 16 x 16 quadrant with
// MFMA over the shared rows.
__global__ void __launch_bounds__(256)
k_coarse_E(const SubDesc* __restrict__ subs, const PairDesc* __restrict__ pairs,
           const int32_t* __restrict__ pair_rows, const int4* __restrict__ items,
           const int32_t* __restrict__ eF, const int64_t* __restrict__ eOff,
           const double* __restrict__ W, double* __restrict__ efac) {
  const int4 it = items[blockIdx.x];
  const PairDesc pr = pairs[it.x];
  const SubDesc di = subs[pr.i], dj = subs[pr.j];
  const bool diag = pr.i == pr.j;
  const double* Wi = W + di.w_off;
  const double* Wj = W + dj.w_off;
  const int32_t* rl = pair_rows + 2 * pr.rows_off;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int bi = wave / 2, bj = wave % 2, li = lane % 16, lk = lane / 16;
  const int l = it.y * TS + 16 * bi + li;     // row of E inside subdomain j's block
  const int k = it.z * TS + 16 * bj + li;     // column of E inside subdomain i's block
  const bool lv = l < dj.p, kv = k < di.p;
  const int nrows = diag ? di.nXi : pr.nrows;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  // the shared rows in steps of 4; EU steps load their operands before their
  // products, so the loads of a batch overlap (same product order)
  constexpr int EU = 8;
  const double* wj = Wj + (int64_t)l * dj.nXi;
  const double* wi = Wi + (int64_t)k * di.nXi;
  int t0 = 0;
  for (; t0 + 4 * EU <= nrows; t0 += 4 * EU) {
    double a[EU], b[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int t = t0 + 4 * u + lk;
      const int rj = diag ? t : rl[2 * t + 1];
      const int ri = diag ? t : rl[2 * t];
      a[u] = lv ? wj[rj] : 0.0;
      b[u] = kv ? wi[ri] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) acc = Mfma<double>::mma(a[u], b[u], acc);
  }
  for (; t0 < nrows; t0 += 4) {
    const int t = t0 + lk;
    double a = 0.0, b = 0.0;
    if (t < nrows) {
      const int rj = diag ? t : rl[2 * t + 1];
      const int ri = diag ? t : rl[2 * t];
      if (lv) a = wj[rj];
      if (kv) b = wi[ri];
    }
    acc = Mfma<double>::mma(a, b, acc);
  }
  for (int v = 0; v < 4; ++v) {
    const int lr = it.y * TS + 16 * bi + Mfma<double>::acc_row(lane, v);
    const int kc = it.z * TS + 16 * bj + Mfma<double>::acc_col(lane, v);
    if (lr >= dj.p || kc >= di.p) continue;
    const int64_t row = dj.cg_off + lr, col = di.cg_off + kc;
    if (diag && row < col) continue;
    const int I = (int)(row / TS), J = (int)(col / TS);
    efac[tile_pos(eF, eOff, I, J) * TT + (col % TS) * TS + (row % TS)] = acc[v];
  }
}

// Diagonal blocks of E for a shifted C: E_ii += s X_i^T X_i, the
// contribution of the rows sqrt(s) e_j (j in Omega_Ii) that the shift adds to
// A.  Same work items and output layout as k_coarse_E; only the items of
// diagonal pairs act, with the interior rows of X_i as the shared rows.
__global__ void __launch_bounds__(256)
k_coarse_E_shift(const SubDesc* __restrict__ subs, const PairDesc* __restrict__ pairs,
                 const int4* __restrict__ items, const int32_t* __restrict__ eF,
                 const int64_t* __restrict__ eOff, const double* __restrict__ X, double shift,
                 double* __restrict__ efac) {
  const int4 it = items[blockIdx.x];
  const PairDesc pr = pairs[it.x];
  if (pr.i != pr.j) return;
  const SubDesc d = subs[pr.i];
  const double* Xi = X + d.x_off;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int bi = wave / 2, bj = wave % 2, li = lane % 16, lk = lane / 16;
  const int l = it.y * TS + 16 * bi + li;
  const int k = it.z * TS + 16 * bj + li;
  const bool lv = l < d.p, kv = k < d.p;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  const double* xl = Xi + (int64_t)l * d.nIp;
  const double* xk = Xi + (int64_t)k * d.nIp;
  for (int t0 = 0; t0 < d.nI; t0 += 4) {
    const int t = t0 + lk;
    const double a = (lv && t < d.nI) ? xl[t] : 0.0;
    const double b = (kv && t < d.nI) ? xk[t] : 0.0;
    acc = Mfma<double>::mma(a, b, acc);
  }
  for (int v = 0; v < 4; ++v) {
    const int lr = it.y * TS + 16 * bi + Mfma<double>::acc_row(lane, v);
    const int kc = it.z * TS + 16 * bj + Mfma<double>::acc_col(lane, v);
    if (lr >= d.p || kc >= d.p) continue;
    const int64_t row = d.cg_off + lr, col = d.cg_off + kc;
    if (row < col) continue;
    const int I = (int)(row / TS), J = (int)(col / TS);
    efac[tile_pos(eF, eOff, I, J) * TT + (col % TS) * TS + (row % TS)] += shift * acc[v];
  }
}

// One step J of the right-looking tile Cholesky of E, fused with the
// trailing update of the previous column.  One launch holds that step for
// several independent diagonal blocks of E (the instances of a batch: step s
// of every instance with more than s tile columns), one job each; a job
// (EJOB_INTS ints: J, first of its rows in erows, their number nr, first of
// the rows of column J - 1 below J, their number npr, first workgroup)
// takes the workgroups from its first up to the next job's.
// - Workgroups below ndiag (panel role) apply column J - 1 to the tiles of
//   column J themselves: A(J, J) -= L(J, J-1) L(J, J-1)^T, and for their
//   panel rows A(I, J) -= L(I, J-1) L(J, J-1)^T.  In every such workgroup
//   wave 0 factors and inverts the diagonal tile in registers while the other
//   waves update their panel tiles, one each; these then form
//   L(I, J) = A(I, J) L_JJ^{-T}.  Workgroup 0 keeps
//   L_JJ^{-1}, the only form of the diagonal tile the solves read, so (J, J)
//   itself is left unchanged.
// - The other workgroups apply the rest of column J - 1's update, one wave
//   per pair of its rows below J: A(Ia, Ib) -= L(Ia, J-1) L(Ib, J-1)^T.
// The two roles touch disjoint tiles (column J against columns > J), and
// every update of column J by columns before J - 1 ran in an earlier launch.
constexpr int ESTEP_WAVES = 8;
constexpr int EPANEL = ESTEP_WAVES - 1;    // panel tiles per workgroup (waves 1..)

__global__ void __launch_bounds__(ESTEP_WAVES * 64)
k_echol_step(const int32_t* __restrict__ eF, const int64_t* __restrict__ eOff,
             const int32_t* __restrict__ erows, const int32_t* __restrict__ jobs, int njobs,
             double* __restrict__ efac, double* __restrict__ edinv, int32_t* __restrict__ status) {
  __shared__ double sW[TS * LDT], sInv[TS * LDT];
  __shared__ double sS[ESTEP_WAVES][TS * LDT];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid / 64, lane = tid % 64;
  // this workgroup's job: the last one whose first workgroup is at most ours
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[EJOB_INTS * mid + 5] <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const int32_t* jb = jobs + EJOB_INTS * lo;
  const int J = jb[0], nr = jb[2], npr = jb[4];
  const int32_t* rows = erows + jb[1];
  const int32_t* prows = erows + jb[3];
  const int bx = (int)blockIdx.x - jb[5];
  const int ndiag = max(1, (nr + EPANEL - 1) / EPANEL);
  double4_t acc[4];
  if (bx >= ndiag) {
    const int64_t gw = (int64_t)(bx - ndiag) * ESTEP_WAVES + wave;
    const int64_t npairs = (int64_t)npr * (npr + 1) / 2;
    if (gw >= npairs) return;
    // pair index -> (a, b), a >= b
    int a = (int)((sqrt(8.0 * gw + 1.0) - 1.0) / 2.0);
    while ((int64_t)a * (a + 1) / 2 > gw) --a;
    while ((int64_t)(a + 1) * (a + 2) / 2 <= gw) ++a;
    const int b = (int)(gw - (int64_t)a * (a + 1) / 2);
    const int Ia = prows[a], Ib = prows[b];
    double* Cab = efac + tile_pos(eF, eOff, Ia, Ib) * TT;
    tile_acc_load<double>(acc, Cab, TS, lane);
    tile_mma_nt<double, true>(acc, efac + tile_pos(eF, eOff, Ia, J - 1) * TT, TS,
                              efac + tile_pos(eF, eOff, Ib, J - 1) * TT, TS, lane);
    tile_acc_store<double>(acc, Cab, TS, lane);
    return;
  }
  const bool prevJ = J > 0 && eF[J] <= J - 1;         // L(J, J-1) is stored
  const double* Ljp = prevJ ? efac + tile_pos(eF, eOff, J, J - 1) * TT : nullptr;
  // wave 0 factors and inverts the diagonal tile; meanwhile waves 1.. hold
  // their panel tiles' A(I, J) - L(I, J-1) L(J, J-1)^T in registers
  const int a = bx * EPANEL + wave - 1;
  const bool mine = wave > 0 && a < nr;
  const int I = mine ? rows[a] : 0;
  if (wave == 0) {
    const double* Ajj = efac + tile_pos(eF, eOff, J, J) * TT;
    for (int e = lane; e < TT; e += 64) sW[(e / TS) * LDT + e % TS] = Ajj[e];
    wave_sync();
    if (prevJ) {
      tile_acc_load<double>(acc, sW, LDT, lane);
      tile_mma_nt<double, true>(acc, Ljp, TS, Ljp, TS, lane);
      wave_sync();
      tile_acc_store<double>(acc, sW, LDT, lane);
      wave_sync();
    }
    const bool ok = tile_potrf_inv_reg<double>(sW, nullptr, sInv, lane);
    if (!ok && lane == 0 && bx == 0) atomicCAS(status, 0, J + 1);
  } else if (mine) {
    tile_acc_load<double>(acc, efac + tile_pos(eF, eOff, I, J) * TT, TS, lane);
    if (prevJ && eF[I] <= J - 1)
      tile_mma_nt<double, true>(acc, efac + tile_pos(eF, eOff, I, J - 1) * TT, TS, Ljp, TS, lane);
  }
  __syncthreads();
  if (bx == 0)
    for (int e = tid; e < TT; e += nthr) edinv[(int64_t)J * TT + e] = sInv[(e / TS) * LDT + e % TS];
  if (mine) {
    double* S = sS[wave];
    tile_acc_store<double>(acc, S, LDT, lane);
    wave_sync();
    tile_acc_zero<double>(acc);
    tile_mma_nt<double, false>(acc, S, LDT, sInv, LDT, lane);
    tile_acc_store<double>(acc, efac + tile_pos(eF, eOff, I, J) * TT, TS, lane);
  }
}

// Full 32 x 32 product fragments for one wave (K = 32): op(A) rows in two
// halves, B columns in two halves; acc[bi * 2 + bj] as in tile_acc_load.
struct TileFrag { double a[2][8], b[2][8]; };

template <bool TA>
__device__ inline void tile_frag_load(TileFrag& f, const double* A, int lda, const double* B, int ldb,
                                      int lane) {
  const int li = lane % 16, lk = lane / 16;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 4 * q + lk;
      f.a[h][q] = TA ? A[(int64_t)(16 * h + li) * lda + k] : A[(int64_t)k * lda + 16 * h + li];
      f.b[h][q] = B[(int64_t)(16 * h + li) * ldb + k];
    }
}

__device__ inline void tile_frag_mma(double4_t acc[4], const TileFrag& f) {
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi * 2 + bj] = Mfma<double>::mma(f.a[bi][q], f.b[bj][q], acc[bi * 2 + bj]);
}

// Dense inverse of E per instance, lower block triangle.  Column block c
// (32 columns) solves L L^T X = I(:, c), rows >= c only: forward substitution
// Y(I) = L_II^{-1} (delta_Ic I - sum_K L(I,K) Y(K)) for I >= c, then backward
// substitution X(K) = L_KK^{-T} (Y(K) - sum_I L(I,K)^T X(I)) for K from the
// last tile down to c.  Both sweeps are left-looking, so every output tile is
// written once.
//
// The band of already computed tiles that a step needs stays in registers:
// wave w keeps the EWIN_SLOTS most recent tiles with index = w (mod 8) as MFMA
// B fragments, so a step reads only the tiles of L (shared by all column
// blocks).  Tiles further back than the window are read from memory.  Eight
// waves of at most 256 registers each run two to a SIMD, so one wave's
// products overlap the other's loads; the first four also form the diagonal
// products, one 16 x 16 quadrant each.  The wave partials of a step are added
// in a fixed order.  Each workgroup works
// through a list of column blocks chosen so that the lists have equal work
// (the work of block c is proportional to the number of tile rows below c).
// The backward sweep multiplies by transposed tiles of L; it reads them from
// a tile-by-tile transposed copy (efacT, edinvT), so that every operand
// fragment load is a column read.
constexpr int EINV_WAVES = 8;
constexpr int EWIN_SLOTS = 2;
constexpr int ELIST = EINV_WAVES * 64;      // backward list entries staged in LDS (one per thread)

struct AFrag { double a[2][8]; };

template <bool TA>
__device__ inline void afrag_load(AFrag& f, const double* A, int lda, int lane) {
  const int li = lane % 16, lk = lane / 16;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 4 * q + lk;
      f.a[h][q] = TA ? A[(int64_t)(16 * h + li) * lda + k] : A[(int64_t)k * lda + 16 * h + li];
    }
}

__device__ inline void frag_mma(double4_t acc[4], const AFrag& f, const double (&b)[2][8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi * 2 + bj] = Mfma<double>::mma(f.a[bi][q], b[bj][q], acc[bi * 2 + bj]);
}

// B fragments of a 32 x 32 column-major tile (leading dimension ld)
__device__ inline void bfrag_load(double (&b)[2][8], const double* B, int ld, int lane) {
  const int li = lane % 16, lk = lane / 16;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 8; ++q) b[h][q] = B[(int64_t)(16 * h + li) * ld + 4 * q + lk];
}

__global__ void __launch_bounds__(EINV_WAVES * 64)
k_einv(const int32_t* __restrict__ eF, const int64_t* __restrict__ eOff,
       const int32_t* __restrict__ seg_of_tile, const SegDesc* __restrict__ segs,
       const int32_t* __restrict__ erows, const int64_t* __restrict__ eptr,
       const int32_t* __restrict__ bin_ptr, const int32_t* __restrict__ bin_cols,
       const double* __restrict__ efac, const double* __restrict__ edinv,
       const double* __restrict__ efacT, const double* __restrict__ edinvT,
       double* __restrict__ einv) {
  __shared__ double sY[TS * LDT], sN[TS * LDT];
  __shared__ double spart[EINV_WAVES][TT];
  __shared__ int32_t sEI[ELIST];            // backward step: rows I of the list (local index)
  __shared__ int64_t sEO[ELIST];            // and the tile index of L(I, K)
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid / 64, lane = tid % 64;
  const int bi = (w / 2) % 2, bj = w % 2;    // quadrant of the diagonal products
  const bool dq = w < 4;                     // waves that form the diagonal products

  auto put_partial = [&](const double4_t acc[4]) {
#pragma unroll
    for (int qd = 0; qd < 4; ++qd)
#pragma unroll
      for (int v = 0; v < 4; ++v) spart[w][(qd * 4 + v) * 64 + lane] = acc[qd][v];
  };
  auto elem_rc = [](int e, int& row, int& col) {
    const int l = e % 64, v = (e / 64) % 4, qd = e / 256;
    row = 16 * (qd / 2) + Mfma<double>::acc_row(l, v);
    col = 16 * (qd % 2) + Mfma<double>::acc_col(l, v);
  };

  for (int item = bin_ptr[blockIdx.x]; item < bin_ptr[blockIdx.x + 1]; ++item) {
    const int cglob = bin_cols[item];
    const SegDesc sg = segs[seg_of_tile[cglob]];
    const int t0 = (int)sg.etile0, nt = (int)sg.etiles;
    const int c = cglob - t0;
    const int ld = nt * TS;
    double* Xc = einv + sg.einv_off + (int64_t)c * TS * ld;
    double win[EWIN_SLOTS][2][8];
    int wk[EWIN_SLOTS];                     // tile index held by each slot (-1: empty)

    // ---- forward
#pragma unroll
    for (int sl = 0; sl < EWIN_SLOTS; ++sl) wk[sl] = -1;
    for (int I = c; I < nt; ++I) {
      const int Ig = t0 + I;
      const int K0 = max(eF[Ig] - t0, c);
      double dfr[8];                         // this step's diagonal inverse, loaded under the products
      if (dq) quad_afrag(dfr, edinv + (int64_t)Ig * TT, TS, bi, lane);
      double4_t acc[4];
      tile_acc_zero<double>(acc);
      // tiles of this wave evicted from its window (the window holds every
      // later tile of the wave, so an empty window means there is none)
      int kold = K0;
#pragma unroll
      for (int sl = EWIN_SLOTS - 1; sl >= 0; --sl)
        if (wk[sl] >= 0) kold = wk[sl];
      for (int K = K0 + ((w - K0 % EINV_WAVES) + EINV_WAVES) % EINV_WAVES; K < kold; K += EINV_WAVES) {
        AFrag f;
        double b[2][8];
        afrag_load<false>(f, efac + tile_pos(eF, eOff, Ig, t0 + K) * TT, TS, lane);
        bfrag_load(b, Xc + K * TS, ld, lane);
        frag_mma(acc, f, b);
      }
#pragma unroll
      for (int sl = 0; sl < EWIN_SLOTS; ++sl)
        if (wk[sl] >= K0) {
          AFrag f;
          afrag_load<false>(f, efac + tile_pos(eF, eOff, Ig, t0 + wk[sl]) * TT, TS, lane);
          frag_mma(acc, f, win[sl]);
        }
      put_partial(acc);
      __syncthreads();
      for (int e = tid; e < TT; e += nthr) {
        int row, col;
        elem_rc(e, row, col);
        double v = (I == c && row == col) ? 1.0 : 0.0;
        for (int q = 0; q < EINV_WAVES; ++q) v -= spart[q][e];
        sY[col * LDT + row] = v;
      }
      __syncthreads();
      if (dq) {
        double4_t y = {0.0, 0.0, 0.0, 0.0};
        quad_mma_pre(y, dfr, sY, LDT, bj, lane);
        quad_store(y, Xc + I * TS, ld, bi, bj, lane);
        quad_store(y, sN, LDT, bi, bj, lane);
      }
      __syncthreads();
      if (I % EINV_WAVES == w) {            // the new tile enters this wave's window
#pragma unroll
        for (int sl = 0; sl + 1 < EWIN_SLOTS; ++sl) {
          wk[sl] = wk[sl + 1];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < 8; ++q) win[sl][h][q] = win[sl + 1][h][q];
        }
        wk[EWIN_SLOTS - 1] = I;
        bfrag_load(win[EWIN_SLOTS - 1], sN, LDT, lane);
      }
    }

    // ---- backward.  The list of rows I > K with F(I) <= K and the tile
    // index of L(I, K) for each is staged in LDS by the whole workgroup one
    // step ahead; a window slot keeps F and the tile offset of its row.
    auto fill_list = [&](int Kg) {
      const int64_t u0 = eptr[Kg];
      const int n = (int)min<int64_t>(eptr[Kg + 1] - u0, ELIST);
      for (int j = tid; j < n; j += nthr) {
        const int Ig = erows[u0 + j];
        sEI[j] = Ig - t0;
        sEO[j] = tile_pos(eF, eOff, Ig, Kg);
      }
    };
    int wF[EWIN_SLOTS];
    int64_t wO[EWIN_SLOTS];
#pragma unroll
    for (int sl = 0; sl < EWIN_SLOTS; ++sl) {
      wk[sl] = -1;
      wF[sl] = 0;
      wO[sl] = 0;
    }
    fill_list(t0 + nt - 1);
    __syncthreads();
    for (int K = nt - 1; K >= c; --K) {
      const int Kg = t0 + K;
      double dfr[8];                         // this step's diagonal inverse, loaded under the products
      if (dq) quad_afrag(dfr, edinvT + (int64_t)Kg * TT, TS, bi, lane);
      // loads whose latency the products hide: this step's tile of Y for the
      // reduction below, and the next step's list (one entry per thread)
      double ypre[TT / (EINV_WAVES * 64)];
#pragma unroll
      for (int i = 0; i < TT / (EINV_WAVES * 64); ++i) {
        int row, col;
        elem_rc(tid + i * EINV_WAVES * 64, row, col);
        ypre[i] = Xc[(int64_t)col * ld + K * TS + row];
      }
      int nxt_n = 0, nxt_I = 0;
      if (K > c) {
        const int64_t un = eptr[Kg - 1];
        nxt_n = (int)min<int64_t>(eptr[Kg] - un, ELIST);
        if (tid < nxt_n) nxt_I = erows[un + tid];
      }
      double4_t acc[4];
      tile_acc_zero<double>(acc);
      // rows of this wave evicted from its window (rows above its oldest
      // slot; an empty window means the wave has no computed row yet)
      int ifar = nt;
#pragma unroll
      for (int sl = EWIN_SLOTS - 1; sl >= 0; --sl)
        if (wk[sl] >= 0) ifar = wk[sl];
      const int64_t u0 = eptr[Kg];
      const int nlist = (int)(eptr[Kg + 1] - u0);
      for (int j = 0; j < nlist; ++j) {
        int I;
        int64_t off;
        if (j < ELIST) {
          I = sEI[j];
          off = sEO[j];
        } else {
          I = erows[u0 + j] - t0;
          off = tile_pos(eF, eOff, t0 + I, Kg);
        }
        if (I % EINV_WAVES != w || I <= ifar) continue;
        AFrag f;
        double b[2][8];
        afrag_load<false>(f, efacT + off * TT, TS, lane);
        bfrag_load(b, Xc + I * TS, ld, lane);
        frag_mma(acc, f, b);
      }
#pragma unroll
      for (int sl = 0; sl < EWIN_SLOTS; ++sl) {
        if (wk[sl] >= 0 && wF[sl] <= Kg) {
          AFrag f;
          afrag_load<false>(f, efacT + (wO[sl] + (Kg - wF[sl])) * TT, TS, lane);
          frag_mma(acc, f, win[sl]);
        }
      }
      const int64_t nxt_O = tid < nxt_n ? tile_pos(eF, eOff, nxt_I, Kg - 1) : 0;
      put_partial(acc);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < TT / (EINV_WAVES * 64); ++i) {
        const int e = tid + i * EINV_WAVES * 64;
        int row, col;
        elem_rc(e, row, col);
        double v = ypre[i];
        for (int q = 0; q < EINV_WAVES; ++q) v -= spart[q][e];
        sY[col * LDT + row] = v;
      }
      __syncthreads();
      if (dq) {
        double4_t x = {0.0, 0.0, 0.0, 0.0};
        quad_mma_pre(x, dfr, sY, LDT, bj, lane);
        quad_store(x, Xc + K * TS, ld, bi, bj, lane);
        quad_store(x, sN, LDT, bi, bj, lane);
      }
      if (tid < nxt_n) {                    // this step's list is no longer read
        sEI[tid] = nxt_I - t0;
        sEO[tid] = nxt_O;
      }
      __syncthreads();
      if (K % EINV_WAVES == w) {
#pragma unroll
        for (int sl = 0; sl + 1 < EWIN_SLOTS; ++sl) {
          wk[sl] = wk[sl + 1];
          wF[sl] = wF[sl + 1];
          wO[sl] = wO[sl + 1];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < 8; ++q) win[sl][h][q] = win[sl + 1][h][q];
        }
        wk[EWIN_SLOTS - 1] = K;
        wF[EWIN_SLOTS - 1] = eF[Kg];
        wO[EWIN_SLOTS - 1] = eOff[Kg];
        bfrag_load(win[EWIN_SLOTS - 1], sN, LDT, lane);
      }
    }
    __syncthreads();
  }
}

// out = in with every 32 x 32 tile transposed
__global__ void __launch_bounds__(256)
k_tile_transpose(int64_t ntiles, const double* __restrict__ in, double* __restrict__ out) {
  __shared__ double sT[TS * LDT];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const double* a = in + t * TT;
    double* b = out + t * TT;
    for (int e = threadIdx.x; e < TT; e += blockDim.x) sT[(e / TS) * LDT + e % TS] = a[e];
    __syncthreads();
    for (int e = threadIdx.x; e < TT; e += blockDim.x) b[e] = sT[(e % TS) * LDT + e / TS];
    __syncthreads();
  }
}

// c_i = X_i^T r(Omega_Ii): r gathered once into LDS (in chunks), one wave per
// coarse vector.
constexpr int RCHUNK = 8192;
template <typename TX>
__global__ void __launch_bounds__(1024)
k_coarse_restrict(const SubDesc* __restrict__ subs, const int32_t* __restrict__ omega,
                  const TX* __restrict__ X, const double* __restrict__ r,
                  double* __restrict__ cvec) {
  __shared__ double sr[RCHUNK];
  __shared__ double sacc[128];
  const SubDesc d = subs[blockIdx.x];
  if (d.p == 0) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
  const int32_t* om = omega + d.omega_off;
  constexpr int EV = 16 / sizeof(TX);
  typedef TX V __attribute__((ext_vector_type(EV)));
  double acc[8];
  for (int kb = 0; kb < d.p; kb += 8 * nwaves) {
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int a0 = 0; a0 < d.nI; a0 += RCHUNK) {
      const int len = min(RCHUNK, d.nI - a0);
      // the chunk in whole 16-byte vectors of X (columns are padded with
      // zeros to a multiple of 32 rows; the copy of r is zero there too)
      const int nvec = (len + EV - 1) / EV;
      __syncthreads();
      for (int a = threadIdx.x; a < nvec * EV; a += blockDim.x) sr[a] = a < len ? r[om[a0 + a]] : 0.0;
      __syncthreads();
#pragma unroll 1
      for (int u = 0; u < 8; ++u) {
        const int k = kb + u * nwaves + wave;
        if (k >= d.p) break;
        const V* xk = reinterpret_cast<const V*>(X + d.x_off + (int64_t)k * d.nIp + a0);
        // four independent 16-byte loads in flight per lane
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        int q = lane;
        for (; q + 3 * 64 < nvec; q += 4 * 64) {
          V xv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) xv[i] = xk[q + 64 * i];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < EV; ++e) s4[i] += (double)xv[i][e] * sr[(q + 64 * i) * EV + e];
        }
        for (int i = 0; q < nvec; q += 64, ++i) {
          const V xv = xk[q];
#pragma unroll
          for (int e = 0; e < EV; ++e) s4[i] += (double)xv[e] * sr[q * EV + e];
        }
        acc[u] += (s4[0] + s4[1]) + (s4[2] + s4[3]);
      }
    }
    for (int u = 0; u < 8; ++u) {
      const int k = kb + u * nwaves + wave;
      if (k >= d.p) break;
      double s = acc[u];
      for (int w = 32; w > 0; w >>= 1) s += __shfl_down(s, w, 64);
      if (lane == 0) cvec[d.cg_off + k] = s;
    }
  }
  (void)sacc;
}

// d = E^{-1} c with the lower block triangle of the symmetric inverse, read
// once.  The triangle is cut into chunks of up to ESYM_ROWTILES row tiles of
// one tile column J (equal work per workgroup).  Pass 1, one workgroup per
// chunk, one row r per thread: the row part P_J(r) = sum_k T(r, k) c_J(k)
// (the diagonal tile's full row sums included) and the chunk's column
// partial sum_r T(r, k) c(r) over its rows below the diagonal tile.  Pass 2:
// d_I = sum_{J <= I} P_J(I) + the column partials of the chunks of column I,
// each sum in a fixed order.
__global__ void __launch_bounds__(256)
k_esym_pass1(const int4* __restrict__ chunks, const int32_t* __restrict__ seg_of_tile,
             const SegDesc* __restrict__ segs, const double* __restrict__ einv,
             const double* __restrict__ cvec, double* __restrict__ part,
             double* __restrict__ ucol) {
  __shared__ double cJ[TS];
  __shared__ double wsum[4][TS];
  const int4 ch = chunks[blockIdx.x];
  const SegDesc sg = segs[seg_of_tile[ch.x]];
  const int J = ch.x - (int)sg.etile0;
  const int64_t ld = sg.etiles * TS;
  const double* Xc = einv + sg.einv_off + (int64_t)J * TS * ld;
  const double* cv = cvec + sg.c0;
  double* P = part + sg.einv_off / TS + (int64_t)J * ld;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  if (tid < TS) cJ[tid] = cv[J * TS + tid];
  __syncthreads();
  const int64_t r = (int64_t)ch.y * TS + tid;
  double col[TS];
  if (tid < ch.z * TS) {
    const double cr = r >= (J + 1) * TS ? cv[r] : 0.0;   // the diagonal tile adds by rows only
    double e[TS];
#pragma unroll
    for (int k = 0; k < TS; ++k) e[k] = Xc[(int64_t)k * ld + r];
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < TS; ++k) {
      rs[k & 3] += e[k] * cJ[k];
      col[k] = e[k] * cr;
    }
    P[r] = (rs[0] + rs[1]) + (rs[2] + rs[3]);
  } else {
#pragma unroll
    for (int k = 0; k < TS; ++k) col[k] = 0.0;
  }
  // column sums over the wave by recursive halving: after the step with
  // offset o (32, 16, .., 2) a lane keeps the half of its entries selected
  // by bit o of its lane id; a last exchange with offset 1 completes lane l's
  // sum for column (l >> 1) with bit reversal of the kept halves.
  int n = TS;
#pragma unroll
  for (int o = 32; o >= 2; o >>= 1) {
    n >>= 1;
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < TS / 2; ++i) {
      if (i < n) {
        const double send = up ? col[i] : col[i + n];
        const double keep = up ? col[i + n] : col[i];
        col[i] = keep + __shfl_xor(send, o, 64);
      }
    }
  }
  double v = col[0] + __shfl_xor(col[0], 1, 64);
  // lane l now holds column k(l): bits 5..1 of l, most significant first,
  // give the halves kept at offsets 32 .. 2
  const int k = ((lane >> 5) & 1) * 16 + ((lane >> 4) & 1) * 8 + ((lane >> 3) & 1) * 4 +
                ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1);
  if ((lane & 1) == 0) wsum[wave][k] = v;
  __syncthreads();
  if (tid < TS)
    ucol[(int64_t)blockIdx.x * TS + tid] = (wsum[0][tid] + wsum[1][tid]) + (wsum[2][tid] + wsum[3][tid]);
}

__global__ void __launch_bounds__(256)
k_esym_pass2(const int32_t* __restrict__ seg_of_tile, const SegDesc* __restrict__ segs,
             const int32_t* __restrict__ chunk_ptr, const double* __restrict__ part,
             const double* __restrict__ ucol, double* __restrict__ dvec) {
  // one workgroup per tile row I: 8 groups of 32 threads split the row
  // partials P_J(I), J <= I, and the column partials of the chunks of column I
  __shared__ double sp[8][TS];
  const int cglob = blockIdx.x;
  const SegDesc sg = segs[seg_of_tile[cglob]];
  const int I = cglob - (int)sg.etile0;
  const int64_t ld = sg.etiles * TS;
  const double* P = part + sg.einv_off / TS;
  const int r = threadIdx.x % TS, g = threadIdx.x / TS;
  double s = 0.0;
  for (int J = g; J <= I; J += 8) s += P[(int64_t)J * ld + I * TS + r];
  for (int q = chunk_ptr[cglob] + g; q < chunk_ptr[cglob + 1]; q += 8) s += ucol[(int64_t)q * TS + r];
  sp[g][r] = s;
  __syncthreads();
  if (threadIdx.x < TS) {
    double acc = 0.0;
    for (int q = 0; q < 8; ++q) acc += sp[q][r];
    dvec[sg.c0 + I * TS + r] = acc;
  }
}

__global__ void k_set_values(int64_t n, const int64_t* __restrict__ idx, double v,
                             double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[idx[k]] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_set_values(hipStream_t st, int64_t n, const int64_t* idx, double v, double* out) {
  if (n == 0) return;
  k_set_values<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, idx, v, out);
}

void launch_gamma_T(hipStream_t st, int nsub, const DevPlan& P, const double* fac, double* Tg) {
  k_gamma_T<<<nsub, 256, 0, st>>>(P.heavy(), P.tileF, P.tileOff, fac, Tg);
}


void launch_coarse_X(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                     const double* dinv, const double* scale, const double* work,
                     const double* sig, double* X) {
  k_coarse_X<<<nsub, 512, 0, st>>>(P.heavy(), P.tileF, P.tileOff, fac, dinv, scale, work, sig, X);
}

void launch_coarse_W(hipStream_t st, int nsub, const DevPlan& P, const DevMatrix& M,
                     const double* X, double* W) {
  k_coarse_W<<<dim3(nsub, 16), 256, 0, st>>>(P.heavy(), P.xi, P.part, P.locown, M.rowptr, M.colind, M.vals, X,
                                   W);
}

void launch_coarse_E(hipStream_t st, int nitems, const DevPlan& P, const DevCoarse& Cc,
                     const double* W, double* efac) {
  if (nitems == 0) return;
  k_coarse_E<<<nitems, 256, 0, st>>>(P.subs, Cc.pairs, Cc.pair_rows, Cc.e_items, Cc.eF, Cc.eOff, W,
                                     efac);
}

void launch_coarse_E_shift(hipStream_t st, int nitems, const DevPlan& P, const DevCoarse& Cc,
                           const double* X, double s, double* efac) {
  if (nitems == 0) return;
  k_coarse_E_shift<<<nitems, 256, 0, st>>>(P.subs, Cc.pairs, Cc.e_items, Cc.eF, Cc.eOff, X, s, efac);
}

int echol_job_blocks(int nr, int npr) {
  const int ndiag = std::max(1, (nr + EPANEL - 1) / EPANEL);
  const int64_t npairs = (int64_t)npr * (npr + 1) / 2;
  return ndiag + (int)((npairs + ESTEP_WAVES - 1) / ESTEP_WAVES);
}

void launch_echol_step(hipStream_t st, const DevCoarse& Cc, const int32_t* jobs, int njobs,
                       int nblocks, double* efac, double* edinv, int32_t* status) {
  if (njobs == 0) return;
  k_echol_step<<<nblocks, ESTEP_WAVES * 64, 0, st>>>(Cc.eF, Cc.eOff, Cc.erows, jobs, njobs, efac,
                                                    edinv, status);
}

void launch_tile_transpose(hipStream_t st, int64_t ntiles, const double* in, double* out) {
  if (ntiles <= 0) return;
  k_tile_transpose<<<(unsigned)std::min<int64_t>(ntiles, 8192), 256, 0, st>>>(ntiles, in, out);
}

void launch_einv(hipStream_t st, int nbins, const DevCoarse& Cc, const double* efac,
                 const double* edinv, const double* efacT, const double* edinvT, double* einv) {
  if (nbins == 0) return;
  k_einv<<<nbins, EINV_WAVES * 64, 0, st>>>(Cc.eF, Cc.eOff, Cc.e_seg_of_tile, Cc.segs, Cc.erows,
                                            Cc.eptr, Cc.einv_bin_ptr, Cc.einv_bin_cols, efac, edinv,
                                            efacT, edinvT, einv);
}

void launch_coarse_restrict(hipStream_t st, int nsub, const DevPlan& P, int max_p, const double* X,
                            const double* r, double* c) {
  if (max_p <= 0) return;
  k_coarse_restrict<double><<<nsub, 1024, 0, st>>>(P.subs, P.omega, X, r, c);
}

void launch_coarse_restrict(hipStream_t st, int nsub, const DevPlan& P, int max_p, const float* X,
                            const double* r, double* c) {
  if (max_p <= 0) return;
  k_coarse_restrict<float><<<nsub, 1024, 0, st>>>(P.subs, P.omega, X, r, c);
}

void launch_einv_gemv(hipStream_t st, int64_t n0, int S, const DevCoarse& Cc, const double* einv,
                      const double* c, double* d) {
  if (n0 == 0) return;
  const int ntiles = (int)(n0 / TS);
  k_esym_pass1<<<Cc.e_nchunks, 256, 0, st>>>(Cc.e_chunks, Cc.e_seg_of_tile, Cc.segs, einv, c,
                                             Cc.e_part, Cc.e_u);
  k_esym_pass2<<<ntiles, 256, 0, st>>>(Cc.e_seg_of_tile, Cc.segs, Cc.e_chunk_ptr, Cc.e_part, Cc.e_u, d);
}

}  // namespace lsq2l
