// Subdomain kernels: local matrices, batched Cholesky, local solves.
//
//   C_ii  = A(:,Omega_i)^T A(:,Omega_i)            (Section 3.1)
//   Ct_GG = A(Xi_i,Omega_Gamma_i)^T A(Xi_i,Omega_Gamma_i)
//           (the only block in which the local SPSD splitting of
//            eq. spsd_normal_eq differs from C_ii: rows outside Xi_i have no
//            entry in Omega_Ii, so Ct_II = C_II and Ct_IG = C_IG)
//   C_ii  = L_i L_i^T                              (Algorithm 1, local Cholesky)
//   z_i   = C_ii^{-1} r_i                          (eq. one_level_schwarz)
//
// One workgroup owns one subdomain; subdomains of uneven size share a launch.
#include "kernels.hpp"

namespace lsq2l {

__global__ void k_gather_values(int64_t nnz, const int32_t* __restrict__ perm,
                                const double* __restrict__ src, double* __restrict__ dst) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) dst[k] = src[perm[k]];
}

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

// Lower triangle of C_ii (tile-envelope layout) and of Ct_GG (dense, ld nGp).
// Thread per local column: every write of a thread lands in its own column,
// so the accumulation order is fixed and no atomics are needed.
__global__ void __launch_bounds__(256)
k_assemble(const SubDesc* __restrict__ subs, const int32_t* __restrict__ omega,
           const int32_t* __restrict__ part, const int32_t* __restrict__ locown,
           const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
           const double* __restrict__ vals, const int32_t* __restrict__ trowptr,
           const int32_t* __restrict__ trow, const double* __restrict__ tvals,
           const int32_t* __restrict__ tileF, const int64_t* __restrict__ tileOff,
           double* __restrict__ fac, double* __restrict__ ctg) {
  const int i = blockIdx.x;
  const SubDesc d = subs[i];
  const int32_t* om = omega + d.omega_off;
  const int32_t* G = om + d.nI;
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  double* A = fac + d.fac_off;
  double* Ct = ctg + d.g_off;
  for (int a = threadIdx.x; a < d.nI + d.nG; a += blockDim.x) {
    const int j = om[a];
    const int posa = a < d.nI ? a : d.nIp + (a - d.nI);
    const int ta = posa / TS, ra = posa % TS;
    for (int k = trowptr[j]; k < trowptr[j + 1]; ++k) {
      const int r = trow[k];
      const double va = tvals[k];
      const int e0 = rowptr[r], e1 = rowptr[r + 1];
      bool inxi = false;
      for (int e = e0; e < e1; ++e) inxi |= (part[colind[e]] == i);
      for (int e = e0; e < e1; ++e) {
        const int posc = local_pos(i, colind[e], part, locown, G, d.nG, d.nIp);
        if (posc < posa) continue;
        const double v = vals[e] * va;
        const int tc = posc / TS;
        A[tile_pos(F, off, tc, ta) * TT + ra * TS + (posc % TS)] += v;
        if (inxi && a >= d.nI) Ct[(int64_t)(posa - d.nIp) * d.nGp + (posc - d.nIp)] += v;
      }
    }
  }
}

// Symmetric diagonal equilibration S C S, S = diag(C)^{-1/2} (an exact
// congruence: C^{-1} = S (S C S)^{-1} S), applied to C_ii and to Ct_GG; the
// padding rows become identity rows.  scale[pos] = S_pos (0 on padding).
// k_equil_scale forms S per subdomain; k_equil_apply scales the stored tiles
// and Ct_GG, workgroup (i, y) taking tile rows y, y + gridDim.y, ...
__global__ void __launch_bounds__(256)
k_equil_scale(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
              const int64_t* __restrict__ tileOff, const double* __restrict__ fac,
              double* __restrict__ scale) {
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  const double* A = fac + d.fac_off;
  double* s = scale + d.loc_off;
  for (int pos = threadIdx.x; pos < d.np; pos += blockDim.x) {
    const bool real = pos < d.nI || (pos >= d.nIp && pos < d.nIp + d.nG);
    const double* diag = A + tile_pos(F, off, pos / TS, pos / TS) * TT + (pos % TS) * TS + pos % TS;
    s[pos] = real ? 1.0 / sqrt(*diag) : 0.0;   // diagonal > 0: every column of Omega_i has a stored entry
  }
}

__global__ void __launch_bounds__(256)
k_equil_apply(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
              const int64_t* __restrict__ tileOff, double* __restrict__ fac,
              double* __restrict__ ctg, const double* __restrict__ scale) {
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  double* A = fac + d.fac_off;
  const double* s = scale + d.loc_off;
  for (int t = blockIdx.y; t < d.ntiles; t += gridDim.y) {
    const int nt = t - F[t] + 1;
    double* row = A + off[t] * TT;
    for (int64_t e = threadIdx.x; e < (int64_t)nt * TT; e += blockDim.x) {
      const int J = F[t] + (int)(e / TT);
      const int rc = (int)(e % TT);
      const int r = t * TS + rc % TS, c = J * TS + rc / TS;
      const double sr = s[r], sc = s[c];
      if (r == c && sr == 0.0) row[e] = 1.0;
      else row[e] *= sr * sc;
    }
  }
  double* Ct = ctg + d.g_off;
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < (int64_t)d.nGp * d.nGp;
       e += (int64_t)gridDim.y * blockDim.x) {
    const int r = (int)(e % d.nGp), c = (int)(e / d.nGp);
    Ct[e] *= s[d.nIp + r] * s[d.nIp + c];   // zero on padding
  }
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

constexpr int ROWCAP = 2048;

// Right-looking tile Cholesky of one envelope matrix per workgroup:
// for each tile column J: factor and invert the diagonal tile in LDS,
// L(I,J) = A(I,J) L(J,J)^{-T} for the envelope rows, then
// A(I,K) -= L(I,J) L(K,J)^T for every pair of envelope rows (MFMA).
template <typename T>
__global__ void __launch_bounds__(256)
k_chol_local(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
             const int64_t* __restrict__ tileOff, T* __restrict__ fac, T* __restrict__ dinv,
             int32_t* __restrict__ status) {
  static_assert(sizeof(T) == sizeof(double), "the local factors are computed in double");
  __shared__ T sW[TS * LDT], sL[TS * LDT], sInv[TS * LDT];
  __shared__ int32_t rows[ROWCAP];
  __shared__ int s_count, s_ok;
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  T* A = fac + d.fac_off;
  T* Di = dinv + d.dinv_off;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid / 64, lane = tid % 64, nwaves = nthr / 64;
  bool failed = false;
  for (int J = 0; J < d.ntiles; ++J) {
    T* Ajj = A + tile_pos(F, off, J, J) * TT;
    for (int e = tid; e < TT; e += nthr) sW[(e / TS) * LDT + e % TS] = Ajj[e];
    __syncthreads();
    if (wave == 0) {
      const bool okw = tile_potrf_inv_reg(sW, sL, sInv, lane);
      if (lane == 0) s_ok = okw;
    }
    __syncthreads();
    const bool ok = s_ok;
    if (!ok) failed = true;
    for (int e = tid; e < TT; e += nthr) {
      Ajj[e] = sL[(e / TS) * LDT + e % TS];
      Di[(int64_t)J * TT + e] = sInv[(e / TS) * LDT + e % TS];
    }
    const int nr = envelope_rows(F, J, d.ntiles, rows, ROWCAP, &s_count);
    if (nr > ROWCAP) { failed = true; break; }
    // panel
    for (int a = wave; a < nr; a += nwaves) {
      T* Aij = A + tile_pos(F, off, rows[a], J) * TT;
      typename Mfma<T>::acc_t acc[4];
      tile_acc_zero<T>(acc);
      tile_mma_nt<T, false>(acc, Aij, TS, sInv, LDT, lane);
      tile_acc_store<T>(acc, Aij, TS, lane);
    }
    __syncthreads();
    // trailing update over pairs (a >= b) of envelope rows
    int item = 0;
    for (int a = 0; a < nr; ++a)
      for (int b = 0; b <= a; ++b, ++item) {
        if (item % nwaves != wave) continue;
        const int Ia = rows[a], Ib = rows[b];
        const T* La = A + tile_pos(F, off, Ia, J) * TT;
        const T* Lb = A + tile_pos(F, off, Ib, J) * TT;
        T* Cab = A + tile_pos(F, off, Ia, Ib) * TT;
        typename Mfma<T>::acc_t acc[4];
        tile_acc_load<T>(acc, Cab, TS, lane);
        tile_mma_nt<T, true>(acc, La, TS, Lb, TS, lane);
        tile_acc_store<T>(acc, Cab, TS, lane);
      }
    __syncthreads();
  }
  if (failed && tid == 0) atomicCAS(status, 0, blockIdx.x + 1);
}

template __global__ void k_chol_local<double>(const SubDesc*, const int32_t*, const int64_t*,
                                              double*, double*, int32_t*);

__global__ void k_to_float(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (float)src[k];
}

// loc_i = S_i R_i r (padding zero)
__global__ void __launch_bounds__(256)
k_gather_local(const SubDesc* __restrict__ subs, const int32_t* __restrict__ omega,
               const double* __restrict__ scale, const double* __restrict__ r,
               double* __restrict__ loc) {
  const SubDesc d = subs[blockIdx.x];
  const int32_t* om = omega + d.omega_off;
  for (int pos = threadIdx.x; pos < d.np; pos += blockDim.x) {
    double v = 0.0;
    if (pos < d.nI) v = r[om[pos]];
    else if (pos >= d.nIp && pos < d.nIp + d.nG) v = r[om[d.nI + pos - d.nIp]];
    loc[d.loc_off + pos] = scale[d.loc_off + pos] * v;
  }
}

// In-place solve L L^T y = loc_i with the tile-envelope factor and the
// inverted diagonal tiles: forward substitution by tile rows, backward
// substitution right-looking (y_K -= L(I,K)^T x_I).
//
// Subdomains with np <= YCAP keep y in LDS for both sweeps.  Each wave owns
// whole tiles: wave w takes tiles w, w + 4, ... of a tile row, so a tile's
// product needs one cross-lane step only.  Forward: lane (r, h) = (l % 32,
// l / 32) holds L(r, 16 h + j), j < 16, and sums its 16 columns; the two
// halves meet in one shuffle.  Backward: lane (c, h) holds the 16 contiguous
// entries L(16 h + j, c) and forms column c of L^T x the same way.  A wave
// loads its next chunk of tiles (which may lie rows ahead) into registers
// while it computes the current one; the factor does not depend on y.  The
// per-wave row partials are added in a fixed order, and the diagonal tile
// products run in wave 0: two block barriers per tile row and sweep.  Larger
// subdomains use a global-memory path with the same arithmetic.
constexpr int YCAP = 8192;
constexpr int SW = 4;                  // waves of the solve workgroup

template <typename T> struct SolveCfg;
template <> struct SolveCfg<float> { static constexpr int KW = 4; };
template <> struct SolveCfg<double> { static constexpr int KW = 2; };

template <typename T>
struct Chunk {
  T v[SolveCfg<T>::KW][16];
  int I, k0, n;                        // row, first tile index in the row, tiles held
};

// Next chunk of wave w at or after (row I, tile index k) in the given sweep
// direction: tiles k, k + SW, ... of row I with index < I - F(I); rows where
// the wave has no tile are skipped.  I = -1 (backward) or nt (forward) ends.
template <typename T>
__device__ inline void chunk_seek(Chunk<T>& C, const int32_t* sF, int nt, int I, int k, bool fwd) {
  constexpr int KW = SolveCfg<T>::KW;
  const int w = threadIdx.x / 64;
  while (I >= 0 && I < nt && k >= I - sF[I]) {
    I += fwd ? 1 : -1;
    k = w;
  }
  C.I = I;
  C.k0 = k;
  C.n = 0;
  if (I < 0 || I >= nt) return;
  const int nk = I - sF[I];
  C.n = min(KW, (nk - k + SW - 1) / SW);
}

template <typename T>
__device__ inline void chunk_load(Chunk<T>& C, const T* __restrict__ A, const int32_t* sF,
                                  const int64_t* sOff, bool fwd) {
  constexpr int KW = SolveCfg<T>::KW;
  if (C.n == 0) return;
  const int lane = threadIdx.x % 64, a = lane % 32, h = lane / 32;
  const T* row = A + sOff[C.I] * TT;          // tile (I, F(I))
#pragma unroll
  for (int q = 0; q < KW; ++q)
    if (q < C.n) {
      const T* t = row + (int64_t)(C.k0 + SW * q) * TT;
#pragma unroll
      for (int j = 0; j < 16; ++j) C.v[q][j] = fwd ? t[(16 * h + j) * TS + a] : t[a * TS + 16 * h + j];
    }
}

// wave 0: 16 elements per lane of a diagonal inverse tile, laid out like the
// off-diagonal tiles of the same sweep
template <typename T>
__device__ inline void dinv_load(T (&D)[16], const T* __restrict__ tile, int lane, bool fwd) {
  const int a = lane % 32, h = lane / 32;
#pragma unroll
  for (int j = 0; j < 16; ++j) D[j] = fwd ? tile[(16 * h + j) * TS + a] : tile[a * TS + 16 * h + j];
}

template <typename T>
__device__ void local_solve_lds(const SubDesc& d, const int32_t* F, const int64_t* off,
                                const T* __restrict__ A, const T* __restrict__ Di,
                                double* __restrict__ yg, double* ys, int32_t* sF, int64_t* sOff,
                                double (*part)[TS], double* sv) {
  constexpr int KW = SolveCfg<T>::KW;
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int a = lane % 32, h = lane / 32;
  const int nt = d.ntiles;
  for (int q = tid; q < d.np; q += blockDim.x) ys[q] = yg[q];
  for (int q = tid; q < nt; q += blockDim.x) { sF[q] = F[q]; sOff[q] = off[q]; }
  __syncthreads();
  Chunk<T> cur, nxt;
  T dcur[16], dnxt[16];

  // ---- forward: y_I = Dinv_I (y_I - sum_K L(I,K) y_K)
  chunk_seek(cur, sF, nt, 0, w, true);
  chunk_load(cur, A, sF, sOff, true);
  if (w == 0 && nt > 0) dinv_load(dcur, Di, lane, true);
  for (int I = 0; I < nt; ++I) {
    if (w == 0 && I + 1 < nt) dinv_load(dnxt, Di + (int64_t)(I + 1) * TT, lane, true);
    double acc = 0.0;
    while (cur.I == I) {
      chunk_seek(nxt, sF, nt, I, cur.k0 + SW * KW, true);
      chunk_load(nxt, A, sF, sOff, true);
      const int K0 = sF[I] + cur.k0;
#pragma unroll
      for (int q = 0; q < KW; ++q)
        if (q < cur.n) {
          const double* yk = ys + (K0 + SW * q) * TS + 16 * h;
#pragma unroll
          for (int j = 0; j < 16; ++j) acc += (double)cur.v[q][j] * yk[j];
        }
      cur = nxt;
    }
    acc += __shfl_xor(acc, 32, 64);
    if (lane < TS) part[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
      if (lane < TS) {
        double s = ys[I * TS + lane];
        for (int q = 0; q < SW; ++q) s -= part[q][lane];
        sv[lane] = s;
      }
      wave_sync();
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) t += (double)dcur[j] * sv[16 * h + j];
      t += __shfl_xor(t, 32, 64);
      if (lane < TS) ys[I * TS + lane] = t;
#pragma unroll
      for (int j = 0; j < 16; ++j) dcur[j] = dnxt[j];
    }
    __syncthreads();
  }

  // ---- backward: x_I = Dinv_I^T y_I, then y_K -= L(I,K)^T x_I
  chunk_seek(cur, sF, nt, nt - 1, w, false);
  chunk_load(cur, A, sF, sOff, false);
  if (w == 0 && nt > 0) dinv_load(dcur, Di + (int64_t)(nt - 1) * TT, lane, false);
  for (int I = nt - 1; I >= 0; --I) {
    if (w == 0) {
      if (I > 0) dinv_load(dnxt, Di + (int64_t)(I - 1) * TT, lane, false);
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) t += (double)dcur[j] * ys[I * TS + 16 * h + j];
      t += __shfl_xor(t, 32, 64);
      wave_sync();
      if (lane < TS) ys[I * TS + lane] = t;
#pragma unroll
      for (int j = 0; j < 16; ++j) dcur[j] = dnxt[j];
    }
    __syncthreads();
    double xr[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) xr[j] = ys[I * TS + 16 * h + j];
    while (cur.I == I) {
      chunk_seek(nxt, sF, nt, I, cur.k0 + SW * KW, false);
      chunk_load(nxt, A, sF, sOff, false);
      const int K0 = sF[I] + cur.k0;
#pragma unroll
      for (int q = 0; q < KW; ++q)
        if (q < cur.n) {
          double v = 0.0;
#pragma unroll
          for (int j = 0; j < 16; ++j) v += (double)cur.v[q][j] * xr[j];
          v += __shfl_xor(v, 32, 64);
          if (lane < TS) ys[(K0 + SW * q) * TS + lane] -= v;
        }
      cur = nxt;
    }
    __syncthreads();
  }
  for (int q = tid; q < d.np; q += blockDim.x) yg[q] = ys[q];
}

template <typename T>
__global__ void __launch_bounds__(256)
k_local_solve(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
              const int64_t* __restrict__ tileOff, const T* __restrict__ fac,
              const T* __restrict__ dinv, double* __restrict__ loc) {
  __shared__ double part[8][TS];
  __shared__ double sv[TS];
  __shared__ double ys[YCAP];
  __shared__ int32_t sF[YCAP / TS];
  __shared__ int64_t sOff[YCAP / TS];
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  const T* A = fac + d.fac_off;
  const T* Di = dinv + d.dinv_off;
  double* y = loc + d.loc_off;
  if (d.np <= YCAP) {
    local_solve_lds<T>(d, F, off, A, Di, y, ys, sF, sOff, part, sv);
    return;
  }
  const int tid = threadIdx.x;
  const int r = tid % TS, g = tid / TS, ng = blockDim.x / TS;
  for (int I = 0; I < d.ntiles; ++I) {
    double acc = 0.0;
    for (int K = F[I] + g; K < I; K += ng) {
      const T* t = A + (off[I] + (K - F[I])) * TT;
      const double* yk = y + K * TS;
#pragma unroll 8
      for (int c = 0; c < TS; ++c) acc += (double)t[c * TS + r] * yk[c];
    }
    part[g][r] = acc;
    __syncthreads();
    if (tid < TS) {
      double s = y[I * TS + tid];
      for (int q = 0; q < ng; ++q) s -= part[q][tid];
      sv[tid] = s;
    }
    __syncthreads();
    if (tid < TS) {
      const T* inv = Di + (int64_t)I * TT;
      double s = 0.0;
#pragma unroll 8
      for (int c = 0; c < TS; ++c) s += (double)inv[c * TS + tid] * sv[c];
      y[I * TS + tid] = s;
    }
    __syncthreads();
  }
  for (int I = d.ntiles - 1; I >= 0; --I) {
    if (tid < TS) {
      const T* inv = Di + (int64_t)I * TT;
      double s = 0.0;
#pragma unroll 8
      for (int c = 0; c < TS; ++c) s += (double)inv[tid * TS + c] * y[I * TS + c];
      sv[tid] = s;
    }
    __syncthreads();
    if (tid < TS) y[I * TS + tid] = sv[tid];
    for (int K = F[I] + g; K < I; K += ng) {
      const T* t = A + (off[I] + (K - F[I])) * TT;
      double s = 0.0;
#pragma unroll 8
      for (int rr = 0; rr < TS; ++rr) s += (double)t[r * TS + rr] * sv[rr];
      y[K * TS + r] -= s;
    }
    __syncthreads();
  }
}

template __global__ void k_local_solve<double>(const SubDesc*, const int32_t*, const int64_t*,
                                               const double*, const double*, double*);
template __global__ void k_local_solve<float>(const SubDesc*, const int32_t*, const int64_t*,
                                              const float*, const float*, double*);

// z_j = sum over the subdomains holding column j of S_pos loc_pos (fixed
// order), plus the coarse prolongation X_i d_i on the interior of its owner.
__global__ void k_scatter_local(int32_t n, const int32_t* __restrict__ own_ptr,
                                const int32_t* __restrict__ own_pos, const double* __restrict__ scale,
                                const double* __restrict__ loc, const int32_t* __restrict__ part,
                                const int32_t* __restrict__ locown, const SubDesc* __restrict__ subs,
                                const double* __restrict__ X, const double* __restrict__ dcoarse,
                                double* __restrict__ z) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int q = own_ptr[j]; q < own_ptr[j + 1]; ++q) {
    const int pos = own_pos[q];
    s += scale[pos] * loc[pos];
  }
  if (dcoarse != nullptr) {
    const SubDesc d = subs[part[j]];
    const int a = locown[j];
    const double* xr = X + d.x_off + a;
    const double* dc = dcoarse + d.cg_off;
    double c = 0.0;
    for (int k = 0; k < d.p; ++k) c += xr[(int64_t)k * d.nIp] * dc[k];
    s += c;
  }
  z[j] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_gather_values(hipStream_t st, int64_t nnz, const int32_t* perm, const double* src,
                          double* dst) {
  if (nnz == 0) return;
  k_gather_values<<<(unsigned)((nnz + 255) / 256), 256, 0, st>>>(nnz, perm, src, dst);
}

void launch_assemble(hipStream_t st, int nsub, const DevPlan& P, const DevMatrix& M, double* fac,
                     double* ctg) {
  k_assemble<<<nsub, 256, 0, st>>>(P.subs, P.omega, P.part, P.locown, M.rowptr, M.colind, M.vals,
                                   M.trowptr, M.trow, M.tvals, P.tileF, P.tileOff, fac, ctg);
}

void launch_equilibrate(hipStream_t st, int nsub, const DevPlan& P, double* fac, double* ctg,
                        double* scale) {
  k_equil_scale<<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, scale);
  k_equil_apply<<<dim3(nsub, 32), 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, ctg, scale);
}

void launch_chol_local(hipStream_t st, int nsub, const DevPlan& P, double* fac, double* dinv,
                       int32_t* status) {
  k_chol_local<double><<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, dinv, status);
}

void launch_to_float(hipStream_t st, int64_t n, const double* src, float* dst) {
  if (n == 0) return;
  k_to_float<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, src, dst);
}

void launch_gather_local(hipStream_t st, int nsub, const DevPlan& P, const double* scale,
                         const double* r, double* loc) {
  k_gather_local<<<nsub, 256, 0, st>>>(P.subs, P.omega, scale, r, loc);
}

void launch_local_solve(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                        const double* dinv, double* loc) {
  k_local_solve<double><<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, dinv, loc);
}

void launch_local_solve_f32(hipStream_t st, int nsub, const DevPlan& P, const float* fac,
                            const float* dinv, double* loc) {
  k_local_solve<float><<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, dinv, loc);
}

void launch_scatter_local(hipStream_t st, int32_t n, const DevPlan& P, const double* scale,
                          const double* loc, const double* X, const double* dcoarse, double* z) {
  if (n == 0) return;
  k_scatter_local<<<(n + 255) / 256, 256, 0, st>>>(n, P.own_ptr, P.own_pos, scale, loc, P.part,
                                                   P.locown, P.subs, X, dcoarse, z);
}

}  // namespace lsq2l
