// Per-iteration local solves of the preconditioner: L L^T y = loc_i for every
// subdomain with its tile-envelope factor (Algorithm 1, the local terms of
// eq. (two_level_schwarz)), in FP64 or with the FP32 copy of the factor.
#include "kernels.hpp"

namespace lsq2l {

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

void launch_local_solve(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                        const double* dinv, double* loc) {
  k_local_solve<double><<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, dinv, loc);
}

void launch_local_solve_f32(hipStream_t st, int nsub, const DevPlan& P, const float* fac,
                            const float* dinv, double* loc) {
  k_local_solve<float><<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, dinv, loc);
}

}  // namespace lsq2l
