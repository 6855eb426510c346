// Per-iteration local solves of the preconditioner: L L^T y = loc_i for every
// subdomain with its tile-envelope factor (Algorithm 1, the local terms of
// eq. (two_level_schwarz)), with FP64 or FP32 factors.
#include <type_traits>

#include "kernels.hpp"

namespace lsq2l {

// Where position q of a subdomain's solve layout lives in the local vectors
// loc: with a permutation sp (the subdomain's slice of the solve layout's
// map, -1 on padding) at loc[sp[q]], else at loc[loc_off + q].
__device__ inline int64_t solve_pos(const int32_t* sp, int64_t loc_off, int q) {
  return sp ? (int64_t)sp[q] : loc_off + q;
}

// ---------------------------------------------------------------------------
// Streaming variant, in two size bins.  The tiles a sweep reads form one
// stream: forward, row by row, the off-diagonal tiles (I, F(I)) ..
// (I, I - 1) followed by the diagonal inverse of row I; the backward sweep
// reads the same stream in reverse.  Since tile rows are stored one after
// the other (F(I) .. I each), stream position t is factor tile t of the
// subdomain, except that the last position of each row, where the diagonal
// block sits, is served from the inverse.
//
// Waves 1..3 (producers) copy the stream in blocks of PB tiles into a
// two-block LDS ring, with PD more blocks in flight in their registers.
// Their global loads are fully coalesced (each instruction reads 1 KiB of
// one tile).  Wave 0 (consumer) does all the arithmetic: it owns every row,
// so no partial sums cross waves.  The LDS copy of a tile is row-major in
// the forward sweep and column-major in the backward sweep, so that in both
// lane (a, h) = (l % 32, l / 32) reads 16 consecutive entries with vector
// loads: forward L(a, 16 h .. 16 h + 15) for row a of L y, backward
// L(16 h .. 16 h + 15, a) for column a of L^T x.  A swap of the wave's
// halves joins h = 0, 1.  Producer and consumer loops execute the same
// number of block barriers.  The consumer computes in the factor's own type:
// with the FP32 factor, the sweeps, their partial sums and the local vector
// held in LDS are FP32 (the result is widened to FP64 on the way out).
//
// Both bins run in one launch, workgroups in decreasing order of stream
// length (the largest subdomains start first).  y lives in LDS: up to
// PCAP_S local unknowns with a ring of PB tiles per block, up to PCAP_B with
// a ring of PB_BIG tiles, in the same dynamic LDS allocation.
// ---------------------------------------------------------------------------
constexpr int PCAP = 4608;            // small bin
constexpr int PCAP_B = 12544;         // large bin
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct PipeCfg;
template <> struct PipeCfg<float> {
  static constexpr int PB = 12, PB_BIG = 9, PD = 2;
  using V = f32x4;
};
template <> struct PipeCfg<double> {
  static constexpr int PB = 7, PB_BIG = 3, PD = 2;
  using V = f64x2;
};
template <int V> using IC = std::integral_constant<int, V>;
template <int B, int E, typename Fn>
__device__ inline void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(IC<B>{});
    static_for<B + 1, E>(fn);
  }
}

// 16 consecutive LDS entries of a tile, converted to R
template <typename T, typename R>
__device__ inline void lds_row16(R (&x)[16], const T* p) {
  using V = typename PipeCfg<T>::V;                  // 16-byte vector of T
  constexpr int NV = 16 * sizeof(T) / sizeof(V);
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const V v = reinterpret_cast<const V*>(p)[c];
    const T* e = reinterpret_cast<const T*>(&v);
#pragma unroll
    for (int i = 0; i < 16 / NV; ++i) x[c * (16 / NV) + i] = (R)e[i];
  }
}

// LDS layout of one bin: y (YC entries), the ring (2 PB tiles of TL
// entries), the envelope starts sF and stream offsets sS of the tile rows,
// and a 32-entry row buffer
template <typename T, int PB, int YC>
struct PipeLds {
  static constexpr int EV = sizeof(typename PipeCfg<T>::V) / sizeof(T);
  static constexpr int TL = TS * (TS + EV);
  static constexpr size_t ys = 0;
  static constexpr size_t ring = ys + (size_t)YC * sizeof(T);
  static constexpr size_t sF = ring + (size_t)2 * PB * TL * sizeof(T);
  static constexpr size_t sS = sF + (size_t)(YC / TS) * sizeof(int32_t);
  static constexpr size_t sv = (sS + (size_t)(YC / TS + 1) * sizeof(int32_t) + 15) / 16 * 16;
  static constexpr size_t bytes = sv + TS * sizeof(T);
};

template <typename T>
constexpr size_t pipe_lds_bytes() {
  constexpr size_t a = PipeLds<T, PipeCfg<T>::PB, PCAP>::bytes;
  constexpr size_t b = PipeLds<T, PipeCfg<T>::PB_BIG, PCAP_B>::bytes;
  return a > b ? a : b;
}
static_assert(pipe_lds_bytes<float>() <= 160 * 1024, "LDS of the FP32 local solve");
static_assert(pipe_lds_bytes<double>() <= 160 * 1024, "LDS of the FP64 local solve");

template <typename T, int PB, int YC>
__device__ __forceinline__ void local_solve_pipe_body(const SubDesc& d, const int32_t* __restrict__ tileF,
                                                      const T* __restrict__ fac,
                                                      const T* __restrict__ dinv,
                                                      double* __restrict__ loc,
                                                      const int32_t* __restrict__ sp,
                                                      unsigned char* smem) {
  using V = typename PipeCfg<T>::V;
  using GV = __attribute__((address_space(1))) V;   // global memory: loads count against vmcnt only
  using LY = PipeLds<T, PB, YC>;
  constexpr int PD = PipeCfg<T>::PD;
  constexpr int EV = LY::EV;                         // entries per vector
  constexpr int NC = TT / EV / 64;                   // vectors per lane and tile
  constexpr int PLD = TS + EV;                       // LDS leading dimension of a tile
  constexpr int TL = LY::TL;
  constexpr int PW = (PB + 2) / 3;                   // tiles per producer wave and block
  constexpr int CB = 4;                              // consumer batch of off-diagonal tiles
  T* ys = reinterpret_cast<T*>(smem + LY::ys);
  T* ring = reinterpret_cast<T*>(smem + LY::ring);
  int32_t* sF = reinterpret_cast<int32_t*>(smem + LY::sF);
  int32_t* sS = reinterpret_cast<int32_t*>(smem + LY::sS);
  T* sv = reinterpret_cast<T*>(smem + LY::sv);
  const int32_t* F = tileF + d.tile_base;
  const T* A = fac + d.fac_off;
  const T* Di = dinv + d.dinv_off;
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int a = lane % 32, h = lane / 32;
  const int nt = d.ntiles;
  for (int q = tid; q < d.np; q += blockDim.x) {
    const int64_t ix = solve_pos(sp, d.loc_off, q);
    ys[q] = ix >= 0 ? (T)loc[ix] : T(0);
  }
  for (int q = tid; q < nt; q += blockDim.x) sF[q] = F[q];
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int I = 0; I < nt; ++I) { sS[I] = acc; acc += I - sF[I] + 1; }
    sS[nt] = acc;
  }
  __syncthreads();
  const int N = sS[nt];                              // stream length
  const int nblk = (N + PB - 1) / PB;

  // ---- producers.  The walk over the stream keeps the row (wI) and its
  // first and one-past-last positions, reading sS once per row.
  int wI = 0, wlo = 0, whi = 0;
  V vals[PD][PW][NC];
  bool have[PD][PW];
  // fetch<r>(b): block b into register slot r
  auto fetch = [&](int b, bool rev, auto slot) {
    constexpr int r = decltype(slot)::value;
    const int pw = w - 1;
    const T* src[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      src[q] = A;
      have[r][q] = false;
    }
#pragma unroll
    for (int j = 0; j < PB; ++j) {
      const int pos = b * PB + j;
      if (pos < N) {
        const int t = rev ? N - 1 - pos : pos;
        if (rev) {
          while (t < wlo) { --wI; whi = wlo; wlo = sS[wI]; }
        } else {
          while (t >= whi) { ++wI; wlo = whi; whi = sS[wI + 1]; }
        }
        if (j % 3 == pw) {
          src[j / 3] = t == whi - 1 ? Di + (int64_t)wI * TT : A + (int64_t)t * TT;
          have[r][j / 3] = true;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < PW; ++q) {
      if (have[r][q]) {
        const GV* v = (const GV*)src[q] + lane;
#pragma unroll
        for (int c = 0; c < NC; ++c) vals[r][q][c] = v[64 * c];
      }
    }
  };
  // commit<r>(buf): register slot r into ring block buf; vector c of lane l
  // holds the EV entries from flat (column-major) index EV (l + 64 c)
  auto commit = [&](int buf, bool rev, auto slot) {
    constexpr int r = decltype(slot)::value;
    const int pw = w - 1;
#pragma unroll
    for (int q = 0; q < PW; ++q)
      if (have[r][q]) {
        T* tile = ring + (size_t)(buf * PB + pw + 3 * q) * TL;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int f0 = EV * (lane + 64 * c), col = f0 / TS, row = f0 % TS;
          if (rev) {
            *reinterpret_cast<V*>(tile + col * PLD + row) = vals[r][q][c];
          } else {
            const T* e = reinterpret_cast<const T*>(&vals[r][q][c]);
#pragma unroll
            for (int i = 0; i < EV; ++i) tile[(row + i) * PLD + col] = e[i];
          }
        }
      }
  };
  // one sweep of the producers: block 0 to the ring, blocks 1 .. PD in
  // flight; during block b, block b + 1 goes to the ring and block
  // b + 1 + PD is fetched into the register slot it freed
  auto producer_sweep = [&](bool rev) {
    wI = rev ? nt - 1 : 0;
    wlo = nt > 0 ? sS[wI] : 0;
    whi = nt > 0 ? sS[wI + 1] : 0;
    fetch(0, rev, IC<0>{});
    commit(0, rev, IC<0>{});
    static_for<1, PD + 1>([&](auto i) {
      if (decltype(i)::value < nblk) fetch(decltype(i)::value, rev, IC<decltype(i)::value % PD>{});
    });
    __syncthreads();
    for (int b0 = 0; b0 < nblk; b0 += PD) {
      static_for<0, PD>([&](auto i) {
        constexpr int r = (decltype(i)::value + 1) % PD;
        const int b = b0 + decltype(i)::value;
        if (b < nblk) {
          if (b + 1 < nblk) {
            commit((b + 1) & 1, rev, IC<r>{});
            if (b + 1 + PD < nblk) fetch(b + 1 + PD, rev, IC<r>{});
          }
          __syncthreads();
        }
      });
    }
  };

  // ---- forward sweep: y_I = Dinv_I (y_I - sum_K L(I,K) y_K).  Wave 0 keeps
  // the row (I, F(I), its number nk of off-diagonal tiles) and the next tile
  // index k in registers and takes the off-diagonal tiles of a block as one
  // run, with four independent partial sums per lane.
  if (w > 0) {
    producer_sweep(false);
  } else {
    __syncthreads();
    int I = 0, k = 0, fI = nt > 0 ? sF[0] : 0, nk = 0;
    T acc[4] = {0, 0, 0, 0};
    for (int b = 0; b < nblk; ++b) {
      const T* rb = ring + (size_t)(b & 1) * PB * TL;
      const int send = min(N - b * PB, PB);
      int s = 0;
      while (s < send && I < nt) {
        const int run = min(nk - k, send - s);
        const T* yk = ys + (fI + k) * TS + 16 * h;
        // batches of CB tiles: all LDS reads of a batch issue before its FMAs
        auto fwd_batch = [&](int u0, auto nbc) {
          constexpr int nb = decltype(nbc)::value;
          T l[nb][16], y[nb][16];
#pragma unroll
          for (int i = 0; i < nb; ++i) {
            lds_row16(l[i], rb + (size_t)(s + u0 + i) * TL + a * PLD + 16 * h);
            lds_row16(y[i], yk + (u0 + i) * TS);
          }
#pragma unroll
          for (int i = 0; i < nb; ++i)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[j & 3] += l[i][j] * y[i][j];
        };
        int u = 0;
        for (; u + CB <= run; u += CB) fwd_batch(u, IC<CB>{});
        for (; u < run; ++u) fwd_batch(u, IC<1>{});
        s += run;
        k += run;
        if (s < send) {                              // the diagonal inverse of row I
          T l[16];
          lds_row16(l, rb + (size_t)s * TL + a * PLD + 16 * h);
          T r = (acc[0] + acc[1]) + (acc[2] + acc[3]);
          r = half_pair_sum(r);
          if (lane < TS) sv[lane] = ys[I * TS + lane] - r;
          wave_sync();
          T v[4] = {0, 0, 0, 0};
#pragma unroll
          for (int j = 0; j < 16; ++j) v[j & 3] += l[j] * sv[16 * h + j];
          T x = (v[0] + v[1]) + (v[2] + v[3]);
          x = half_pair_sum(x);
          wave_sync();
          if (lane < TS) ys[I * TS + lane] = x;
          wave_sync();
          ++s;
          ++I;
          k = 0;
          if (I < nt) { fI = sF[I]; nk = I - fI; }
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = 0.0;
        }
      }
      __syncthreads();
    }
  }

  // ---- backward sweep, the stream in reverse: x_I = Dinv_I^T y_I, then
  // y_K -= L(I,K)^T x_I over the off-diagonal tiles of row I, K = F(I) + k
  // for k = nk - 1 .. 0 (k = nk stands for the diagonal inverse).
  if (w > 0) {
    producer_sweep(true);
  } else {
    __syncthreads();
    int I = nt - 1, fI = nt > 0 ? sF[nt - 1] : 0;
    int nk = nt > 0 ? I - fI : 0, k = nk;
    T xr[16];
    for (int b = 0; b < nblk; ++b) {
      const T* rb = ring + (size_t)(b & 1) * PB * TL;
      const int send = min(N - b * PB, PB);
      int s = 0;
      while (s < send) {
        if (k == nk) {
          T l[16];
          lds_row16(l, rb + (size_t)s * TL + a * PLD + 16 * h);
          T v[4] = {0, 0, 0, 0};
#pragma unroll
          for (int j = 0; j < 16; ++j) v[j & 3] += l[j] * ys[I * TS + 16 * h + j];
          T x = (v[0] + v[1]) + (v[2] + v[3]);
          x = half_pair_sum(x);
          wave_sync();
          if (lane < TS) ys[I * TS + lane] = x;
          wave_sync();
#pragma unroll
          for (int j = 0; j < 16; ++j) xr[j] = ys[I * TS + 16 * h + j];
          ++s;
          --k;
        } else {
          const int run = min(k + 1, send - s);
          auto bwd_batch = [&](int u0, auto nbc) {
            constexpr int nb = decltype(nbc)::value;
            T l[nb][16], x[nb];
#pragma unroll
            for (int i = 0; i < nb; ++i) lds_row16(l[i], rb + (size_t)(s + u0 + i) * TL + a * PLD + 16 * h);
#pragma unroll
            for (int i = 0; i < nb; ++i) {
              T v[4] = {0, 0, 0, 0};
#pragma unroll
              for (int j = 0; j < 16; ++j) v[j & 3] += l[i][j] * xr[j];
              x[i] = (v[0] + v[1]) + (v[2] + v[3]);
            }
#pragma unroll
            for (int i = 0; i < nb; ++i) x[i] = half_pair_sum(x[i]);
#pragma unroll
            for (int i = 0; i < nb; ++i)
              if (lane < TS) ys[(fI + k - u0 - i) * TS + lane] -= x[i];
          };
          int u = 0;
          for (; u + CB <= run; u += CB) bwd_batch(u, IC<CB>{});
          for (; u < run; ++u) bwd_batch(u, IC<1>{});
          s += run;
          k -= run;
        }
        if (k < 0) {                                 // row I done: move to row I - 1
          if (I == 0) break;
          wave_sync();
          --I;
          fI = sF[I];
          nk = I - fI;
          k = nk;
        }
      }
      __syncthreads();
    }
  }
  for (int q = tid; q < d.np; q += blockDim.x) {
    const int64_t ix = solve_pos(sp, d.loc_off, q);
    if (ix >= 0) loc[ix] = ys[q];
  }
}

// Workgroup b solves subdomain order[b] (decreasing stream length) in the
// bin its size selects; subdomains above PCAP_B are left to k_local_solve.
template <typename T>
__global__ void __launch_bounds__(256)
k_local_solve_pipe(const SubDesc* __restrict__ subs, const int32_t* __restrict__ order,
                   const int32_t* __restrict__ tileF, const T* __restrict__ fac,
                   const T* __restrict__ dinv, double* __restrict__ loc,
                   const int32_t* __restrict__ sperm) {
  extern __shared__ __align__(16) unsigned char smem[];
  const SubDesc d = subs[order[blockIdx.x]];
  const int32_t* sp = sperm ? sperm + d.loc_off : nullptr;
  if (d.np <= PCAP)
    local_solve_pipe_body<T, PipeCfg<T>::PB, PCAP>(d, tileF, fac, dinv, loc, sp, smem);
  else if (d.np <= PCAP_B)
    local_solve_pipe_body<T, PipeCfg<T>::PB_BIG, PCAP_B>(d, tileF, fac, dinv, loc, sp, smem);
}

// Subdomains above PCAP_B local unknowns: forward and backward substitution
// by tile rows with y in global memory, workgroup per subdomain, 32 rows of
// threads each summing every eighth tile of a row (fixed order), the
// diagonal blocks applied through their inverses.
template <typename T>
__global__ void __launch_bounds__(256)
k_local_solve(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
              const int64_t* __restrict__ tileOff, const T* __restrict__ fac,
              const T* __restrict__ dinv, double* __restrict__ loc,
              const int32_t* __restrict__ sperm, double* __restrict__ scratch) {
  __shared__ double part[8][TS];
  __shared__ double sv[TS];
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  const T* A = fac + d.fac_off;
  const T* Di = dinv + d.dinv_off;
  if (d.np <= PCAP_B) return;               // done by k_local_solve_pipe
  const int32_t* sp = sperm ? sperm + d.loc_off : nullptr;
  // y in global memory: in place in loc, or, for a permuted layout, in the
  // subdomain's slice of scratch
  double* y = sp ? scratch + d.loc_off : loc + d.loc_off;
  const int tid = threadIdx.x;
  if (sp) {
    for (int q = tid; q < d.np; q += blockDim.x) y[q] = sp[q] >= 0 ? loc[sp[q]] : 0.0;
    __syncthreads();
  }
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
  if (sp)
    for (int q = tid; q < d.np; q += blockDim.x)
      if (sp[q] >= 0) loc[sp[q]] = y[q];
}

template __global__ void k_local_solve<double>(const SubDesc*, const int32_t*, const int64_t*,
                                               const double*, const double*, double*,
                                               const int32_t*, double*);
template __global__ void k_local_solve<float>(const SubDesc*, const int32_t*, const int64_t*,
                                              const float*, const float*, double*,
                                              const int32_t*, double*);

void launch_local_solve(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                        const double* dinv, double* loc) {
  k_local_solve_pipe<double><<<nsub, 256, pipe_lds_bytes<double>(), st>>>(
      P.subs, P.solve_order, P.tileF, fac, dinv, loc, P.sperm);
  if (P.max_np > PCAP_B)
    k_local_solve<double><<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, dinv, loc,
                                                 P.sperm, P.yscratch);
}

void launch_local_solve_f32(hipStream_t st, int nsub, const DevPlan& P, const float* fac,
                            const float* dinv, double* loc) {
  k_local_solve_pipe<float><<<nsub, 256, pipe_lds_bytes<float>(), st>>>(
      P.subs, P.solve_order, P.tileF, fac, dinv, loc, P.sperm);
  if (P.max_np > PCAP_B)
    k_local_solve<float><<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, dinv, loc,
                                                P.sperm, P.yscratch);
}

hipError_t local_solve_configure() {
  hipError_t e = hipFuncSetAttribute((const void*)k_local_solve_pipe<double>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)pipe_lds_bytes<double>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_local_solve_pipe<float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)pipe_lds_bytes<float>());
  return e;
}

}  // namespace lsq2l
