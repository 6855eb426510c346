// Local factors and interface factors from thin QR factorizations, without
// forming C_ii (Remark 3.1, Section 3.1; Remark 3.2, Section 3.3.2).
//
// R of A(rows, Omega_i) S (S the column scaling of the equilibration, so
// that R^T R is the equilibrated C_ii) is built by merging the rows of A into
// R, QB rows at a time, tile column by tile column: for the block B of rows
// and the tile column J of its first nonzero,
//     [R(J, J) R(J, K...)]          [R'(J, J) R'(J, K...)]
//     [B(:, J) B(:, K...)]  <-  Q^T [   0     B'(:, K...)]
// with Q the product of the 32 Householder reflectors that zero B(:, J)
// against the triangle R(J, J) (the LAPACK reflector convention: beta =
// -sign(alpha) ||x||, tau = (beta - alpha) / beta).  The tiles K are the
// tile rows of the envelope that reach column J (F(K) <= J): a row of B that
// is nonzero in tile K when tile J is eliminated either had an entry there
// (coupling columns J and K in C_ii) or received it from a row of R, so R
// stays inside the envelope of C_ii that the Cholesky factor uses, and L =
// R^T is written over the same layout.  The block is done when no tile of it
// is nonzero.  At the end the rows of R get a positive diagonal (then L is
// the Cholesky factor of the equilibrated C_ii) and the diagonal tiles of L
// are inverted for the triangular solves.
//
// Three uses (one workgroup per subdomain):
//   QR_SEL    rows Xi_i in the [Omega_Ii, Omega_Gamma_i] layout, interior
//             tile columns only: L_I and L_GI, what the coarse selection and
//             the coarse basis read (rows outside Xi_i have no interior entry
//             and do not change them);
//   QR_SOLVE  every row of A with an entry in Omega_i, in the solve layout
//             of each subdomain (global column order or [I, Gamma]): the
//             factor of C_ii the local solves read;
//   QR_GAMMA  rows Xi_i restricted to Omega_Gamma_i into a dense n_G x n_G
//             upper triangle R_G (column-major, ld nGp, in the interface
//             work matrix): R_G^T R_G = Ct_GG, the input of the
//             principal-angle selection.
// Rows enter in the order of their first position in the layout (found
// through the columns of A^T, no sort), as in Givens row merging: R is then
// still empty past the rows merged so far, and a block stops within a few
// tiles of where it starts.
// The rows of a block live in a per-subdomain strip of QB x np doubles in
// global memory (position-major, QB rows contiguous), which is all zero
// between blocks: every tile a block touches is zeroed when it is eliminated
// (or, for QR_SEL, at the end of the block).
#include <climits>

#include "kernels.hpp"

namespace lsq2l {

namespace {

constexpr int QB = QR_STRIP_ROWS;   // rows merged per block
constexpr int QR_THREADS = 256;   // four waves; lane (kc, h): column kc, rows 16 h .. 16 h + 15
constexpr int QR_TMAX = 1024;     // tiles per side held in LDS (32,768 positions)
constexpr int QR_CH = 512;        // rows of the stream buffered in LDS

// 1 / x from the hardware estimate and two Newton steps (a few units in the
// last place, in a fraction of a division's latency)
__device__ inline double rcp2(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// sum of a[q] b[q] over 16 entries in four independent chains
__device__ inline double dot16(const double* a, const double* b, double init) {
  double p0 = init, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
  for (int q = 0; q < 16; q += 4) {
    p0 = fma(a[q], b[q], p0);
    p1 = fma(a[q + 1], b[q + 1], p1);
    p2 = fma(a[q + 2], b[q + 2], p2);
    p3 = fma(a[q + 3], b[q + 3], p3);
  }
  return (p0 + p1) + (p2 + p3);
}

// exclusive scan of v over the 256 threads, total in *tot
__device__ inline int block_scan_256(int v, int* sh, int* tot) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  int before = 0, all = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) before += sh[w];
    all += sh[w];
  }
  __syncthreads();
  *tot = all;
  return before + x - v;
}

}  // namespace

template <int MODE>
__global__ void __launch_bounds__(QR_THREADS)
k_qr_local(const SubDesc* __restrict__ subs, const SubDesc* __restrict__ psubs,
           const int32_t* __restrict__ tileF, const int64_t* __restrict__ tileOff,
           const int32_t* __restrict__ omega, int32_t* __restrict__ qscr, int64_t qcol_off,
           const int32_t* __restrict__ part, const int32_t* __restrict__ locown,
           const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
           const double* __restrict__ vals, const int32_t* __restrict__ trowptr,
           const int32_t* __restrict__ trow, const int32_t* __restrict__ inv,
           const double* __restrict__ scale, double* __restrict__ out,
           double* __restrict__ dinv, double* __restrict__ strip, int32_t* __restrict__ status) {
  __shared__ double sV[TS * LDT];         // reflector c: sV[c * QB + row]; the inverse tile at the end
  __shared__ double sTau[TS], sSgn[TS];
  __shared__ double sX[TS * LDT];
  double* const sInv = sV;
  __shared__ int32_t sF[QR_TMAX], sO[QR_TMAX], sGen[QR_TMAX], sRows[QR_TMAX], sBuf[QR_CH];
  __shared__ uint8_t sNZ[QR_TMAX];       // tile of the list left nonzero in the block
  __shared__ int s_jmin, s_jmax, s_count, s_fail, s_q;
  __shared__ int s_scan[4];
  const SubDesc d = subs[blockIdx.x];
  const SubDesc pd = psubs[d.id];
  const int i = d.id;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64, kc = lane & 31, h = lane >> 5;
  const int32_t* om = omega + pd.omega_off;
  const int32_t* G = om + pd.nI;
  // layout written: tiles per side, interior tiles, the envelope (dense for QR_GAMMA)
  const int ntiles = MODE == QR_GAMMA ? pd.nGp / TS : d.ntiles;
  const int ntI = MODE == QR_GAMMA ? 0 : d.ntI;
  const int ld = pd.nGp;
  if (ntiles > QR_TMAX) {
    if (tid == 0) atomicCAS(status, 0, i + 1);
    return;
  }
  if (MODE != QR_GAMMA)
    for (int I = tid; I < ntiles; I += QR_THREADS) {
      sF[I] = tileF[d.tile_base + I];
      sO[I] = (int32_t)tileOff[d.tile_base + I];
    }
  for (int I = tid; I < ntiles; I += QR_THREADS) sGen[I] = -1;
  if (tid == 0) s_fail = 0;
  double* Lf = MODE == QR_GAMMA ? out + pd.g_off : out + d.fac_off;
  double* Di = MODE == QR_GAMMA ? nullptr : dinv + d.dinv_off;
  double* Bs = strip + (int64_t)QB * pd.loc_off;
  // element (c, kk) of R(J, K) (row 32 J + c, column 32 K + kk) is base[c * sc + kk * sk]
  auto rtile = [&](int J, int K) -> double* {
    if (MODE == QR_GAMMA) return Lf + (int64_t)(K * TS) * ld + J * TS;
    return Lf + ((int64_t)sO[K] + (J - sF[K])) * TT;
  };
  const int sc = MODE == QR_GAMMA ? 1 : TS, sk = MODE == QR_GAMMA ? ld : 1;
  // position of a global column in the layout written, -1 if not there
  auto layout_pos = [&](int c, int* posP) -> int {
    const int p = local_pos(i, c, part, locown, G, pd.nG, pd.nIp);
    *posP = p;
    if (p < 0) return -1;
    if (MODE == QR_GAMMA) return p >= pd.nIp ? p - pd.nIp : -1;
    if (MODE == QR_SOLVE && d.spare) return inv[pd.loc_off + p];
    return p;
  };
  // ---- the row stream: rows ordered by their first position in the layout
  // (the order of Givens row merging; a row that arrives after R has filled
  // behind it would carry its fill down every remaining tile).  Candidate t
  // is entry t - qpre[q] of column col_at(q) of A^T; a row is taken at the
  // position q where it starts.  QR_SEL: rows of Xi_i (they start at an
  // interior position); QR_GAMMA: rows of Xi_i by their first interface
  // column; QR_SOLVE: every row with an entry in Omega_i.
  const int npos = MODE == QR_SEL ? pd.nI : MODE == QR_GAMMA ? pd.nG : d.np;
  int32_t* qpre = qscr + pd.loc_off + d.id;       // npos + 1 entries
  int32_t* qcol = qscr + qcol_off + pd.loc_off;   // QR_SOLVE, global order: column at each position
  if (MODE == QR_SOLVE && d.spare) {
    for (int p = tid; p < pd.np; p += QR_THREADS) {
      const int q = inv[pd.loc_off + p];
      if (q >= 0) qcol[q] = p < pd.nI ? om[p] : G[p - pd.nIp];
    }
    __syncthreads();
  }
  auto col_at = [&](int q) -> int {
    if (MODE == QR_SEL) return om[q];
    if (MODE == QR_GAMMA) return G[q];
    if (d.spare) return q < pd.nI + pd.nG ? qcol[q] : -1;
    if (q < pd.nI) return om[q];
    return (q >= pd.nIp && q < pd.nIp + pd.nG) ? G[q - pd.nIp] : -1;
  };
  int ncand = 0;
  for (int b0 = 0; b0 <= npos; b0 += QR_THREADS) {
    const int q = b0 + tid;
    int len = 0;
    if (q < npos) {
      const int c = col_at(q);
      if (c >= 0) len = trowptr[c + 1] - trowptr[c];
    }
    int tot;
    const int ex = block_scan_256(len, s_scan, &tot);
    if (q <= npos) qpre[q] = ncand + ex;
    ncand += tot;
  }
  __syncthreads();
  int cand = 0, qcur = 0, nbuf = 0;
  int64_t blk = 0;
  while (true) {
    // refill the buffer, QR_THREADS candidates at a time, keeping their order
    while (nbuf <= QR_CH - QR_THREADS && cand < ncand) {
      const int t = cand + tid;
      int take = -1, qt = npos;
      if (t < ncand) {
        int lo = qcur, hi = npos - 1;             // largest q with qpre[q] <= t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (qpre[mid] <= t) lo = mid; else hi = mid - 1;
        }
        qt = lo;
        const int r = trow[trowptr[col_at(lo)] + (t - qpre[lo])];
        int first = INT_MAX;
        bool interior = false;
        for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
          const int c = colind[e];
          interior |= part[c] == i;
          int posP;
          const int pos = layout_pos(c, &posP);
          if (pos >= 0) first = min(first, pos);
        }
        if (first == lo && (MODE != QR_GAMMA || interior)) take = r;
      }
      int tot;
      const int ex = block_scan_256(take >= 0 ? 1 : 0, s_scan, &tot);
      if (take >= 0) sBuf[nbuf + ex] = take;
      if (tid == QR_THREADS - 1) s_q = qt;
      __syncthreads();
      nbuf += tot;
      cand += QR_THREADS;
      qcur = min(s_q, max(npos - 1, 0));
      __syncthreads();
    }
    if (nbuf == 0) break;
    int head = 0;
    while (nbuf - head >= QB || (cand >= ncand && head < nbuf)) {
    const int nrow = min(QB, nbuf - head);
    const int gen = (int)blk++;
    if (tid == 0) { s_jmin = INT_MAX; s_jmax = -1; }
    __syncthreads();
    // ---- the rows of the block into the strip (one thread per row)
    if (tid < nrow) {
      const int r = sBuf[head + tid];
      int jmin = INT_MAX, jmax = -1;
      for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        int posP;
        const int pos = layout_pos(colind[e], &posP);
        if (pos < 0) continue;
        Bs[(int64_t)pos * QB + tid] = vals[e] * scale[pd.loc_off + posP];
        const int K = pos / TS;
        sGen[K] = gen;
        jmin = min(jmin, K);
        jmax = max(jmax, K);
      }
      if (jmax >= 0) { atomicMin(&s_jmin, jmin); atomicMax(&s_jmax, jmax); }
    }
    __syncthreads();
    // ---- tile columns of the block, ascending
    int J = s_jmin;
    while (true) {
      while (J <= s_jmax && sGen[J] != gen) ++J;
      if (J > s_jmax || (MODE == QR_SEL && J >= ntI)) break;
      int nr;
      if (MODE == QR_GAMMA) {
        nr = ntiles - J - 1;
        for (int a = tid; a < nr; a += QR_THREADS) sRows[a] = J + 1 + a;
        __syncthreads();
      } else {
        nr = envelope_rows(sF, J, ntiles, sRows, QR_TMAX, &s_count);
      }
      for (int a = tid; a < nr; a += QR_THREADS) sNZ[a] = 0;
      // panel: the triangle R(J, J) over B(:, J), on wave 0.  Lane (kc, h)
      // holds column kc of the tile, B rows 16 h .. 16 h + 15 and R rows
      // 16 h .. 16 h + 15; a column's two lanes are 32 apart, so its sums
      // take one lane swap and no workgroup barrier is needed.  Reflector c
      // goes to LDS (sV, sTau) for the other columns and the trailing tiles.
      double* Rjj = rtile(J, J);
      if (wave == 0) {
        double* Bj = Bs + (int64_t)(J * TS + kc) * QB + 16 * h;
        double b[16], rr[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          b[q] = Bj[q];
          rr[q] = Rjj[(16 * h + q) * sc + kc * sk];
        }
#pragma unroll
        for (int c = 0; c < TS; ++c) {
          const int hc = c >> 4, ic = c & 15;
          const double s2 = half_pair_sum(dot16(b, b, 0.0));
          const double al = half_pair_sum(h == hc ? rr[ic] : 0.0);
          const double s2c = lane_bcast(s2, c), alpha = lane_bcast(al, c);
          double tau = 0.0, beta = alpha, scl = 0.0;
          if (s2c > 0.0) {
            double nrm;
            bool keep = true;
            if (s2c >= 1e-280) {
              const double t = fma(alpha, alpha, s2c);
              nrm = t * rsqrt_refined(t);
            } else {
              // entries left by rounding can be so small that their squares
              // underflow: the column scaled by a power of two near its largest
              // entry first (all below 1e-290: not reflected, dropped)
              double mx = 0.0;
#pragma unroll
              for (int q = 0; q < 16; ++q) mx = fmax(mx, fabs(b[q]));
              mx = lane_bcast(fmax(mx, __shfl_xor(mx, 32, 64)), c);
              const double p2 = ldexp(1.0, -ilogb(fmax(mx, fabs(alpha))));
              double t2 = 0.0;
#pragma unroll
              for (int q = 0; q < 16; ++q) t2 += (b[q] * p2) * (b[q] * p2);
              t2 = lane_bcast(half_pair_sum(t2), c);
              nrm = sqrt((alpha * p2) * (alpha * p2) + t2) / p2;
              keep = mx > 1e-290;
            }
            if (keep) {
              beta = alpha > 0.0 ? -nrm : nrm;
              tau = (beta - alpha) * rcp2(beta);
              scl = rcp2(alpha - beta);
            }
          }
          if (kc == c) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
              b[q] *= scl;
              sV[c * QB + 16 * h + q] = b[q];
            }
            if (h == hc) rr[ic] = beta;
            if (h == 0) sTau[c] = tau;
          }
          wave_sync();
          if (tau != 0.0) {
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = sV[c * QB + 16 * h + q];
            const double w = half_pair_sum(dot16(v, b, h == hc ? rr[ic] : 0.0)) * tau;
            if (kc > c) {
              if (h == hc) rr[ic] -= w;
#pragma unroll
              for (int q = 0; q < 16; ++q) b[q] = fma(-v[q], w, b[q]);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          Rjj[(16 * h + q) * sc + kc * sk] = rr[q];
          Bj[q] = 0.0;
        }
      }
      __syncthreads();
      // the reflectors applied to the tiles right of J in the envelope, one
      // wave per tile with the same lane map
      for (int a = wave; a < nr; a += QR_THREADS / 64) {
        const int K = sRows[a];
        double* Rjk = rtile(J, K);
        double* Bk = Bs + (int64_t)(K * TS + kc) * QB + 16 * h;
        double b[16], rr[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          b[q] = Bk[q];
          rr[q] = Rjk[(16 * h + q) * sc + kc * sk];
        }
#pragma unroll
        for (int c = 0; c < TS; ++c) {
          const double tau = sTau[c];
          if (tau == 0.0) continue;
          const int hc = c >> 4, ic = c & 15;
          double v[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) v[q] = sV[c * QB + 16 * h + q];
          const double w = half_pair_sum(dot16(v, b, h == hc ? rr[ic] : 0.0)) * tau;
          if (h == hc) rr[ic] -= w;
#pragma unroll
          for (int q = 0; q < 16; ++q) b[q] = fma(-v[q], w, b[q]);
        }
        bool nz = false;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          Rjk[(16 * h + q) * sc + kc * sk] = rr[q];
          Bk[q] = b[q];
          nz |= b[q] != 0.0;
        }
        if (nz) sNZ[a] = 1;
      }
      __syncthreads();
      // a tile joins the block only if some row of it is nonzero there:
      // exact zeros stay zeros, and the block ends where its rows do
      if (tid == 0)
        for (int a = 0; a < nr; ++a)
          if (sNZ[a]) {
            sGen[sRows[a]] = gen;
            s_jmax = max(s_jmax, sRows[a]);
          }
      __syncthreads();
      ++J;
    }
    if (MODE == QR_SEL) {
      // interface tiles of the block were not eliminated: clear them
      for (int K = ntI; K < ntiles; ++K) {
        if (sGen[K] != gen) continue;
        double* Bk = Bs + (int64_t)K * TS * QB;
        for (int e = tid; e < TS * QB; e += QR_THREADS) Bk[e] = 0.0;
      }
      __syncthreads();
    }
    head += nrow;
    }
    // the rows not yet merged (fewer than a block) to the front
    const int rem = nbuf - head;
    const int keep = tid < rem ? sBuf[head + tid] : 0;
    __syncthreads();
    if (tid < rem) sBuf[tid] = keep;
    nbuf = rem;
    __syncthreads();
    if (cand >= ncand && nbuf == 0) break;
  }
  if (MODE == QR_GAMMA) return;
  // ---- positive diagonal, identity on padding, inverse diagonal tiles
  const int ncol = MODE == QR_SEL ? ntI : ntiles;
  for (int J = 0; J < ncol; ++J) {
    const int nr = envelope_rows(sF, J, ntiles, sRows, QR_TMAX, &s_count);
    double* Ljj = rtile(J, J);
    if (tid < TS) {
      const int c = tid, pos = J * TS + c;
      const bool real = (MODE == QR_SOLVE && d.spare) ? pos < pd.nI + pd.nG
                                                     : (pos < pd.nI || (pos >= pd.nIp && pos < pd.nIp + pd.nG));
      const double dg = Ljj[c * TS + c];
      double sg = dg < 0.0 ? -1.0 : 1.0;
      if (!real) {
        Ljj[c * TS + c] = 1.0;
        sg = 1.0;
      } else if (!(fabs(dg) > 0.0) || !(fabs(dg) < INFINITY)) {
        s_fail = 1;
        Ljj[c * TS + c] = 1.0;
        sg = 1.0;
      }
      sSgn[c] = sg;
    }
    __syncthreads();
    // column c of L in every tile of tile column J times its sign
    for (int a = -1; a < nr; ++a) {
      double* T = a < 0 ? Ljj : rtile(J, sRows[a]);
      for (int e = tid; e < TT; e += QR_THREADS) {
        const int c = e / TS, rw = e % TS;
        if (a < 0 && rw < c) continue;
        T[e] *= sSgn[c];
      }
    }
    __syncthreads();
    // L(J, J)^{-1}, lane c forming column c by forward substitution
    for (int e = tid; e < TT; e += QR_THREADS) sX[(e / TS) * LDT + e % TS] = Ljj[e];
    __syncthreads();
    if (tid < TS) {
      // column c of the inverse, lane c, by forward substitution
      const int c = tid;
      double x[TS];
#pragma unroll
      for (int a = 0; a < TS; ++a) {
        double t = a == c ? 1.0 : 0.0;
#pragma unroll
        for (int bq = 0; bq < a; ++bq) t = fma(-sX[bq * LDT + a], x[bq], t);
        x[a] = a < c ? 0.0 : t / sX[a * LDT + a];
      }
#pragma unroll
      for (int a = 0; a < TS; ++a) sInv[c * LDT + a] = x[a];
    }
    __syncthreads();
    for (int e = tid; e < TT; e += QR_THREADS) Di[(int64_t)J * TT + e] = sInv[(e / TS) * LDT + e % TS];
    __syncthreads();
  }
  if (tid == 0 && s_fail) atomicCAS(status, 0, i + 1);
}

void launch_qr_local(hipStream_t st, int mode, int nsub, const DevPlan& P, const DevPlan& Lay,
                     const DevMatrix& M, const int32_t* inv, const double* scale, double* out,
                     double* dinv, double* strip, int32_t* qscr, int64_t total_loc, int32_t* status) {
  if (nsub <= 0) return;
  const int64_t qcol_off = total_loc + nsub;
#define LSQ2L_QR_ARGS                                                                              \
  Lay.heavy(), P.subs, Lay.tileF, Lay.tileOff, P.omega, qscr, qcol_off, P.part, P.locown, M.rowptr, \
      M.colind, M.vals, M.trowptr, M.trow, inv, scale, out, dinv, strip, status
  if (mode == QR_SEL) k_qr_local<QR_SEL><<<nsub, QR_THREADS, 0, st>>>(LSQ2L_QR_ARGS);
  else if (mode == QR_SOLVE) k_qr_local<QR_SOLVE><<<nsub, QR_THREADS, 0, st>>>(LSQ2L_QR_ARGS);
  else k_qr_local<QR_GAMMA><<<nsub, QR_THREADS, 0, st>>>(LSQ2L_QR_ARGS);
#undef LSQ2L_QR_ARGS
}

// scale[pos] = 1 / ||A(:, c)|| for the column c at position pos of Omega_i
// (0 on padding): the equilibration S C_ii S of the Cholesky route, read off
// the columns of A instead of the diagonal of the formed C_ii.
__global__ void __launch_bounds__(256)
k_col_scale(const SubDesc* __restrict__ subs, const int32_t* __restrict__ omega,
            const int32_t* __restrict__ trowptr, const double* __restrict__ tvals,
            double* __restrict__ scale) {
  const SubDesc d = subs[blockIdx.x];
  const int32_t* om = omega + d.omega_off;
  for (int pos = blockIdx.y * blockDim.x + threadIdx.x; pos < d.np; pos += gridDim.y * blockDim.x) {
    int a = -1;
    if (pos < d.nI) a = pos;
    else if (pos >= d.nIp && pos < d.nIp + d.nG) a = d.nI + (pos - d.nIp);
    double s = 0.0;
    if (a >= 0) {
      const int c = om[a];
      double t = 0.0;
      for (int e = trowptr[c]; e < trowptr[c + 1]; ++e) t += tvals[e] * tvals[e];
      s = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
    }
    scale[d.loc_off + pos] = s;
  }
}

void launch_col_scale(hipStream_t st, int nsub, const DevPlan& P, const DevMatrix& M, double* scale) {
  if (nsub <= 0) return;
  const int ny = (int)std::min(64, (P.max_np + 255) / 256);
  k_col_scale<<<dim3(nsub, std::max(ny, 1)), 256, 0, st>>>(P.subs, P.omega, M.trowptr, M.tvals, scale);
}

}  // namespace lsq2l
