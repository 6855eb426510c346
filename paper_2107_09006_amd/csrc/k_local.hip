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
#include <algorithm>

#include "kernels.hpp"

namespace lsq2l {

__global__ void k_gather_values(int64_t nnz, const int32_t* __restrict__ perm,
                                const double* __restrict__ src, double* __restrict__ dst) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) dst[k] = src[perm[k]];
}

// Lower triangle of C_ii (tile-envelope layout) and of Ct_GG (dense, ld nGp);
// with fac null, only the envelope Fg below.
// Thread per local column: every write of a thread lands in its own column,
// so the accumulation order is fixed and no atomics are needed.  Workgroup
// (i, y) takes the columns y * 256 + t, (y + gridDim.y) * 256 + t, ... of
// subdomain i, so that a large subdomain spreads over several compute units.
// With inv given, it also finds the tile envelope of C_ii in the global
// column order (see k_solve_inv): the thread of column a sees every column
// coupled to it, so the first coupled position of row inv[a] in that order
// is the minimum it meets, one atomicMin per column into Fg.
// With scl given (S = diag(C_ii)^{-1/2} per local position, which is
// 1 / ||A(:, c)||: C_ii holds whole columns of A), every product is scaled as
// it is added, so the result is S C_ii S and S Ct_GG S directly, with unit
// diagonal entries on the padding positions (the equilibration in one pass).
__global__ void __launch_bounds__(256)
k_assemble(const SubDesc* __restrict__ subs, const int32_t* __restrict__ omega,
           const int32_t* __restrict__ part, const int32_t* __restrict__ locown,
           const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
           const double* __restrict__ vals, const int32_t* __restrict__ trowptr,
           const int32_t* __restrict__ trow, const double* __restrict__ tvals,
           const int32_t* __restrict__ tileF, const int64_t* __restrict__ tileOff,
           double* __restrict__ fac, double* __restrict__ ctg, const int32_t* __restrict__ inv,
           const SubDesc* __restrict__ gsub, int32_t* __restrict__ Fg,
           const double* __restrict__ scl) {
  const SubDesc d = subs[blockIdx.x];
  const int i = d.id;
  const double* sl = scl ? scl + d.loc_off : nullptr;
  const int32_t* iv = inv ? inv + d.loc_off : nullptr;
  const int32_t* om = omega + d.omega_off;
  const int32_t* G = om + d.nI;
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  double* A = fac ? fac + d.fac_off : nullptr;    // null: the envelope Fg only
  double* Ct = ctg ? ctg + d.g_off : nullptr;
  for (int a = blockIdx.y * blockDim.x + threadIdx.x; a < d.nI + d.nG; a += gridDim.y * blockDim.x) {
    const int j = om[a];
    const int posa = a < d.nI ? a : d.nIp + (a - d.nI);
    const int ta = posa / TS, ra = posa % TS;
    const int qa = iv ? iv[posa] : 0;
    const double sa = sl ? sl[posa] : 1.0;
    int fmin = qa;
    for (int k = trowptr[j]; k < trowptr[j + 1]; ++k) {
      const int r = trow[k];
      const double va = tvals[k];
      const int e0 = rowptr[r], e1 = rowptr[r + 1];
      bool inxi = false;
      if (A) for (int e = e0; e < e1; ++e) inxi |= (part[colind[e]] == i);
      for (int e = e0; e < e1; ++e) {
        const int posc = local_pos(i, colind[e], part, locown, G, d.nG, d.nIp);
        if (iv && posc >= 0) fmin = min(fmin, iv[posc]);
        if (!A || posc < posa) continue;
        const double v = sl ? vals[e] * va * (sa * sl[posc]) : vals[e] * va;
        const int tc = posc / TS;
        A[tile_pos(F, off, tc, ta) * TT + ra * TS + (posc % TS)] += v;
        if (inxi && a >= d.nI) Ct[(int64_t)(posa - d.nIp) * d.nGp + (posc - d.nIp)] += v;
      }
    }
    if (iv) atomicMin(&Fg[gsub[i].tile_base + qa / TS], fmin / TS);
  }
  if (A && sl && blockIdx.y == 0)
    for (int pos = threadIdx.x; pos < d.np; pos += blockDim.x) {
      const bool real = pos < d.nI || (pos >= d.nIp && pos < d.nIp + d.nG);
      if (!real) A[tile_pos(F, off, pos / TS, pos / TS) * TT + (pos % TS) * TS + pos % TS] = 1.0;
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
  // pairs of entries (rows r, r + 1 of one column c) as 16-byte accesses
  typedef double d2 __attribute__((ext_vector_type(2)));
  for (int t = blockIdx.y; t < d.ntiles; t += gridDim.y) {
    const int nt = t - F[t] + 1;
    d2* row = reinterpret_cast<d2*>(A + off[t] * TT);
    for (int64_t e2 = threadIdx.x; e2 < (int64_t)nt * (TT / 2); e2 += blockDim.x) {
      const int64_t e = 2 * e2;
      const int J = F[t] + (int)(e / TT);
      const int rc = (int)(e % TT);
      const int r = t * TS + rc % TS, c = J * TS + rc / TS;
      const double sr0 = s[r], sr1 = s[r + 1], sc = s[c];
      d2 v = row[e2];
      v.x = (r == c && sr0 == 0.0) ? 1.0 : v.x * (sr0 * sc);
      v.y = (r + 1 == c && sr1 == 0.0) ? 1.0 : v.y * (sr1 * sc);
      row[e2] = v;
    }
  }
  double* Ct = ctg + d.g_off;
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < (int64_t)d.nGp * d.nGp;
       e += (int64_t)gridDim.y * blockDim.x) {
    const int r = (int)(e % d.nGp), c = (int)(e / d.nGp);
    Ct[e] *= s[d.nIp + r] * s[d.nIp + c];   // zero on padding
  }
}

constexpr int ROWCAP = 2048;
constexpr int CHOL_TMAX = 2048;   // tile rows whose envelope the factorization keeps in LDS

// Right-looking tile Cholesky of one envelope matrix per workgroup:
// for each tile column J: the diagonal tile factored and inverted in
// registers (one step ahead, see below), L(I,J) = A(I,J) L(J,J)^{-T} for the
// envelope rows, then A(I,K) -= L(I,J) L(K,J)^T for every pair of envelope
// rows (MFMA).  Wave 0 applies column J to tile (J+1, J+1) first and factors
// it while the other waves work through the remaining pairs.  T is double or
// float (FP32 MFMA with FP32 accumulation).  With interior_only, the factor
// stops after the interior tile columns and the interface rows never update
// each other: the result holds L_I and L_GI only (what the coarse selection
// reads; the local solves then use factors of their own).
template <typename T>
__global__ void __launch_bounds__(256)
k_chol_local(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
             const int64_t* __restrict__ tileOff, T* __restrict__ fac, T* __restrict__ dinv,
             int32_t* __restrict__ status, int interior_only) {
  __shared__ T sW[TS * LDT], sL[TS * LDT], sInv[TS * LDT];
  __shared__ int32_t rows[ROWCAP];
  __shared__ int32_t sF[CHOL_TMAX], sO[CHOL_TMAX];
  __shared__ int s_count, s_ok;
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  // the envelope (first tile column and offset of each tile row) in LDS, so
  // that finding a tile costs no global round trip
  const bool staged = d.ntiles <= CHOL_TMAX;
  if (staged)
    for (int I = threadIdx.x; I < d.ntiles; I += blockDim.x) {
      sF[I] = F[I];
      sO[I] = (int32_t)off[I];
    }
  __syncthreads();
  const int32_t* Fp = staged ? sF : F;
  auto tpos = [&](int I, int J) -> int64_t {
    return staged ? (int64_t)sO[I] + (J - sF[I]) : tile_pos(F, off, I, J);
  };
  T* A = fac + d.fac_off;
  T* Di = dinv + d.dinv_off;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid / 64, lane = tid % 64, nwaves = nthr / 64;
  bool failed = false;
  __shared__ int s_next;
  // factor and invert diagonal tile J (its updates applied) by wave 0; the
  // tile is in sW on entry
  auto diag_factor = [&]() {
    const bool okw = tile_potrf_inv_reg(sW, sL, sInv, lane);
    if (lane == 0) s_ok = okw;
  };
  // tile columns to factor, and the first row of the block whose mutual
  // updates are skipped
  const int ncol = interior_only ? d.ntI : d.ntiles;
  const int skip_from = interior_only ? d.ntI : d.ntiles;
  if (wave == 0 && ncol > 0) {
    const T* A00 = A + tpos(0, 0) * TT;
    for (int e = lane; e < TT; e += 64) sW[(e / TS) * LDT + e % TS] = A00[e];
    wave_sync();
    diag_factor();
  }
  __syncthreads();
  for (int J = 0; J < ncol; ++J) {
    T* Ajj = A + tpos(J, J) * TT;
    const bool ok = s_ok;
    if (!ok) failed = true;
    for (int e = tid; e < TT; e += nthr) {
      Ajj[e] = sL[(e / TS) * LDT + e % TS];
      Di[(int64_t)J * TT + e] = sInv[(e / TS) * LDT + e % TS];
    }
    const int nr = envelope_rows(Fp, J, d.ntiles, rows, ROWCAP, &s_count);
    if (nr > ROWCAP) { failed = true; break; }
    // panel
    for (int a = wave; a < nr; a += nwaves) {
      T* Aij = A + tpos(rows[a], J) * TT;
      typename Mfma<T>::acc_t acc[4];
      tile_acc_zero<T>(acc);
      tile_mma_nt<T, false>(acc, Aij, TS, sInv, LDT, lane);
      tile_acc_store<T>(acc, Aij, TS, lane);
    }
    // the next diagonal tile gets its update from column J (when coupled)
    // and is factored by wave 0 while the other waves take the remaining
    // pairs (a >= b) of envelope rows from a shared counter; wave 0 joins
    // them when done
    const bool next = J + 1 < ncol;
    const bool next_coupled = next && nr > 0 && rows[0] == J + 1;
    const int npairs = nr * (nr + 1) / 2;
    if (tid == 0) s_next = next_coupled ? 1 : 0;
    __syncthreads();
    if (wave == 0 && next) {
      const T* Ann = A + tpos(J + 1, J + 1) * TT;
      if (next_coupled) {
        const T* Ln = A + tpos(J + 1, J) * TT;
        typename Mfma<T>::acc_t acc[4];
        tile_acc_load<T>(acc, Ann, TS, lane);
        tile_mma_nt<T, true>(acc, Ln, TS, Ln, TS, lane);
        tile_acc_store<T>(acc, sW, LDT, lane);
      } else {
        for (int e = lane; e < TT; e += 64) sW[(e / TS) * LDT + e % TS] = Ann[e];
      }
      wave_sync();
      diag_factor();
    }
    while (true) {
      int it = 0;
      if (lane == 0) it = atomicAdd(&s_next, 1);
      it = __shfl(it, 0, 64);
      if (it >= npairs) break;
      int a = (int)((sqrt(8.0 * it + 1.0) - 1.0) / 2.0);
      while (a * (a + 1) / 2 > it) --a;
      while ((a + 1) * (a + 2) / 2 <= it) ++a;
      const int b = it - a * (a + 1) / 2;
      const int Ia = rows[a], Ib = rows[b];
      if (Ib >= skip_from) continue;     // both rows at or past skip_from (rows ascend)
      const T* La = A + tpos(Ia, J) * TT;
      const T* Lb = A + tpos(Ib, J) * TT;
      T* Cab = A + tpos(Ia, Ib) * TT;
      typename Mfma<T>::acc_t acc[4];
      tile_acc_load<T>(acc, Cab, TS, lane);
      tile_mma_nt<T, true>(acc, La, TS, Lb, TS, lane);
      tile_acc_store<T>(acc, Cab, TS, lane);
    }
    __syncthreads();
  }
  if (failed && tid == 0) atomicCAS(status, 0, d.id + 1);
}

template __global__ void k_chol_local<double>(const SubDesc*, const int32_t*, const int64_t*,
                                              double*, double*, int32_t*, int);
template __global__ void k_chol_local<float>(const SubDesc*, const int32_t*, const int64_t*,
                                             float*, float*, int32_t*, int);

// ---------------------------------------------------------------------------
// The factor used by the per-iteration local solves.  C_ii^{-1} r does not
// depend on the order of Omega_i, and the order [Omega_Ii, Omega_Gamma_i]
// that the coarse selection needs (T = L_GI L_GI^T) makes the interface rows
// of L dense across the interior.  The solve factor therefore orders
// Omega_i by global column (the order of the columns of A) where that stores
// fewer tiles: position q of that order is the q-th smallest column of
// Omega_i.  Its envelope comes from the assembled C_ii itself (the first
// nonzero of each row after the permutation), which the factorization
// cannot leave; its values are gathered from the assembled, equilibrated
// C_ii before that is factored in place.
// ---------------------------------------------------------------------------

// inv[loc_off + pos] = position of the column at [I, Gamma] position pos in
// the global-column order of Omega_i (-1 on padding): the column's rank
// among the interior columns plus its rank among the interface columns
__global__ void __launch_bounds__(256)
k_solve_inv(const SubDesc* __restrict__ subs, const int32_t* __restrict__ omega,
            int32_t* __restrict__ inv) {
  const SubDesc d = subs[blockIdx.x];
  const int32_t* om = omega + d.omega_off;
  const int32_t* G = om + d.nI;
  auto rank = [](const int32_t* v, int n, int32_t c) {   // entries of v below c
    int lo = 0, hi = n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (v[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  for (int pos = threadIdx.x; pos < d.np; pos += blockDim.x) {
    int q = -1;
    if (pos < d.nI) q = pos + rank(G, d.nG, om[pos]);
    else if (pos >= d.nIp && pos < d.nIp + d.nG) q = (pos - d.nIp) + rank(om, d.nI, G[pos - d.nIp]);
    inv[d.loc_off + pos] = q;
  }
}

// Fg[tile_base + t] = t for every tile row t of the global-order layout
__global__ void __launch_bounds__(256)
k_solve_env_init(const SubDesc* __restrict__ gsub, int32_t* __restrict__ Fg) {
  const SubDesc g = gsub[blockIdx.x];
  for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) Fg[g.tile_base + t] = t;
}

// sperm[loc_off + q] = loc index of the entry the solve layout holds at
// position q (-1: padding): the global-column order where ssub.spare is set,
// the [I, Gamma] layout itself otherwise.  sperm is -1 on entry.
__global__ void __launch_bounds__(256)
k_solve_perm(const SubDesc* __restrict__ subs, const SubDesc* __restrict__ ssub,
             const int32_t* __restrict__ inv, int32_t* __restrict__ sperm) {
  const SubDesc d = subs[blockIdx.x];
  const SubDesc s = ssub[d.id];
  for (int pos = threadIdx.x; pos < d.np; pos += blockDim.x) {
    if (s.spare) {
      const int q = inv[d.loc_off + pos];
      if (q >= 0) sperm[s.loc_off + q] = (int32_t)(d.loc_off + pos);
    } else {
      sperm[s.loc_off + pos] = (int32_t)(d.loc_off + pos);
    }
  }
}

constexpr int GATHER_TMAX = 2048;

// The solve layout's matrix (tile envelope, double) from the assembled and
// equilibrated [I, Gamma] C_ii: entry (q_r, q_c) is C_ii(p_r, p_c) with
// p = sperm - loc_off, zero outside the [I, Gamma] envelope, and the
// identity on padding.  Workgroup (i, y) writes tile rows y, y + gridDim.y, ...
__global__ void __launch_bounds__(256)
k_gather_solve(const SubDesc* __restrict__ subs, const SubDesc* __restrict__ ssub,
               const int32_t* __restrict__ tileF, const int64_t* __restrict__ tileOff,
               const double* __restrict__ fac, const int32_t* __restrict__ stileF,
               const int64_t* __restrict__ stileOff, const int32_t* __restrict__ sperm,
               double* __restrict__ out) {
  __shared__ int32_t lF[GATHER_TMAX], lO[GATHER_TMAX];
  const SubDesc d = subs[blockIdx.x];
  const SubDesc s = ssub[d.id];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  const double* A = fac + d.fac_off;
  const int32_t* Fs = stileF + s.tile_base;
  const int64_t* offs = stileOff + s.tile_base;
  const int32_t* sp = sperm + s.loc_off;
  double* O = out + s.fac_off;
  // the [I, Gamma] envelope table in LDS (looked up for every entry)
  const bool staged = d.ntiles <= GATHER_TMAX;
  if (staged)
    for (int I = threadIdx.x; I < d.ntiles; I += blockDim.x) {
      lF[I] = F[I];
      lO[I] = (int32_t)off[I];
    }
  __syncthreads();
  for (int I = blockIdx.y; I < s.ntiles; I += gridDim.y) {
    const int nk = I - Fs[I] + 1;
    double* row = O + offs[I] * TT;
    for (int e = threadIdx.x; e < nk * TT; e += blockDim.x) {
      const int J = Fs[I] + e / TT, rc = e % TT;
      const int qr = I * TS + rc % TS, qc = J * TS + rc / TS;
      const int pr = sp[qr], pc = sp[qc];
      double v;
      if (pr < 0 || pc < 0) {
        v = (qr == qc) ? 1.0 : 0.0;
      } else {
        const int hi = (int)(max(pr, pc) - d.loc_off), lo = (int)(min(pr, pc) - d.loc_off);
        const int th = hi / TS, tl = lo / TS;
        const int fh = staged ? lF[th] : F[th];
        const int64_t t = staged ? (int64_t)lO[th] + (tl - fh) : tile_pos(F, off, th, tl);
        v = tl >= fh ? A[t * TT + (lo % TS) * TS + hi % TS] : 0.0;
      }
      row[e] = v;
    }
  }
}

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


// z_j = sum over the subdomains holding column j of S_pos loc_pos (fixed
// order), plus the coarse prolongation X_i d_i on the interior of its owner.
// Without loc only the prolongation is formed, without dcoarse only the sum.
// With `restricted`, column j takes only the value of its own subdomain's
// interior (R_i^T D_i of eq. RAS: D_i is zero on Omega_Gamma_i).
template <typename TX>
__global__ void k_scatter_local(int32_t n, const int32_t* __restrict__ own_ptr,
                                const int32_t* __restrict__ own_pos, const double* __restrict__ scale,
                                const double* __restrict__ loc, const int32_t* __restrict__ part,
                                const int32_t* __restrict__ locown, const SubDesc* __restrict__ subs,
                                const TX* __restrict__ X, const double* __restrict__ dcoarse,
                                double* __restrict__ z, int restricted) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  if (loc != nullptr) {
    if (restricted) {
      const int64_t pos = subs[part[j]].loc_off + locown[j];
      s = scale[pos] * loc[pos];
    } else {
      for (int q = own_ptr[j]; q < own_ptr[j + 1]; ++q) {
        const int pos = own_pos[q];
        s += scale[pos] * loc[pos];
      }
    }
  }
  if (dcoarse != nullptr) {
    const SubDesc d = subs[part[j]];
    const int a = locown[j];
    const TX* xr = X + d.x_off + a;
    const double* dc = dcoarse + d.cg_off;
    // eight independent loads in flight per thread
    double c8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 8 <= d.p; k += 8)
#pragma unroll
      for (int i = 0; i < 8; ++i) c8[i] += (double)xr[(int64_t)(k + i) * d.nIp] * dc[k + i];
    for (int i = 0; k < d.p; ++k, ++i) c8[i] += (double)xr[(int64_t)k * d.nIp] * dc[k];
    s += ((c8[0] + c8[1]) + (c8[2] + c8[3])) + ((c8[4] + c8[5]) + (c8[6] + c8[7]));
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
                     double* ctg, const int32_t* inv, const SubDesc* gsub, int32_t* Fg,
                     const double* scale) {
  // workgroups per subdomain: enough for the largest one to take 2 columns
  // per thread (at most 64)
  const int ny = std::max(1, std::min(64, (P.max_np + 511) / 512));
  k_assemble<<<dim3(nsub, ny), 256, 0, st>>>(P.heavy(), P.omega, P.part, P.locown, M.rowptr,
                                             M.colind, M.vals, M.trowptr, M.trow, M.tvals, P.tileF,
                                             P.tileOff, fac, ctg, inv, gsub, Fg, scale);
}

void launch_equilibrate(hipStream_t st, int nsub, const DevPlan& P, double* fac, double* ctg,
                        double* scale) {
  k_equil_scale<<<nsub, 256, 0, st>>>(P.heavy(), P.tileF, P.tileOff, fac, scale);
  k_equil_apply<<<dim3(nsub, 32), 256, 0, st>>>(P.heavy(), P.tileF, P.tileOff, fac, ctg, scale);
}

void launch_chol_local(hipStream_t st, int nsub, const DevPlan& P, double* fac, double* dinv,
                       int32_t* status, bool interior_only) {
  k_chol_local<double><<<nsub, 256, 0, st>>>(P.heavy(), P.tileF, P.tileOff, fac, dinv, status,
                                             interior_only ? 1 : 0);
}

void launch_solve_inv(hipStream_t st, int nsub, const DevPlan& P, int32_t* inv) {
  k_solve_inv<<<nsub, 256, 0, st>>>(P.heavy(), P.omega, inv);
}

void launch_solve_env_init(hipStream_t st, int nsub, const SubDesc* gsub, int32_t* Fg) {
  k_solve_env_init<<<nsub, 256, 0, st>>>(gsub, Fg);
}

void launch_solve_perm(hipStream_t st, int nsub, const DevPlan& P, const SubDesc* ssub,
                       const int32_t* inv, int32_t* sperm) {
  k_solve_perm<<<nsub, 256, 0, st>>>(P.heavy(), ssub, inv, sperm);
}

void launch_gather_solve(hipStream_t st, int nsub, const DevPlan& P, const DevPlan& Ps,
                         const double* fac, double* out) {
  k_gather_solve<<<dim3(nsub, 16), 256, 0, st>>>(P.heavy(), Ps.subs, P.tileF, P.tileOff, fac,
                                                  Ps.tileF, Ps.tileOff, Ps.sperm, out);
}

void launch_chol_local_f32(hipStream_t st, int nsub, const DevPlan& P, float* fac, float* dinv,
                           int32_t* status) {
  k_chol_local<float><<<nsub, 256, 0, st>>>(P.heavy(), P.tileF, P.tileOff, fac, dinv, status, 0);
}

void launch_to_float(hipStream_t st, int64_t n, const double* src, float* dst) {
  if (n == 0) return;
  k_to_float<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, src, dst);
}

void launch_gather_local(hipStream_t st, int nsub, const DevPlan& P, const double* scale,
                         const double* r, double* loc) {
  k_gather_local<<<nsub, 256, 0, st>>>(P.subs, P.omega, scale, r, loc);
}



void launch_scatter_local(hipStream_t st, int32_t n, const DevPlan& P, const double* scale,
                          const double* loc, const double* X, const double* dcoarse, double* z,
                          bool restricted) {
  if (n == 0) return;
  k_scatter_local<double><<<(n + 255) / 256, 256, 0, st>>>(n, P.own_ptr, P.own_pos, scale, loc,
                                                           P.part, P.locown, P.subs, X, dcoarse, z,
                                                           restricted ? 1 : 0);
}

void launch_scatter_local(hipStream_t st, int32_t n, const DevPlan& P, const double* scale,
                          const double* loc, const float* X, const double* dcoarse, double* z,
                          bool restricted) {
  if (n == 0) return;
  k_scatter_local<float><<<(n + 255) / 256, 256, 0, st>>>(n, P.own_ptr, P.own_pos, scale, loc,
                                                          P.part, P.locown, P.subs, X, dcoarse, z,
                                                          restricted ? 1 : 0);
}

// ||C(Omega_Ii, :)||_F^2 from the lower triangle of the assembled C_ii: the
// rows of C owned by subdomain i are its interior rows, and every column
// they couple to lies in Omega_i.  Entries (r, c), r >= c, count twice when
// both are interior (the upper mirror), once on the diagonal and once in the
// (Gamma, I) block; the (Gamma, Gamma) block belongs to other subdomains.
// One workgroup per subdomain, the sum in a fixed order.
__global__ void __launch_bounds__(256)
k_frob_interior(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
                const int64_t* __restrict__ tileOff, const double* __restrict__ fac,
                double* __restrict__ out) {
  __shared__ double sh[4];
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  const double* A = fac + d.fac_off;
  double acc = 0.0;
  for (int t = 0; t < d.ntiles; ++t) {
    const int nt = t - F[t] + 1;
    const double* row = A + off[t] * TT;
    for (int64_t e = threadIdx.x; e < (int64_t)nt * TT; e += blockDim.x) {
      const int J = F[t] + (int)(e / TT);
      const int rc = (int)(e % TT);
      const int r = t * TS + rc % TS, c = J * TS + rc / TS;
      if (r < c || c >= d.nI) continue;      // upper part, or a column outside the interior
      const double v = row[e];
      const double wgt = (r < d.nI) ? (r == c ? 1.0 : 2.0) : 1.0;
      acc += wgt * v * v;
    }
  }
  acc = wave_allsum(acc);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// C_ii += s I on the positions of real columns (the padding keeps its zero
// diagonal until the equilibration turns it into identity rows)
__global__ void __launch_bounds__(256)
k_add_diag(const SubDesc* __restrict__ subs, const int32_t* __restrict__ tileF,
           const int64_t* __restrict__ tileOff, double s, double* __restrict__ fac) {
  const SubDesc d = subs[blockIdx.x];
  const int32_t* F = tileF + d.tile_base;
  const int64_t* off = tileOff + d.tile_base;
  double* A = fac + d.fac_off;
  for (int pos = threadIdx.x; pos < d.np; pos += blockDim.x) {
    const bool real = pos < d.nI || (pos >= d.nIp && pos < d.nIp + d.nG);
    if (real) A[tile_pos(F, off, pos / TS, pos / TS) * TT + (pos % TS) * TS + pos % TS] += s;
  }
}

void launch_frob_interior(hipStream_t st, int nsub, const DevPlan& P, const double* fac,
                          double* out) {
  k_frob_interior<<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, fac, out);
}

void launch_add_diag(hipStream_t st, int nsub, const DevPlan& P, double s, double* fac) {
  k_add_diag<<<nsub, 256, 0, st>>>(P.subs, P.tileF, P.tileOff, s, fac);
}

}  // namespace lsq2l
