// Host replay of the QR local factors of the library (k_qr.hip): the same
// row stream (rows by first layout position), blocks of 32 rows, tile-column order, envelope lists, strip
// layout and final pass, computed on the CPU with every strip, factor and
// interface-matrix access checked against its buffer and the tile envelope.
// It also checks the property the kernel relies on: when tile column J of a
// block is eliminated, a tile K > J outside the envelope list of J is zero
// in every row the reflectors touch.  The results are compared with the
// definitions: L L^T = S C_ii S (dense Cholesky of the formed matrix) for the
// solve factors in both orders, the interior columns of the selection's
// factor, and R_G^T R_G = S Ct_GG S.  No GPU is used.
// Input: the file of plan_check.cpp followed by the nnz values of A.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "../../paper_2107_09006_amd/csrc/plan.hpp"
using namespace lsq2l;
#define CHECK(c, ...) do { if (!(c)) { fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); fprintf(stderr, __VA_ARGS__); fprintf(stderr, "\n"); exit(1); } } while (0)

namespace lsq2l {
void* host_block_take(size_t bytes, size_t* got) { *got = bytes; return std::malloc(bytes); }
void host_block_give(void* p, size_t) { std::free(p); }
}  // namespace lsq2l

enum { SEL = 0, SOLVE = 1, GAMMA = 2 };
constexpr int QB = 32;

struct Lay {                      // layout written by one run
  int np = 0, ntiles = 0, ntI = 0;
  std::vector<int32_t> F;         // envelope (empty: dense, GAMMA)
  std::vector<int64_t> off;
  int64_t stored = 0;
  bool global = false;
};

struct Ctx {
  int m, n;
  const std::vector<int32_t>*rp, *ci, *part, *trp, *tcol;
  const std::vector<double>*vals, *tvals;
  const HostPlan* H;
};

static double maxerr = 0.0;
static int64_t panels = 0, max_panels = 0, max_blocks = 0;   // tile columns eliminated

// The kernel's arithmetic for subdomain i in one mode; returns the factor
// (stored tiles, or the dense nGp x nGp R_G) and the inverse diagonal tiles.
static void replay(const Ctx& X, int i, int mode, const Lay& L, const std::vector<int32_t>& inv,
                   const std::vector<double>& scale, std::vector<double>& out,
                   std::vector<double>& dinv) {
  const HostPlan& H = *X.H;
  const SubDesc& d = H.subs[i];
  const int32_t* om = &H.omega[d.omega_off];
  const int32_t* G = om + d.nI;
  const auto& rp = *X.rp; const auto& ci = *X.ci; const auto& part = *X.part;
  const int ntiles = mode == GAMMA ? d.nGp / TS : L.ntiles;
  const int ntI = mode == GAMMA ? 0 : L.ntI;
  const int ld = d.nGp;
  const bool dense = mode == GAMMA;
  out.assign(dense ? (size_t)ld * ld : (size_t)L.stored * TT, 0.0);
  dinv.assign((size_t)ntiles * TT, 0.0);
  std::vector<double> B((size_t)QB * d.np, 0.0);
  std::vector<int> gen(ntiles, -1);
  auto local_pos = [&](int c) -> int {
    if (part[c] == i) return H.locown[c];
    int lo = 0, hi = d.nG;
    while (lo < hi) { int mid = (lo + hi) / 2; if (G[mid] < c) lo = mid + 1; else hi = mid; }
    return (lo < d.nG && G[lo] == c) ? d.nIp + lo : -1;
  };
  auto layout_pos = [&](int c, int* posP) -> int {
    const int p = local_pos(c);
    *posP = p;
    if (p < 0) return -1;
    if (mode == GAMMA) return p >= d.nIp ? p - d.nIp : -1;
    if (mode == SOLVE && L.global) return inv[d.loc_off + p];
    return p;
  };
  auto in_env = [&](int J, int K) { return dense || (K < ntiles && J <= K && J >= L.F[K]); };
  // element (c, kk) of R(J, K)
  auto R = [&](int J, int K, int c, int kk) -> double& {
    CHECK(J >= 0 && J <= K && K < ntiles && c >= 0 && c < TS && kk >= 0 && kk < TS, "R index");
    size_t idx;
    if (dense) {
      idx = (size_t)(K * TS + kk) * ld + J * TS + c;
      CHECK(idx < out.size(), "R_G index %zu", idx);
    } else {
      CHECK(in_env(J, K), "tile (%d,%d) outside the envelope of sub %d", K, J, i);
      const int64_t t = L.off[K] + (J - L.F[K]);
      CHECK(t >= 0 && t < L.stored, "tile %lld of %lld", (long long)t, (long long)L.stored);
      idx = (size_t)t * TT + (size_t)c * TS + kk;
    }
    return out[idx];
  };
  auto Bat = [&](int pos, int l) -> double& {
    CHECK(pos >= 0 && (int64_t)pos * QB + l < (int64_t)B.size() && l >= 0 && l < QB, "strip index");
    return B[(size_t)pos * QB + l];
  };
  // the row stream: rows in the order of their first position in the layout,
  // found through the columns of A^T (position ascending, A^T order inside)
  const int npos = mode == SEL ? d.nI : mode == GAMMA ? d.nG : L.np;
  std::vector<int> qcol(L.np, -1);
  if (mode == SOLVE && L.global)
    for (int p = 0; p < d.np; ++p) {
      const int q = inv[d.loc_off + p];
      if (q >= 0) qcol[q] = p < d.nI ? om[p] : G[p - d.nIp];
    }
  auto col_at = [&](int q) -> int {
    if (mode == SEL) return om[q];
    if (mode == GAMMA) return G[q];
    if (L.global) return q < d.nI + d.nG ? qcol[q] : -1;
    if (q < d.nI) return om[q];
    return (q >= d.nIp && q < d.nIp + d.nG) ? G[q - d.nIp] : -1;
  };
  std::vector<int> stream;
  for (int q = 0; q < npos; ++q) {
    const int c = col_at(q);
    if (c < 0) continue;
    for (int k = (*X.trp)[c]; k < (*X.trp)[c + 1]; ++k) {
      const int r = (*X.tcol)[k];
      int first = INT32_MAX;
      bool interior = false;
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        interior |= part[ci[e]] == i;
        int posP;
        const int pos = layout_pos(ci[e], &posP);
        if (pos >= 0) first = std::min(first, pos);
      }
      if (first == q && (mode != GAMMA || interior)) stream.push_back(r);
    }
  }
  {
    // every row the mode needs, exactly once
    std::vector<int> want;
    for (int r = 0; r < X.m; ++r) {
      bool in_omega = false, interior = false, gamma = false;
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const int p = local_pos(ci[e]);
        in_omega |= p >= 0;
        interior |= part[ci[e]] == i;
        gamma |= p >= d.nIp;
      }
      if ((mode == SEL && interior) || (mode == SOLVE && in_omega) || (mode == GAMMA && interior && gamma))
        want.push_back(r);
    }
    std::vector<int> got(stream);
    std::sort(got.begin(), got.end());
    CHECK(got == want, "row stream of sub %d (mode %d): %zu rows, %zu wanted", i, mode, got.size(), want.size());
  }
  const int64_t nstream = (int64_t)stream.size();
  const int64_t p0 = panels;
  struct Tally { int64_t p0, nb; ~Tally() { const int64_t n = panels - p0; if (n > max_panels) { max_panels = n; max_blocks = nb; } } } tally{p0, (nstream + QB - 1) / QB};
  for (int64_t blk = 0; blk * QB < nstream; ++blk) {
    const int gn = (int)blk;
    int jmin = INT32_MAX, jmax = -1;
    for (int l = 0; l < QB; ++l) {
      const int64_t s = blk * QB + l;
      if (s >= nstream) break;
      const int r = stream[s];
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        int posP;
        const int pos = layout_pos(ci[e], &posP);
        if (pos < 0) continue;
        CHECK(pos < (dense ? ld : L.np), "position %d beyond the layout", pos);
        CHECK(Bat(pos, l) == 0.0, "strip entry not clear");
        Bat(pos, l) = (*X.vals)[e] * scale[d.loc_off + posP];
        gen[pos / TS] = gn;
        jmin = std::min(jmin, pos / TS);
        jmax = std::max(jmax, pos / TS);
      }
    }
    int J = jmin;
    while (true) {
      while (J <= jmax && gen[J] != gn) ++J;
      if (J > jmax || (mode == SEL && J >= ntI)) break;
      std::vector<int> rows;
      for (int K = J + 1; K < ntiles; ++K) if (dense || L.F[K] <= J) rows.push_back(K);
      ++panels;
      // panel
      double V[TS][QB], tau[TS];
      for (int c = 0; c < TS; ++c) {
        // the column scaled by a power of two near its largest entry before
        // the squares (rounding residue can underflow)
        const double alpha = R(J, J, c, c);
        double mx = 0.0;
        for (int l = 0; l < QB; ++l) mx = std::max(mx, std::fabs(Bat(J * TS + c, l)));
        const double p2 = mx > 0.0 ? std::ldexp(1.0, -std::ilogb(std::max(mx, std::fabs(alpha)))) : 1.0;
        double s2 = 0.0;
        for (int l = 0; l < QB; ++l) s2 += (Bat(J * TS + c, l) * p2) * (Bat(J * TS + c, l) * p2);
        double t = 0.0, beta = alpha, scl = 0.0;
        if (mx > 1e-290) {
          const double nrm = std::sqrt((alpha * p2) * (alpha * p2) + s2) / p2;
          beta = alpha > 0.0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scl = 1.0 / (alpha - beta);
        }
        for (int l = 0; l < QB; ++l) { Bat(J * TS + c, l) *= scl; V[c][l] = Bat(J * TS + c, l); }
        R(J, J, c, c) = beta;
        tau[c] = t;
        if (t == 0.0) continue;
        for (int kk = c + 1; kk < TS; ++kk) {
          double w = R(J, J, c, kk);
          for (int l = 0; l < QB; ++l) w += V[c][l] * Bat(J * TS + kk, l);
          w *= t;
          R(J, J, c, kk) -= w;
          for (int l = 0; l < QB; ++l) Bat(J * TS + kk, l) -= V[c][l] * w;
        }
      }
      for (int c = 0; c < TS; ++c) for (int l = 0; l < QB; ++l) Bat(J * TS + c, l) = 0.0;
      // tiles outside the list: zero wherever a reflector is nonzero
      for (int K = J + 1; K < ntiles; ++K) {
        if (std::find(rows.begin(), rows.end(), K) != rows.end() || gen[K] != gn) continue;
        for (int l = 0; l < QB; ++l) {
          bool touched = false;
          for (int c = 0; c < TS; ++c) touched |= V[c][l] != 0.0 && tau[c] != 0.0;
          if (!touched) continue;
          for (int kk = 0; kk < TS; ++kk)
            CHECK(Bat(K * TS + kk, l) == 0.0, "sub %d: tile %d of row %d nonzero outside the envelope list of %d", i, K, l, J);
        }
      }
      for (int K : rows) {
        for (int c = 0; c < TS; ++c) {
          if (tau[c] == 0.0) continue;
          for (int kk = 0; kk < TS; ++kk) {
            double w = R(J, K, c, kk);
            for (int l = 0; l < QB; ++l) w += V[c][l] * Bat(K * TS + kk, l);
            w *= tau[c];
            R(J, K, c, kk) -= w;
            for (int l = 0; l < QB; ++l) Bat(K * TS + kk, l) -= V[c][l] * w;
          }
        }
        bool nz = false;
        for (int kk = 0; kk < TS; ++kk) for (int l = 0; l < QB; ++l) nz |= Bat(K * TS + kk, l) != 0.0;
        if (nz) { gen[K] = gn; jmax = std::max(jmax, K); }
      }
      ++J;
    }
    if (mode == SEL)
      for (int K = ntI; K < ntiles; ++K)
        if (gen[K] == gn) for (int e = 0; e < TS * QB; ++e) B[(size_t)K * TS * QB + e] = 0.0;
    for (double v : B) CHECK(v == 0.0, "strip not clear after block %lld of sub %d", (long long)blk, i);
  }
  if (mode == GAMMA) return;
  const int ncol = mode == SEL ? ntI : ntiles;
  for (int J = 0; J < ncol; ++J) {
    double sg[TS];
    for (int c = 0; c < TS; ++c) {
      const int pos = J * TS + c;
      const bool real = (mode == SOLVE && L.global) ? pos < d.nI + d.nG
                                                    : (pos < d.nI || (pos >= d.nIp && pos < d.nIp + d.nG));
      double& dg = R(J, J, c, c);
      sg[c] = dg < 0.0 ? -1.0 : 1.0;
      if (!real) { dg = 1.0; sg[c] = 1.0; }
      CHECK(!real || std::fabs(dg) > 0.0, "zero diagonal at %d of sub %d", pos, i);
    }
    for (int K = J; K < ntiles; ++K) {
      if (!dense && L.F[K] > J) continue;
      for (int c = 0; c < TS; ++c)
        for (int kk = 0; kk < TS; ++kk)
          if (K > J || kk >= c) R(J, K, c, kk) *= sg[c];
    }
    // inverse of L(J, J) = R(J, J)^T by forward substitution
    for (int c = 0; c < TS; ++c) {
      double x[TS];
      for (int a = 0; a < TS; ++a) {
        double t = a == c ? 1.0 : 0.0;
        for (int b = 0; b < a; ++b) t -= R(J, J, b, a) * x[b];
        x[a] = a < c ? 0.0 : t / R(J, J, a, a);
      }
      for (int a = 0; a < TS; ++a) dinv[(size_t)J * TT + c * TS + a] = x[a];
    }
  }
}

// dense Cholesky (lower) in place; false if not positive definite
static bool chol(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    const double dj = std::sqrt(s);
    A[(size_t)j * n + j] = dj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / dj;
    }
    for (int k = j + 1; k < n; ++k) A[(size_t)j * n + k] = 0.0;
  }
  return true;
}

int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  CHECK(f, "input");
  int32_t hdr[5];
  CHECK(fread(hdr, 4, 5, f) == 5, "header");
  const int32_t m = hdr[0], n = hdr[1], nnz = hdr[2], nparts = hdr[3];
  std::vector<int32_t> rp(m + 1), ci(nnz), part(n), sop(nparts);
  std::vector<double> vals(nnz);
  CHECK(fread(rp.data(), 4, m + 1, f) == (size_t)m + 1 && fread(ci.data(), 4, nnz, f) == (size_t)nnz &&
        fread(part.data(), 4, n, f) == (size_t)n && fread(sop.data(), 4, nparts, f) == (size_t)nparts &&
        fread(vals.data(), 8, nnz, f) == (size_t)nnz, "body");
  fclose(f);
  std::vector<int32_t> trp, tcol, tperm;
  plan_transpose(m, n, rp.data(), ci.data(), trp, tcol, tperm);
  std::vector<double> tvals(nnz);
  for (int k = 0; k < nnz; ++k) tvals[k] = vals[tperm[k]];
  HostPlan H; std::string err;
  CHECK(plan_build(m, n, rp.data(), ci.data(), part.data(), nparts, sop, H, err), "%s", err.c_str());
  CHECK(plan_maps(n, H, err), "%s", err.c_str());
  Ctx X{m, n, &rp, &ci, &part, &trp, &tcol, &vals, &tvals, &H};
  const int maxcheck = argc > 2 ? atoi(argv[2]) : 1200;
  std::vector<double> scale(H.total_loc, 0.0);
  std::vector<int32_t> inv(H.total_loc, -1);
  int checked = 0;
  for (int i = 0; i < nparts; ++i) {
    const SubDesc& d = H.subs[i];
    const int32_t* om = &H.omega[d.omega_off];
    const int32_t* G = om + d.nI;
    auto rank = [](const int32_t* v, int cnt, int32_t c) { return (int)(std::lower_bound(v, v + cnt, c) - v); };
    std::vector<int> colof(d.np, -1);           // global column at each [I, Gamma] position
    for (int pos = 0; pos < d.np; ++pos) {
      int a = -1;
      if (pos < d.nI) a = pos;
      else if (pos >= d.nIp && pos < d.nIp + d.nG) a = d.nI + pos - d.nIp;
      if (a < 0) continue;
      const int c = om[a];
      colof[pos] = c;
      double t = 0.0;
      for (int e = trp[c]; e < trp[c + 1]; ++e) t += tvals[e] * tvals[e];
      scale[d.loc_off + pos] = 1.0 / std::sqrt(t);
      inv[d.loc_off + pos] = pos < d.nI ? pos + rank(G, d.nG, c) : (pos - d.nIp) + rank(om, d.nI, c);
    }
    // layouts: [I, Gamma] from the plan; global order with its envelope
    Lay P;
    P.np = d.np; P.ntiles = d.ntiles; P.ntI = d.ntI;
    P.F.assign(&H.tileF[d.tile_base], &H.tileF[d.tile_base] + d.ntiles);
    P.off.assign(&H.tileOff[d.tile_base], &H.tileOff[d.tile_base] + d.ntiles);
    P.stored = P.off.back() + (d.ntiles - 1 - P.F.back()) + 1;
    Lay Gl;
    Gl.global = true;
    Gl.np = (d.nI + d.nG + TS - 1) / TS * TS;
    Gl.ntiles = Gl.np / TS;
    Gl.ntI = d.ntI;
    Gl.F.resize(Gl.ntiles);
    for (int t = 0; t < Gl.ntiles; ++t) Gl.F[t] = t;
    for (int pos = 0; pos < d.np; ++pos) {
      if (colof[pos] < 0) continue;
      const int q = inv[d.loc_off + pos];
      int fmin = q;
      for (int e = trp[colof[pos]]; e < trp[colof[pos] + 1]; ++e) {
        const int r = tcol[e];
        for (int e2 = rp[r]; e2 < rp[r + 1]; ++e2) {
          const int c = ci[e2];
          int p2 = -1;
          if (part[c] == i) p2 = H.locown[c];
          else { const int g = rank(G, d.nG, c); if (g < d.nG && G[g] == c) p2 = d.nIp + g; }
          if (p2 >= 0) fmin = std::min(fmin, inv[d.loc_off + p2]);
        }
      }
      Gl.F[q / TS] = std::min(Gl.F[q / TS], fmin / TS);
    }
    Gl.off.resize(Gl.ntiles);
    int64_t run = 0;
    for (int t = 0; t < Gl.ntiles; ++t) { Gl.off[t] = run; run += t - Gl.F[t] + 1; }
    Gl.stored = run;
    std::vector<double> fsel, dsel, fsp, dsp, fgl, dgl, rg, dg;
    replay(X, i, SEL, P, inv, scale, fsel, dsel);
    replay(X, i, SOLVE, P, inv, scale, fsp, dsp);
    replay(X, i, SOLVE, Gl, inv, scale, fgl, dgl);
    if (d.nG > 0) replay(X, i, GAMMA, P, inv, scale, rg, dg);
    if (d.np > maxcheck) continue;
    ++checked;
    // S C_ii S and S Ct_GG S from their definitions, in [I, Gamma] positions
    const int np = d.np;
    std::vector<double> C((size_t)np * np, 0.0), Ct((size_t)np * np, 0.0);
    std::vector<int> posof(n, -1);
    for (int pos = 0; pos < np; ++pos) if (colof[pos] >= 0) posof[colof[pos]] = pos;
    std::vector<char> inxi(m, 0);
    for (int a = 0; a < d.nXi; ++a) inxi[H.xi[d.xi_off + a]] = 1;
    for (int r = 0; r < m; ++r) {
      std::vector<std::pair<int, double>> ent;
      for (int e = rp[r]; e < rp[r + 1]; ++e)
        if (posof[ci[e]] >= 0) ent.push_back({posof[ci[e]], vals[e] * scale[d.loc_off + posof[ci[e]]]});
      for (auto& x : ent)
        for (auto& y : ent) {
          C[(size_t)x.first * np + y.first] += x.second * y.second;
          if (inxi[r]) Ct[(size_t)x.first * np + y.first] += x.second * y.second;
        }
    }
    for (int pos = 0; pos < np; ++pos) if (colof[pos] < 0) C[(size_t)pos * np + pos] = 1.0;
    // solve factors, [I, Gamma] and global order, against the dense Cholesky
    for (int which = 0; which < 2; ++which) {
      const Lay& Lw = which ? Gl : P;
      const std::vector<double>& fac = which ? fgl : fsp;
      const std::vector<double>& di = which ? dgl : dsp;
      const int nw = Lw.np;
      std::vector<int> at(nw, -1);             // [I, Gamma] position at each layout position
      for (int pos = 0; pos < np; ++pos) {
        if (colof[pos] < 0) continue;
        const int q = which ? inv[d.loc_off + pos] : pos;
        at[q] = pos;
      }
      std::vector<double> Cw((size_t)nw * nw, 0.0);
      for (int a = 0; a < nw; ++a)
        for (int b = 0; b < nw; ++b)
          Cw[(size_t)a * nw + b] = (at[a] >= 0 && at[b] >= 0) ? C[(size_t)at[a] * np + at[b]] : (a == b ? 1.0 : 0.0);
      CHECK(chol(Cw, nw), "C_ii not positive definite in sub %d", i);
      double scl = 0.0, e = 0.0;
      for (int a = 0; a < nw; ++a)
        for (int b = 0; b <= a; ++b) {
          const int I = a / TS, Jt = b / TS;
          double v = 0.0;
          if (Jt >= Lw.F[I]) v = fac[(size_t)(Lw.off[I] + Jt - Lw.F[I]) * TT + (b % TS) * TS + a % TS];
          scl = std::max(scl, std::fabs(Cw[(size_t)a * nw + b]));
          e = std::max(e, std::fabs(v - Cw[(size_t)a * nw + b]));
        }
      CHECK(e <= 1e-10 * scl, "solve factor (%s) of sub %d off by %g", which ? "global" : "split", i, e / scl);
      maxerr = std::max(maxerr, e / scl);
      // the inverse diagonal tiles
      for (int J = 0; J < Lw.ntiles; ++J)
        for (int a = 0; a < TS; ++a)
          for (int c = 0; c < TS; ++c) {
            double t = 0.0;
            for (int b = 0; b < TS; ++b) {
              const double l = b <= a ? fac[(size_t)(Lw.off[J] + J - Lw.F[J]) * TT + b * TS + a] : 0.0;
              t += l * di[(size_t)J * TT + c * TS + b];
            }
            CHECK(std::fabs(t - (a == c ? 1.0 : 0.0)) <= 1e-8, "inverse tile %d of sub %d", J, i);
          }
    }
    // the selection's factor: interior columns (L_I, L_GI) of the [I, Gamma] Cholesky
    {
      std::vector<double> Cp(C);
      CHECK(chol(Cp, np), "C_ii");
      double scl = 0.0, e = 0.0;
      for (int a = 0; a < np; ++a)
        for (int b = 0; b <= a && b < d.nIp; ++b) {
          const int I = a / TS, Jt = b / TS;
          double v = 0.0;
          if (Jt >= P.F[I]) v = fsel[(size_t)(P.off[I] + Jt - P.F[I]) * TT + (b % TS) * TS + a % TS];
          scl = std::max(scl, std::fabs(Cp[(size_t)a * np + b]));
          e = std::max(e, std::fabs(v - Cp[(size_t)a * np + b]));
        }
      CHECK(e <= 1e-10 * scl, "selection factor of sub %d off by %g", i, e / scl);
      maxerr = std::max(maxerr, e / scl);
    }
    // R_G^T R_G = S Ct_GG S
    if (d.nG > 0) {
      const int ld = d.nGp;
      double scl = 0.0, e = 0.0;
      for (int a = 0; a < d.nG; ++a)
        for (int b = 0; b < d.nG; ++b) {
          double t = 0.0;
          for (int k = 0; k < ld; ++k) t += rg[(size_t)a * ld + k] * rg[(size_t)b * ld + k];
          const double ref = Ct[(size_t)(d.nIp + a) * np + d.nIp + b];
          scl = std::max(scl, std::fabs(ref));
          e = std::max(e, std::fabs(t - ref));
        }
      for (int a = 0; a < ld; ++a)
        for (int k = a + 1; k < ld; ++k) CHECK(rg[(size_t)a * ld + k] == 0.0, "R_G not upper triangular");
      CHECK(e <= 1e-12 * std::max(scl, 1.0), "R_G of sub %d off by %g", i, e);
    }
  }
  printf("panels: %lld in all, at most %lld in one factor (%lld blocks)\n", (long long)panels,
         (long long)max_panels, (long long)max_blocks);
  printf("OK %d subdomains replayed, %d checked against the definitions, max rel error %.3g\n", nparts,
         checked, maxerr);
  return 0;
}
