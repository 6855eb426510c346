// Host-logic check of the lsq2l planner: builds the real host plan (index
// sets, tile envelopes, overlap maps, coarse numbering and the envelope of E)
// for a problem read from a file, then replays the address arithmetic of
// every device kernel on the CPU and fails on the first access outside its
// buffer or outside a tile envelope.  No GPU is used.
// Input file: int32 header {m, n, nnz, nparts, ninstances}, then rowptr,
// colind, part (concatenated instances) and the instance of every part.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>
#include "../../paper_2107_09006_amd/csrc/plan.hpp"
using namespace lsq2l;
#define CHECK(c, ...) do { if (!(c)) { fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); fprintf(stderr, __VA_ARGS__); fprintf(stderr, "\n"); exit(1); } } while (0)

// the planner's host arrays live on the heap here
namespace lsq2l {
void* host_block_take(size_t bytes, size_t* got) { *got = bytes; return std::malloc(bytes); }
void host_block_give(void* p, size_t) { std::free(p); }
}  // namespace lsq2l

// The index sets, envelopes, overlap map and shared-row pairs straight from
// their definitions (sets of rows and columns), compared with the plan.
static void check_against_definitions(int m, int n, int nparts, const std::vector<int32_t>& rp,
                                      const std::vector<int32_t>& ci, const std::vector<int32_t>& part,
                                      const std::vector<int32_t>& trp, const std::vector<int32_t>& tcol,
                                      const HostPlan& H) {
  std::vector<std::vector<int32_t>> interior(nparts), xi(nparts);
  for (int j = 0; j < n; ++j) interior[part[j]].push_back(j);
  std::vector<std::set<int32_t>> rowparts(m);
  for (int r = 0; r < m; ++r) {
    for (int e = rp[r]; e < rp[r + 1]; ++e) rowparts[r].insert(part[ci[e]]);
    for (int i : rowparts[r]) xi[i].push_back(r);
  }
  std::vector<std::map<int32_t, int32_t>> posmap(nparts);   // column -> local position
  for (int i = 0; i < nparts; ++i) {
    const SubDesc& d = H.subs[i];
    CHECK(d.nI == (int)interior[i].size() && d.nXi == (int)xi[i].size(), "sizes of sub %d", i);
    for (int a = 0; a < d.nXi; ++a) CHECK(H.xi[d.xi_off + a] == xi[i][a], "Xi of sub %d", i);
    std::set<int32_t> gam;
    for (int r : xi[i])
      for (int e = rp[r]; e < rp[r + 1]; ++e)
        if (part[ci[e]] != i) gam.insert(ci[e]);
    CHECK(d.nG == (int)gam.size(), "Gamma size of sub %d", i);
    int g = 0;
    for (int c : gam) CHECK(H.omega[d.omega_off + d.nI + g++] == c, "Gamma of sub %d", i);
    for (int a = 0; a < d.nI; ++a) {
      CHECK(H.omega[d.omega_off + a] == interior[i][a], "interior of sub %d", i);
      posmap[i][interior[i][a]] = a;
    }
    g = 0;
    for (int c : gam) posmap[i][c] = d.nIp + g++;
    // envelope: every row holding a column of Omega_i couples its columns in Omega_i
    std::set<int32_t> rows;
    for (const auto& kv : posmap[i])
      for (int k = trp[kv.first]; k < trp[kv.first + 1]; ++k) rows.insert(tcol[k]);
    std::vector<int32_t> f(d.np);
    for (int a = 0; a < d.np; ++a) f[a] = a;
    for (int r : rows) {
      std::vector<int32_t> q;
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        auto it = posmap[i].find(ci[e]);
        if (it != posmap[i].end()) q.push_back(it->second);
      }
      const int best = *std::min_element(q.begin(), q.end());
      for (int x : q) f[x] = std::min(f[x], best);
    }
    for (int t = 0; t < d.ntiles; ++t) {
      int mn = t * TS;
      for (int a = t * TS; a < (t + 1) * TS; ++a) mn = std::min(mn, f[a]);
      CHECK(H.tileF[d.tile_base + t] == mn / TS, "envelope of sub %d tile %d", i, t);
    }
  }
  // overlap map: positions of every column, by increasing subdomain
  std::vector<std::vector<int32_t>> own(n);
  for (int i = 0; i < nparts; ++i)
    for (const auto& kv : posmap[i]) own[kv.first].push_back((int32_t)(H.subs[i].loc_off + kv.second));
  for (int j = 0; j < n; ++j) {
    CHECK(H.own_ptr[j + 1] - H.own_ptr[j] == (int)own[j].size(), "own count of column %d", j);
    for (size_t q = 0; q < own[j].size(); ++q) CHECK(H.own_pos[H.own_ptr[j] + q] == own[j][q], "own of column %d", j);
  }
  // shared rows of every pair i < j, pairs in order of first occurrence
  std::map<std::pair<int, int>, std::vector<int32_t>> shared;
  std::vector<std::pair<int, int>> first;
  std::vector<std::map<int32_t, int32_t>> rank(nparts);
  for (int i = 0; i < nparts; ++i)
    for (size_t a = 0; a < xi[i].size(); ++a) rank[i][xi[i][a]] = (int32_t)a;
  for (int r = 0; r < m; ++r)
    for (int u : rowparts[r])
      for (int v : rowparts[r]) {
        if (v <= u) continue;
        auto key = std::make_pair(u, v);
        if (!shared.count(key)) first.push_back(key);
        shared[key].push_back(rank[u][r]);
        shared[key].push_back(rank[v][r]);
      }
  CHECK(H.cpair_ij.size() == 2 * first.size(), "pair count");
  for (size_t k = 0; k < first.size(); ++k) {
    CHECK(H.cpair_ij[2 * k] == first[k].first && H.cpair_ij[2 * k + 1] == first[k].second, "pair %zu", k);
    const auto& rows = shared[first[k]];
    CHECK(2 * (H.cpair_ptr[k + 1] - H.cpair_ptr[k]) == (int64_t)rows.size(), "rows of pair %zu", k);
    for (size_t q = 0; q < rows.size(); ++q) CHECK(H.cpair_rows[2 * H.cpair_ptr[k] + q] == rows[q], "row of pair %zu", k);
  }
}

int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  int32_t hdr[5];
  fread(hdr, 4, 5, f);
  int32_t m = hdr[0], n = hdr[1], nnz = hdr[2], nparts = hdr[3], S = hdr[4];
  std::vector<int32_t> rp(m + 1), ci(nnz), part(n), sop(nparts);
  fread(rp.data(), 4, m + 1, f); fread(ci.data(), 4, nnz, f); fread(part.data(), 4, n, f); fread(sop.data(), 4, nparts, f);
  fclose(f);
  std::vector<int32_t> trp, tcol, tperm;
  plan_transpose(m, n, rp.data(), ci.data(), trp, tcol, tperm);
  for (int k = 0; k < nnz; ++k) CHECK(tperm[k] >= 0 && tperm[k] < nnz, "tperm");
  // row-sorted iteration copy (row_order) and k_permute_rows: every source
  // row read once, every destination entry inside [0, nnz) written once
  RowOrder ro;
  row_order(m, n, rp.data(), ci.data(), ro);
  if (ro.use) {
    CHECK((int64_t)ro.perm.size() == m && (int64_t)ro.prp.size() == (int64_t)m + 1, "row order sizes");
    std::vector<char> seen(m, 0), written(nnz, 0);
    CHECK(ro.prp[0] == 0 && ro.prp[m] == nnz, "permuted row starts");
    for (int i = 0; i < m; ++i) {
      const int r = ro.perm[i];
      CHECK(r >= 0 && r < m && !seen[r], "perm entry %d", i);
      seen[r] = 1;
      CHECK(i == 0 || (rp[ro.perm[i - 1]] < rp[ro.perm[i - 1] + 1] ? ci[rp[ro.perm[i - 1]]] : n) <=
                      (rp[r] < rp[r + 1] ? ci[rp[r]] : n), "rows not sorted by first column at %d", i);
      int d = ro.prp[i];
      for (int k = rp[r]; k < rp[r + 1]; ++k, ++d) {
        CHECK(d >= 0 && d < nnz && !written[d], "permuted entry %d of row %d", d, i);
        written[d] = 1;
      }
      CHECK(d == ro.prp[i + 1], "row %d length", i);
    }
    printf("row order: permuted\n");
  }
  HostPlan H; std::string err;
  CHECK(plan_build(m, n, rp.data(), ci.data(), part.data(), nparts, sop, H, err), "%s", err.c_str());
  CHECK(plan_maps(n, H, err), "%s", err.c_str());
  check_against_definitions(m, n, nparts, rp, ci, part, trp, tcol, H);
  int64_t maxrows = 0;
  for (int i = 0; i < nparts; ++i) {
    const SubDesc& d = H.subs[i];
    const int64_t fac_end = (i + 1 < nparts) ? H.subs[i + 1].fac_off : H.total_fac;
    const int64_t stored = (fac_end - d.fac_off) / TT;
    const int32_t* F = &H.tileF[d.tile_base];
    const int64_t* off = &H.tileOff[d.tile_base];
    auto tp = [&](int I, int J) -> int64_t {
      CHECK(I >= 0 && I < d.ntiles && J <= I && J >= F[I], "tile (%d,%d) outside envelope of sub %d (F=%d)", I, J, i, I < d.ntiles ? F[I] : -1);
      int64_t t = off[I] + (J - F[I]);
      CHECK(t >= 0 && t < stored, "tile index %lld out of %lld", (long long)t, (long long)stored);
      return t;
    };
    CHECK(off[0] == 0, "first tile offset");
    CHECK(off[d.ntiles - 1] + (d.ntiles - 1 - F[d.ntiles - 1]) + 1 == stored, "stored count");
    const int32_t* om = &H.omega[d.omega_off];
    const int32_t* G = om + d.nI;
    auto local_pos = [&](int c) -> int {
      if (part[c] == i) return H.locown[c];
      int lo = 0, hi = d.nG;
      while (lo < hi) { int mid = (lo + hi) / 2; if (G[mid] < c) lo = mid + 1; else hi = mid; }
      return (lo < d.nG && G[lo] == c) ? d.nIp + lo : -1;
    };
    for (int a = 0; a < d.nI; ++a) CHECK(part[om[a]] == i && H.locown[om[a]] == a, "interior order");
    // k_assemble
    for (int a = 0; a < d.nI + d.nG; ++a) {
      const int j = om[a];
      const int posa = a < d.nI ? a : d.nIp + (a - d.nI);
      for (int k = trp[j]; k < trp[j + 1]; ++k) {
        const int r = tcol[k];
        for (int e = rp[r]; e < rp[r + 1]; ++e) {
          const int posc = local_pos(ci[e]);
          if (posc < posa) continue;
          CHECK(posc < d.np, "posc");
          tp(posc / TS, posa / TS);
          if (a >= d.nI) CHECK((int64_t)(posa - d.nIp) * d.nGp + (posc - d.nIp) < (int64_t)d.nGp * d.nGp, "ct");
        }
      }
    }
    // k_chol_local / k_local_solve
    for (int J = 0; J < d.ntiles; ++J) {
      tp(J, J);
      std::vector<int> rows;
      for (int I = J + 1; I < d.ntiles; ++I) if (F[I] <= J) rows.push_back(I);
      CHECK(rows.size() <= 2048, "ROWCAP");
      maxrows = std::max<int64_t>(maxrows, rows.size());
      for (size_t x = 0; x < rows.size(); ++x) {
        tp(rows[x], J);
        for (size_t y = 0; y <= x; ++y) tp(rows[x], rows[y]);
      }
      for (int K = F[J]; K < J; ++K) tp(J, K);
    }
    // k_gamma_T
    for (int a = 0; a < d.ntiles - d.ntI; ++a)
      for (int b = 0; b <= a; ++b) {
        const int Ia = d.ntI + a, Ib = d.ntI + b;
        for (int K = std::max(F[Ia], F[Ib]); K < d.ntI; ++K) { tp(Ia, K); tp(Ib, K); }
      }
    // k_coarse_X (interior backward solve)
    for (int J = 0; J < d.ntI; ++J)
      for (int I = d.ntI; I < d.ntiles; ++I) if (F[I] <= J) tp(I, J);
    for (int I = 0; I < d.ntI; ++I) for (int K = F[I]; K < I; ++K) tp(I, K);
    CHECK(d.loc_off + d.np <= H.total_loc, "loc");
    CHECK(d.g_off + (int64_t)d.nGp * d.nGp <= H.total_g, "g");
    CHECK(d.dinv_off + (int64_t)d.ntiles * TT <= H.total_dinv, "dinv");
    CHECK(d.nG <= 1024, "eig limit");
  }
  // ---- layout of the solve factors (solve_layout in api.cpp; kernels
  // k_solve_inv, k_solve_env, k_solve_perm, k_gather_solve and the local
  // solves with a permutation).  The envelope comes from the structural
  // pattern of C_ii here, a superset of the numerical nonzeros the device
  // reads.  Both forced choices: global order everywhere, split everywhere.
  for (int mode = 0; mode < 2; ++mode) {
    std::vector<SubDesc> g(H.subs.begin(), H.subs.end());
    int64_t tb = 0, lo = 0;
    for (SubDesc& d : g) {
      const int32_t np_main = d.np;
      d.np = (d.nI + d.nG + TS - 1) / TS * TS;
      d.ntiles = d.np / TS;
      d.tile_base = tb; tb += d.ntiles;
      d.loc_off = lo; lo += std::max(np_main, d.np);
    }
    std::vector<int32_t> inv(H.total_loc, -2), Fg(tb, -1);
    std::vector<std::vector<std::pair<int, int>>> pairs(nparts);   // (posc >= posa) of C_ii
    for (int i = 0; i < nparts; ++i) {
      const SubDesc& d = H.subs[i];
      const int32_t* om = &H.omega[d.omega_off];
      const int32_t* G = om + d.nI;
      auto rank = [](const int32_t* v, int cnt, int32_t c) {
        int a = 0, b = cnt;
        while (a < b) { int mid = (a + b) / 2; if (v[mid] < c) a = mid + 1; else b = mid; }
        return a;
      };
      std::vector<char> hit(d.nI + d.nG, 0);
      for (int pos = 0; pos < d.np; ++pos) {
        int q = -1;
        if (pos < d.nI) q = pos + rank(G, d.nG, om[pos]);
        else if (pos >= d.nIp && pos < d.nIp + d.nG) q = (pos - d.nIp) + rank(om, d.nI, G[pos - d.nIp]);
        CHECK(d.loc_off + pos < H.total_loc, "inv index");
        inv[d.loc_off + pos] = q;
        if (q >= 0) { CHECK(q < d.nI + d.nG && !hit[q], "inv not a bijection in sub %d", i); hit[q] = 1; }
      }
      for (int t = 0; t < g[i].ntiles; ++t) { CHECK(g[i].tile_base + t < tb, "Fg index"); Fg[g[i].tile_base + t] = t; }
      auto local_pos = [&](int c) -> int {
        if (part[c] == i) return H.locown[c];
        const int k = rank(G, d.nG, c);
        return (k < d.nG && G[k] == c) ? d.nIp + k : -1;
      };
      for (int a = 0; a < d.nI + d.nG; ++a) {
        const int j = om[a];
        const int posa = a < d.nI ? a : d.nIp + (a - d.nI);
        for (int k = trp[j]; k < trp[j + 1]; ++k) {
          const int r = tcol[k];
          for (int e = rp[r]; e < rp[r + 1]; ++e) {
            const int posc = local_pos(ci[e]);
            if (posc < posa) continue;
            pairs[i].push_back({posc, posa});
            const int qr = inv[d.loc_off + posc], qc = inv[d.loc_off + posa];
            CHECK(qr >= 0 && qc >= 0, "pattern entry on padding");
            int32_t& f = Fg[g[i].tile_base + std::max(qr, qc) / TS];
            f = std::min(f, std::min(qr, qc) / TS);
          }
        }
      }
    }
    // choice and offsets, as in solve_layout
    std::vector<SubDesc> sd(g);
    std::vector<int32_t> sF;
    std::vector<int64_t> sOff;
    int64_t ftiles = 0, dtiles = 0, stb = 0;
    for (int i = 0; i < nparts; ++i) {
      const SubDesc& mn = H.subs[i];
      const bool use_g = mode == 0;
      SubDesc& d = sd[i];
      d.np = use_g ? g[i].np : mn.np;
      d.ntiles = use_g ? g[i].ntiles : mn.ntiles;
      d.spare = use_g;
      d.tile_base = stb; stb += d.ntiles;
      d.fac_off = ftiles * TT;
      d.dinv_off = dtiles * TT; dtiles += d.ntiles;
      int64_t run = 0;
      for (int t = 0; t < d.ntiles; ++t) {
        const int32_t f = use_g ? Fg[g[i].tile_base + t] : H.tileF[mn.tile_base + t];
        CHECK(f >= 0 && f <= t, "solve envelope start");
        sF.push_back(f);
        sOff.push_back(run);
        run += t - f + 1;
      }
      ftiles += run;
    }
    const int64_t s_total_fac = ftiles * TT, s_total_dinv = dtiles * TT;
    // k_solve_perm: every slot written at most once, inside the layout
    std::vector<int32_t> sperm(lo, -1);
    for (int i = 0; i < nparts; ++i) {
      const SubDesc& d = H.subs[i];
      const SubDesc& sv = sd[i];
      CHECK(sv.loc_off + sv.np <= lo, "solve layout slice");
      for (int pos = 0; pos < d.np; ++pos) {
        int64_t at;
        if (sv.spare) {
          const int q = inv[d.loc_off + pos];
          if (q < 0) continue;
          at = sv.loc_off + q;
        } else {
          at = sv.loc_off + pos;
        }
        CHECK(at >= 0 && at < lo && sperm[at] == -1, "sperm write in sub %d", i);
        sperm[at] = (int32_t)(d.loc_off + pos);
      }
    }
    for (int i = 0; i < nparts; ++i) {
      const SubDesc& d = H.subs[i];
      const SubDesc& sv = sd[i];
      const int32_t* F = &H.tileF[d.tile_base];
      const int64_t* off = &H.tileOff[d.tile_base];
      const int32_t* Fs = &sF[sv.tile_base];
      const int64_t* offs = &sOff[sv.tile_base];
      const int64_t fac_end = (i + 1 < nparts) ? sd[i + 1].fac_off : s_total_fac;
      const int64_t stored = (fac_end - sv.fac_off) / TT;
      const int64_t mstored = ((i + 1 < nparts ? H.subs[i + 1].fac_off : H.total_fac) - d.fac_off) / TT;
      auto stp = [&](int I, int J) -> int64_t {
        CHECK(I >= 0 && I < sv.ntiles && J <= I && J >= Fs[I], "solve tile (%d,%d) outside envelope of sub %d", I, J, i);
        const int64_t t = offs[I] + (J - Fs[I]);
        CHECK(t >= 0 && t < stored, "solve tile index");
        return t;
      };
      // every entry of C_ii lies inside the solve envelope
      for (const auto& pr : pairs[i]) {
        const int qr = sv.spare ? inv[d.loc_off + pr.first] : pr.first;
        const int qc = sv.spare ? inv[d.loc_off + pr.second] : pr.second;
        stp(std::max(qr, qc) / TS, std::min(qr, qc) / TS);
      }
      // k_gather_solve
      for (int I = 0; I < sv.ntiles; ++I)
        for (int J = Fs[I]; J <= I; ++J) {
          stp(I, J);
          for (int rc = 0; rc < TT; ++rc) {
            const int qr = I * TS + rc % TS, qc = J * TS + rc / TS;
            CHECK(qr < sv.np && qc < sv.np, "gather position");
            const int32_t pr = sperm[sv.loc_off + qr], pc = sperm[sv.loc_off + qc];
            if (pr < 0 || pc < 0) continue;
            const int64_t hi = std::max(pr, pc) - d.loc_off, lw = std::min(pr, pc) - d.loc_off;
            CHECK(hi >= 0 && hi < d.np && lw >= 0, "gather source");
            const int th = (int)(hi / TS), tl = (int)(lw / TS);
            if (tl >= F[th]) {
              const int64_t t = off[th] + (tl - F[th]);
              CHECK(t >= 0 && t < mstored, "gather main tile");
            }
          }
        }
      // the local solves: y in and out through sperm, scratch slice
      for (int q = 0; q < sv.np; ++q) {
        const int32_t ix = sperm[sv.loc_off + q];
        CHECK(ix == -1 || (ix >= d.loc_off && ix < d.loc_off + d.np), "solve position %d of sub %d", q, i);
      }
      // k_chol_local on the solve envelope
      for (int J = 0; J < sv.ntiles; ++J) {
        int rows = 0;
        for (int I = J + 1; I < sv.ntiles; ++I) if (Fs[I] <= J) { ++rows; stp(I, J); }
        CHECK(rows <= 2048, "ROWCAP (solve layout)");
      }
      CHECK(sv.dinv_off + (int64_t)sv.ntiles * TT <= s_total_dinv, "solve dinv");
    }
    printf("solve layout (%s): %lld tiles against %lld\n", mode == 0 ? "global" : "split",
           (long long)ftiles, (long long)(H.total_fac / TT));
  }
  for (size_t q = 0; q < H.own_pos.size(); ++q) CHECK(H.own_pos[q] >= 0 && H.own_pos[q] < H.total_loc, "own_pos");
  CHECK(H.own_ptr[n] == (int32_t)H.own_pos.size(), "own_ptr");
  // coarse plan with random p
  std::mt19937 rng(7);
  for (int trial = 0; trial < 3; ++trial) {
    std::vector<int32_t> ph(nparts);
    for (int i = 0; i < nparts; ++i) {
      int nG = H.subs[i].nG;
      ph[i] = (trial == 2) ? 0 : (nG ? (int)(rng() % (nG + 1)) : 0);
      if (trial == 1 && i % 3 == 0) ph[i] = 0;
    }
    HostPlan H2 = H;
    CoarsePlan C;
    plan_coarse(H2, S, m, ph, C);
    int64_t xt = 0, wt = 0;
    for (int i = 0; i < nparts; ++i) {
      const SubDesc& d = H2.subs[i];
      CHECK(d.x_off + (int64_t)d.nIp * d.p <= C.xtot, "x");
      CHECK(d.w_off + (int64_t)d.nXi * d.p <= C.wtot, "w");
      CHECK(d.p == 0 || d.cg_off + d.p <= C.segs[d.seg].c0 + C.segs[d.seg].n0, "cg");
      xt += (int64_t)d.nIp * d.p; wt += (int64_t)d.nXi * d.p;
    }
    CHECK(xt == C.xtot && wt == C.wtot, "totals");
    auto etp = [&](int64_t I, int64_t J) -> int64_t {
      CHECK(I >= 0 && I < C.etiles && J <= I && J >= C.eF[I], "E tile (%lld,%lld) outside envelope", (long long)I, (long long)J);
      int64_t t = C.eOff[I] + (J - C.eF[I]);
      CHECK(t >= 0 && t < C.efac_tiles, "E tile index");
      return t;
    };
    for (const PairDesc& pr : C.pairs) {
      const SubDesc &di = H2.subs[pr.i], &dj = H2.subs[pr.j];
      CHECK(pr.i <= pr.j && di.seg == dj.seg, "pair order/segment");
      if (pr.i != pr.j)
        for (int t = 0; t < pr.nrows; ++t) {
          CHECK(C.pair_rows[2 * (pr.rows_off + t)] < di.nXi && C.pair_rows[2 * (pr.rows_off + t) + 1] < dj.nXi, "pair rows");
          CHECK(H2.xi[di.xi_off + C.pair_rows[2 * (pr.rows_off + t)]] == H2.xi[dj.xi_off + C.pair_rows[2 * (pr.rows_off + t) + 1]], "shared row");
        }
      for (int k = 0; k < di.p; ++k)
        for (int l = 0; l < dj.p; ++l) {
          int64_t row = dj.cg_off + l, col = di.cg_off + k;
          if (pr.i == pr.j && row < col) continue;
          etp(row / TS, col / TS);
        }
    }
    for (int64_t q : C.pad_idx) CHECK(q >= 0 && q < C.efac_tiles * TT, "pad");
    CHECK(C.items.size() % 4 == 0, "items");
    for (size_t a = 0; a < C.items.size(); a += 4) {
      const int q = C.items[a], tr = C.items[a + 1], tc = C.items[a + 2];
      CHECK(q >= 0 && q < (int)C.pairs.size(), "item pair");
      const SubDesc &di = H2.subs[C.pairs[q].i], &dj = H2.subs[C.pairs[q].j];
      CHECK(tr * TS < dj.p && tc * TS < di.p, "item block");
      if (C.pairs[q].i == C.pairs[q].j) CHECK(tc <= tr, "item lower");
    }
    for (int64_t J = 0; J < C.etiles; ++J) {
      etp(J, J);
      for (int64_t a = C.eptr[J]; a < C.eptr[J + 1]; ++a) {
        etp(C.erows[a], J);
        for (int64_t b = C.eptr[J]; b <= a; ++b) etp(C.erows[a], C.erows[b]);
      }
    }
    // k_echol_step: step J reads column J - 1 for the tiles of column J and
    // updates the pairs of column J - 1's rows below J
    for (int64_t J = 0; J < C.etiles; ++J) {
      const bool prevJ = J > 0 && C.eF[J] <= J - 1;
      if (prevJ) etp(J, J - 1);
      for (int64_t a = C.eptr[J]; a < C.eptr[J + 1]; ++a) {
        const int64_t I = C.erows[a];
        CHECK(I > J, "row list of column %lld", (long long)J);
        if (prevJ && C.eF[I] <= J - 1) etp(I, J - 1);
      }
      if (J == 0) continue;
      int64_t p0 = C.eptr[J - 1], p1 = C.eptr[J];
      if (p0 < p1 && C.erows[p0] == J) ++p0;
      for (int64_t a = p0; a < p1; ++a) {
        CHECK(C.erows[a] > J, "trailing rows of column %lld", (long long)(J - 1));
        etp(C.erows[a], J - 1);
        for (int64_t b = p0; b <= a; ++b) etp(C.erows[a], C.erows[b]);
      }
    }
    for (int s = 0; s < S; ++s) {
      const SegDesc& sg = C.segs[s];
      const int64_t t0 = sg.etile0, nt = sg.etiles;
      for (int64_t c = 0; c < nt; ++c) {
        for (int64_t I = c; I < nt; ++I) for (int64_t K = std::max<int64_t>(C.eF[t0 + I] - t0, c); K < I; ++K) etp(t0 + I, t0 + K);
        for (int64_t K = nt - 1; K >= c; --K) {
          CHECK(C.eF[t0 + K] - t0 >= 0, "eF segment");
          for (int64_t u = C.eptr[t0 + K]; u < C.eptr[t0 + K + 1]; ++u) {
            const int64_t Ig = C.erows[u];
            CHECK(Ig > t0 + K && Ig < t0 + nt, "backward row outside segment");
            etp(Ig, t0 + K);
          }
        }
      }
      CHECK(sg.einv_off + nt * TS * nt * TS <= C.einv_tot, "einv");
      CHECK(sg.einv_off % TS == 0 && sg.einv_off / TS + nt * (nt * TS) <= C.einv_tot / TS, "esym partials");
    }
  }
  printf("OK subdomains=%d total_fac=%lld maxrows=%lld total_loc=%lld\n", nparts, (long long)H.total_fac, (long long)maxrows, (long long)H.total_loc);
  return 0;
}
