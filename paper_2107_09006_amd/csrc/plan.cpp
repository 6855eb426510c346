// Host-side setup planner: index sets of Section 3 (Algorithm 1, lines
// FindNonzeroRows / FindNonzeroColumns), the padded local index spaces, the
// tile envelopes of the local matrices, and the inverse overlap map used by
// the deterministic sum over overlapping subdomains.
//
// Everything here is integer work on the sparsity pattern; the floating-point
// work of the setup runs on the device.
#include "plan.hpp"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>
#include <thread>

namespace lsq2l {

static inline int32_t roundup32(int32_t x) { return (x + TS - 1) / TS * TS; }

bool plan_transpose(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* colind,
                    std::vector<int32_t>& trowptr, std::vector<int32_t>& tcol,
                    std::vector<int32_t>& tperm) {
  // Stable counting sort by column, parallel over row blocks: thread t counts
  // its rows per column, the per-(column, thread) offsets keep row blocks in
  // order, so rows ascend inside each column exactly as in a serial pass.
  const int64_t nnz = rowptr[m];
  trowptr.assign((size_t)n + 1, 0);
  tcol.resize((size_t)nnz);
  tperm.resize((size_t)nnz);
  unsigned nth = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  if (nnz < (1 << 20)) nth = 1;
  std::vector<int32_t> r0(nth + 1);
  for (unsigned t = 0; t <= nth; ++t) {
    // split rows so that every thread gets about nnz / nth entries
    const int64_t target = nnz * (int64_t)t / nth;
    r0[t] = (int32_t)(std::lower_bound(rowptr, rowptr + m + 1, target) - rowptr);
  }
  r0[nth] = m;
  std::vector<std::vector<int32_t>> cnt(nth);
  auto par = [&](auto&& fn) {
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t) pool.emplace_back(fn, t);
    for (auto& th : pool) th.join();
  };
  par([&](unsigned t) {
    cnt[t].assign((size_t)n, 0);
    for (int32_t e = rowptr[r0[t]]; e < rowptr[r0[t + 1]]; ++e) cnt[t][colind[e]]++;
  });
  // column totals, then each thread's first slot in every column
  for (int32_t j = 0; j < n; ++j) {
    int32_t tot = 0;
    for (unsigned t = 0; t < nth; ++t) tot += cnt[t][j];
    trowptr[j + 1] = tot;
  }
  for (int32_t j = 0; j < n; ++j) trowptr[j + 1] += trowptr[j];
  par([&](unsigned t) {
    const int32_t j0 = (int32_t)((int64_t)n * t / nth), j1 = (int32_t)((int64_t)n * (t + 1) / nth);
    for (int32_t j = j0; j < j1; ++j) {
      int32_t run = trowptr[j];
      for (unsigned u = 0; u < nth; ++u) { const int32_t c = cnt[u][j]; cnt[u][j] = run; run += c; }
    }
  });
  par([&](unsigned t) {
    std::vector<int32_t>& pos = cnt[t];
    for (int32_t r = r0[t]; r < r0[t + 1]; ++r)
      for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const int32_t k = pos[colind[e]]++;
        tcol[k] = r;      // rows ascend inside each column (stable)
        tperm[k] = e;     // value of A^T entry k is vals[e]
      }
  });
  return true;
}

namespace {

// A set of indices as a bitmap: mark() records an index and the range seen,
// drain() appends the marked indices in ascending order and clears them, so
// the bitmap is all zero between uses.
struct BitSet {
  std::vector<uint64_t> w;
  int64_t lo = INT64_MAX, hi = -1;
  explicit BitSet(int64_t n) : w((size_t)(n / 64 + 1), 0) {}
  void mark(int32_t x) {
    w[(size_t)x >> 6] |= 1ull << (x & 63);
    lo = std::min<int64_t>(lo, x);
    hi = std::max<int64_t>(hi, x);
  }
  void drain(std::vector<int32_t>& out) {
    for (int64_t k = lo >> 6; hi >= 0 && k <= (hi >> 6); ++k) {
      uint64_t x = w[(size_t)k];
      if (!x) continue;
      w[(size_t)k] = 0;
      while (x) {
        out.push_back((int32_t)(k * 64 + __builtin_ctzll(x)));
        x &= x - 1;
      }
    }
    lo = INT64_MAX;
    hi = -1;
  }
};

unsigned planner_threads() {
  return std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

template <typename F>
void run_threads(unsigned nth, F&& fn) {
  if (nth == 1) {
    fn(0u);
    return;
  }
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t) pool.emplace_back(fn, t);
  for (auto& th : pool) th.join();
}

// Distinct parts of the columns of row r, ascending, into buf; returns their
// number.  Row r belongs to Xi_i exactly for the parts i of this list.
inline int row_parts(const int32_t* rowptr, const int32_t* colind, const int32_t* part, int32_t r,
                     int32_t* buf) {
  int k = 0;
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int32_t v = part[colind[e]];
    int q = k;
    while (q > 0 && buf[q - 1] > v) --q;
    if (q > 0 && buf[q - 1] == v) continue;
    for (int u = k; u > q; --u) buf[u] = buf[u - 1];
    buf[q] = v;
    ++k;
  }
  return k;
}

struct LocalOut {
  std::vector<int32_t> gamma, F;
};

// Interface set and tile envelope of subdomain i, given Xi_i (ascending) and
// the rows that hold columns of several parts (bnd).  Work is proportional
// to the entries of A in the rows of Xi_i.
void plan_one(int32_t i, const int32_t* rowptr, const int32_t* colind, const int32_t* part,
              const int32_t* locown, const uint8_t* bnd, const int32_t* own_cols,
              const int32_t* fown, int32_t nI, const int32_t* xi,
              int32_t nXi, BitSet& colset, std::vector<int32_t>& f, std::vector<int32_t>& rpos,
              std::vector<int32_t>& gpos, LocalOut& out) {
  // Omega_Gamma_i: columns of A(Xi_i, :) outside Omega_Ii, ascending; only
  // rows with columns in several parts hold such columns
  out.gamma.clear();
  for (int32_t a = 0; a < nXi; ++a) {
    const int32_t r = xi[a];
    if (!bnd[r]) continue;
    for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
      if (part[colind[e]] != i) colset.mark(colind[e]);
  }
  colset.drain(out.gamma);
  const int32_t nG = (int32_t)out.gamma.size();
  // position of each interface column in Omega_Gamma_i (entries of other
  // columns are stale and never read: every column of a row of Xi_i outside
  // Omega_Ii is in Omega_Gamma_i)
  for (int32_t k = 0; k < nG; ++k) gpos[out.gamma[k]] = k;
  const int32_t nIp = roundup32(nI), np = nIp + roundup32(nG);
  // Row envelope of C_ii: f(a) = smallest local position coupled to a, the
  // minimum over the rows holding column a of the row's smallest local
  // position.  Only the rows of Xi_i are visited.  A row outside Xi_i holds
  // interface columns only, so it couples positions >= nIp among themselves;
  // every interface column also sits in a row of Xi_i next to an interior
  // column, whose position (< nIp) already bounds f there.  Such rows thus
  // never lower a tile's first column, and their entries of C_ii lie inside
  // the envelope.
  // The rows with all their columns in part i were taken into fown while
  // Xi was built (fown[c]: least position coupled to c by such rows); the
  // rows with columns in several parts are visited here.
  f.resize((size_t)np);
  for (int32_t a = 0; a < nI; ++a) f[a] = std::min(a, fown[own_cols[a]]);
  for (int32_t a = nI; a < np; ++a) f[a] = a;
  for (int32_t a = 0; a < nXi; ++a) {
    const int32_t r = xi[a];
    const int32_t e0 = rowptr[r], e1 = rowptr[r + 1];
    if (bnd[r]) {
      rpos.clear();
      int32_t best = INT32_MAX;
      for (int32_t e = e0; e < e1; ++e) {
        const int32_t c = colind[e];
        int32_t q;
        if (part[c] == i) {
          q = locown[c];
        } else {
          q = nIp + gpos[c];
        }
        rpos.push_back(q);
        best = std::min(best, q);
      }
      for (int32_t q : rpos) f[q] = std::min(f[q], best);
    }
  }
  const int32_t nt = np / TS;
  out.F.assign(nt, 0);
  for (int32_t t = 0; t < nt; ++t) {
    int32_t mn = t * TS;
    for (int32_t a = t * TS; a < (t + 1) * TS; ++a) mn = std::min(mn, f[a]);
    out.F[t] = mn / TS;
  }
}

}  // namespace

bool plan_build(int32_t m, int32_t n, const int32_t* rowptr, const int32_t* colind,
                const int32_t* part, int32_t nparts, const std::vector<int32_t>& seg_of_part,
                HostPlan& P, std::string& err, const std::function<void(int64_t)>& wait_nnz) {
  P.nparts = nparts;
  const unsigned nth = std::min<unsigned>(planner_threads(), (unsigned)std::max(nparts, 1));
  // columns of each part, ascending, and each column's position in its part:
  // a counting sort over column ranges, one per thread (each range's columns
  // follow those of the earlier ranges inside every part)
  std::vector<int64_t> pptr((size_t)nparts + 1, 0);
  HostVec<int32_t> pcols;
  if (!pcols.resize((size_t)n) || !P.locown.resize((size_t)n)) { err = "host allocation failed"; return false; }
  {
    const unsigned ct = n < (1 << 16) ? 1u : nth;
    std::vector<std::vector<int64_t>> cnt(ct, std::vector<int64_t>((size_t)nparts, 0));
    auto crange = [&](unsigned t, int32_t& a, int32_t& b) {
      a = (int32_t)((int64_t)n * t / ct);
      b = (int32_t)((int64_t)n * (t + 1) / ct);
    };
    run_threads(ct, [&](unsigned t) {
      int32_t a, b;
      crange(t, a, b);
      for (int32_t j = a; j < b; ++j) cnt[t][part[j]]++;
    });
    for (int32_t i = 0; i < nparts; ++i) {
      int64_t run = 0;
      for (unsigned t = 0; t < ct; ++t) { const int64_t c = cnt[t][i]; cnt[t][i] = run; run += c; }
      if (run == 0) { err = "part " + std::to_string(i) + " is empty"; return false; }
      pptr[i + 1] = pptr[i] + run;
    }
    run_threads(ct, [&](unsigned t) {
      int32_t a, b;
      crange(t, a, b);
      for (int32_t j = a; j < b; ++j) {
        const int32_t i = part[j];
        const int64_t r = cnt[t][i]++;          // rank of j inside part i
        pcols[pptr[i] + r] = j;
        P.locown[j] = (int32_t)r;
      }
    });
  }
  // Xi_i, row-major: row r belongs to Xi_i for every part i among its
  // columns.  Two passes over row ranges (count rows per (range, part), then
  // place them), so every Xi_i comes out ascending.  The placing pass marks
  // the rows with columns in several parts and records, for every two parts
  // i < j of such a row, the row's positions in Xi_i and Xi_j.
  const unsigned rt = m < (1 << 16) ? 1u : planner_threads();
  const int64_t nnz = rowptr[m];
  std::vector<int32_t> rb(rt + 1, m);   // row ranges of about nnz / rt entries
  for (unsigned t = 0; t < rt; ++t)
    rb[t] = (int32_t)(std::lower_bound(rowptr, rowptr + m + 1, (int32_t)(nnz * (int64_t)t / rt)) - rowptr);
  rb[rt] = m;
  // the counting pass keeps every row's list (length, then the parts) for
  // the placing pass
  // The same pass folds every row with all its columns in one part into
  // fown: for each column c, the least local position of the first column
  // of such a row through c (columns ascend in a row and locown increases
  // inside a part, so that is the row's least position).
  std::vector<std::vector<int64_t>> xcnt(rt, std::vector<int64_t>((size_t)nparts, 0));
  std::vector<HostVec<int32_t>> lists(rt);
  std::vector<uint8_t> ok(rt, 1);
  // Each thread folds its rows into a table of its own over the column
  // range its rows touch; the tables are merged by column ranges afterwards.
  std::vector<HostVec<int32_t>> fpriv(rt);
  std::vector<int32_t> flo(rt, 0), fhi(rt, -1);
  HostVec<int32_t> fown;
  if (!fown.resize((size_t)n)) { err = "host allocation failed"; return false; }
  run_threads(rt, [&](unsigned t) {
    const int32_t a = rb[t], b = std::max(rb[t], rb[t + 1]);
    if (wait_nnz) wait_nnz(rowptr[b]);       // this range's column indices are in place
    int32_t cmin = INT32_MAX, cmax = -1;
    for (int32_t e = rowptr[a]; e < rowptr[b]; ++e) {
      cmin = std::min(cmin, colind[e]);
      cmax = std::max(cmax, colind[e]);
    }
    if (cmax < cmin) cmin = 0;
    flo[t] = cmin;
    fhi[t] = cmax;
    if (!lists[t].resize((size_t)(b - a) + (size_t)(rowptr[b] - rowptr[a])) ||
        !fpriv[t].resize((size_t)std::max(cmax - cmin + 1, 1))) {
      ok[t] = 0;
      return;
    }
    int32_t* out = lists[t].data();
    const int32_t* lo = P.locown.data();
    int32_t* fo = fpriv[t].data();            // column c at c - cmin
    std::fill(fo, fo + std::max(cmax - cmin + 1, 1), INT32_MAX);
    for (int32_t r = a; r < b; ++r) {
      const int k = row_parts(rowptr, colind, part, r, out + 1);
      *out = k;
      for (int q = 0; q < k; ++q) xcnt[t][out[1 + q]]++;
      out += 1 + k;
      if (k != 1) continue;
      const int32_t best = lo[colind[rowptr[r]]];
      for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        int32_t& slot = fo[colind[e] - cmin];
        slot = std::min(slot, best);
      }
    }
  });
  for (unsigned t = 0; t < rt; ++t)
    if (!ok[t]) { err = "host allocation failed"; return false; }
  run_threads(rt, [&](unsigned t) {
    const int32_t a = (int32_t)((int64_t)n * t / rt), b = (int32_t)((int64_t)n * (t + 1) / rt);
    std::fill(fown.data() + a, fown.data() + b, INT32_MAX);
    for (unsigned u = 0; u < rt; ++u) {
      const int32_t c0 = std::max(a, flo[u]), c1 = std::min(b - 1, fhi[u]);
      const int32_t* fu = fpriv[u].data();
      for (int32_t c = c0; c <= c1; ++c) fown[c] = std::min(fown[c], fu[c - flo[u]]);
    }
  });
  fpriv.clear();
  std::vector<int64_t> xoff((size_t)nparts + 1, 0);
  for (int32_t i = 0; i < nparts; ++i) {
    int64_t run = 0;
    for (unsigned t = 0; t < rt; ++t) { const int64_t c = xcnt[t][i]; xcnt[t][i] = run; run += c; }
    xoff[i + 1] = xoff[i] + run;
  }
  if (!P.xi.resize((size_t)xoff[nparts])) { err = "host allocation failed"; return false; }
  HostVec<uint8_t> bnd;
  if (!bnd.resize((size_t)m)) { err = "host allocation failed"; return false; }
  P.shared_rows.assign(rt, {});
  run_threads(rt, [&](unsigned t) {
    std::vector<int32_t> rank(64);
    std::vector<int32_t>& rec = P.shared_rows[t];
    const int32_t* in = lists[t].data();
    for (int32_t r = rb[t]; r < rb[t + 1]; ++r) {
      const int k = *in++;
      if ((size_t)k > rank.size()) rank.resize((size_t)k);
      for (int u = 0; u < k; ++u) {
        const int64_t q = xcnt[t][in[u]]++;     // rank of r in Xi of that part
        rank[u] = (int32_t)q;
        P.xi[xoff[in[u]] + q] = r;
      }
      bnd[r] = k > 1;
      for (int u = 0; u < k; ++u)
        for (int v = u + 1; v < k; ++v) rec.insert(rec.end(), {in[u], in[v], rank[u], rank[v]});
      in += k;
    }
  });
  lists.clear();
  // interface sets and envelopes, largest subdomains first, claimed one at
  // a time by the threads
  std::vector<LocalOut> outs((size_t)nparts);
  {
    std::vector<int32_t> order((size_t)nparts);
    for (int32_t i = 0; i < nparts; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      return xoff[x + 1] - xoff[x] > xoff[y + 1] - xoff[y];
    });
    std::atomic<int32_t> next{0};
    run_threads(nth, [&](unsigned) {
      BitSet colset(n);
      std::vector<int32_t> f, rpos, gpos((size_t)n);
      for (int32_t w = next++; w < nparts; w = next++) {
        const int32_t i = order[w];
        plan_one(i, rowptr, colind, part, P.locown.data(), bnd.data(), pcols.data() + pptr[i],
                 fown.data(), (int32_t)(pptr[i + 1] - pptr[i]), P.xi.data() + xoff[i],
                 (int32_t)(xoff[i + 1] - xoff[i]), colset, f, rpos, gpos, outs[i]);
      }
    });
  }
  // offsets
  P.subs.assign((size_t)nparts, SubDesc{});
  int64_t omega_off = 0, loc_off = 0, tile_base = 0, fac_tiles = 0, g_off = 0;
  int64_t dinv_tiles = 0;
  for (int32_t i = 0; i < nparts; ++i) {
    SubDesc& d = P.subs[i];
    d.nI = (int32_t)(pptr[i + 1] - pptr[i]);
    d.nG = (int32_t)outs[i].gamma.size();
    d.nIp = roundup32(d.nI);
    d.nGp = roundup32(d.nG);
    d.np = d.nIp + d.nGp;
    d.ntiles = d.np / TS;
    d.ntI = d.nIp / TS;
    d.nXi = (int32_t)(xoff[i + 1] - xoff[i]);
    d.p = 0;
    d.seg = seg_of_part[i];
    d.id = i;
    d.omega_off = omega_off; omega_off += d.nI + d.nG;
    d.xi_off = xoff[i];
    d.loc_off = loc_off; loc_off += d.np;
    d.tile_base = tile_base; tile_base += d.ntiles;
    d.fac_off = fac_tiles * TT;
    int64_t stored = 0;
    for (int32_t t = 0; t < d.ntiles; ++t) stored += t - outs[i].F[t] + 1;
    fac_tiles += stored;
    d.dinv_off = dinv_tiles * TT; dinv_tiles += d.ntiles;   // separate array
    d.g_off = g_off; g_off += (int64_t)d.nGp * d.nGp;
  }
  if (loc_off >= (int64_t)1 << 31) { err = "local index space exceeds 2^31"; return false; }
  P.total_loc = loc_off;
  P.total_tiles = tile_base;
  P.total_fac = fac_tiles * TT;
  P.total_g = g_off;
  if (!P.omega.resize((size_t)omega_off) || !P.tileF.resize((size_t)tile_base) ||
      !P.tileOff.resize((size_t)tile_base)) {
    err = "host allocation failed";
    return false;
  }
  // per-subdomain copies into the flat arrays (disjoint ranges), in parallel
  run_threads(nth, [&](unsigned t) {
    for (int32_t i = (int32_t)t; i < nparts; i += (int32_t)nth) {
      const SubDesc& d = P.subs[i];
      std::memcpy(&P.omega[d.omega_off], pcols.data() + pptr[i], sizeof(int32_t) * d.nI);
      if (d.nG) std::memcpy(&P.omega[d.omega_off + d.nI], outs[i].gamma.data(), sizeof(int32_t) * d.nG);
      int64_t off = 0;   // relative to the subdomain's first tile (fac_off / TT)
      for (int32_t q = 0; q < d.ntiles; ++q) {
        P.tileF[d.tile_base + q] = outs[i].F[q];
        P.tileOff[d.tile_base + q] = off;
        off += q - outs[i].F[q] + 1;
      }
    }
  });
  P.total_dinv = dinv_tiles * TT;
  return true;
}

bool plan_maps(int32_t n, HostPlan& P, std::string& err) {
  const int32_t nparts = P.nparts;
  const unsigned nth = std::min<unsigned>(planner_threads(), (unsigned)std::max(nparts, 1));
  // inverse overlap map: for every column, the local positions holding it,
  // in increasing subdomain order (deterministic summation order).  Counted
  // and placed by subdomain in parallel, then every column's short list is
  // sorted: local positions grow with the subdomain index.
  if (!P.own_ptr.assign((size_t)n + 1, 0)) { err = "host allocation failed"; return false; }
  int32_t* cnt = P.own_ptr.data() + 1;
  run_threads(nth, [&](unsigned t) {
    for (int32_t i = (int32_t)t; i < nparts; i += (int32_t)nth) {
      const SubDesc& d = P.subs[i];
      for (int32_t a = 0; a < d.nI + d.nG; ++a)
        __atomic_fetch_add(&cnt[P.omega[d.omega_off + a]], 1, __ATOMIC_RELAXED);
    }
  });
  for (int32_t j = 0; j < n; ++j) P.own_ptr[j + 1] += P.own_ptr[j];
  if (!P.own_pos.resize((size_t)P.own_ptr[n])) { err = "host allocation failed"; return false; }
  {
    HostVec<int32_t> fill;
    if (!fill.resize((size_t)n)) { err = "host allocation failed"; return false; }
    std::memcpy(fill.data(), P.own_ptr.data(), sizeof(int32_t) * n);
    int32_t* fp = fill.data();
    run_threads(nth, [&](unsigned t) {
      for (int32_t i = (int32_t)t; i < nparts; i += (int32_t)nth) {
        const SubDesc& d = P.subs[i];
        for (int32_t a = 0; a < d.nI + d.nG; ++a) {
          const int32_t pos = (int32_t)(d.loc_off + (a < d.nI ? a : d.nIp + (a - d.nI)));
          P.own_pos[__atomic_fetch_add(&fp[P.omega[d.omega_off + a]], 1, __ATOMIC_RELAXED)] = pos;
        }
      }
    });
    run_threads(nth, [&](unsigned t) {
      const int32_t j0 = (int32_t)((int64_t)n * t / nth), j1 = (int32_t)((int64_t)n * (t + 1) / nth);
      for (int32_t j = j0; j < j1; ++j)
        if (P.own_ptr[j + 1] - P.own_ptr[j] > 1)
          std::sort(P.own_pos.begin() + P.own_ptr[j], P.own_pos.begin() + P.own_ptr[j + 1]);
    });
  }
  // pairs of subdomains sharing rows: ids in order of first occurrence (row
  // ranges in row order), then the rows of every pair grouped by id
  std::vector<std::vector<std::pair<int32_t, int32_t>>> adj((size_t)nparts);   // (j, id)
  std::vector<int32_t> rid;
  std::vector<int64_t> pcnt;
  P.cpair_ij.clear();
  for (const auto& rec : P.shared_rows)
    for (size_t e = 0; e < rec.size(); e += 4) {
      const int32_t i = rec[e], j = rec[e + 1];
      int32_t id = -1;
      for (const auto& pr : adj[i])
        if (pr.first == j) { id = pr.second; break; }
      if (id < 0) {
        id = (int32_t)pcnt.size();
        adj[i].push_back({j, id});
        P.cpair_ij.push_back(i);
        P.cpair_ij.push_back(j);
        pcnt.push_back(0);
      }
      ++pcnt[id];
      rid.push_back(id);
    }
  P.cpair_ptr.assign(pcnt.size() + 1, 0);
  for (size_t k = 0; k < pcnt.size(); ++k) P.cpair_ptr[k + 1] = P.cpair_ptr[k] + pcnt[k];
  P.cpair_rows.resize((size_t)(2 * P.cpair_ptr.back()));
  std::vector<int64_t> cur(P.cpair_ptr.begin(), P.cpair_ptr.end() - 1);
  size_t x = 0;
  for (const auto& rec : P.shared_rows)
    for (size_t e = 0; e < rec.size(); e += 4, ++x) {
      const int64_t at = cur[rid[x]]++;
      P.cpair_rows[2 * at] = rec[e + 2];
      P.cpair_rows[2 * at + 1] = rec[e + 3];
    }
  P.shared_rows.clear();
  P.shared_rows.shrink_to_fit();
  return true;
}

void plan_coarse(HostPlan& H, int S, int32_t m, const std::vector<int32_t>& ph, CoarsePlan& C) {
  const int nparts = H.nparts;
  C.segs.assign(S, SegDesc{});
  for (int i = 0; i < nparts; ++i) C.segs[H.subs[i].seg].n0 += ph[i];
  int64_t cglob = 0;
  for (int s = 0; s < S; ++s) {
    SegDesc& sg = C.segs[s];
    sg.c0 = cglob;
    const int64_t n0p = (sg.n0 + TS - 1) / TS * TS;
    sg.etile0 = cglob / TS;
    sg.etiles = n0p / TS;
    cglob += n0p;
  }
  std::vector<int64_t> seg_fill(S, 0);
  int64_t xoff = 0, woff = 0;
  for (int i = 0; i < nparts; ++i) {
    SubDesc& d = H.subs[i];
    d.p = ph[i];
    d.x_off = xoff; xoff += (int64_t)d.nIp * d.p;
    d.w_off = woff; woff += (int64_t)d.nXi * d.p;
    d.c_off = seg_fill[d.seg];
    d.cg_off = C.segs[d.seg].c0 + d.c_off;
    seg_fill[d.seg] += d.p;
  }
  int64_t einv_off = 0;
  C.n0 = 0;
  for (int s = 0; s < S; ++s) {
    C.segs[s].einv_off = einv_off;
    einv_off += C.segs[s].etiles * TS * C.segs[s].etiles * TS;
    C.n0 += C.segs[s].n0;
  }
  C.n0tot = cglob;
  C.etiles = cglob / TS;
  C.xtot = xoff;
  C.wtot = woff;
  C.einv_tot = einv_off;
  // pairs of subdomains with p > 0 that share rows (diagonal pairs first,
  // using all of Xi_i; then the sharing pairs in order of first occurrence)
  C.pairs.clear();
  C.pair_rows.clear();
  for (int i = 0; i < nparts; ++i)
    if (ph[i] > 0) C.pairs.push_back(PairDesc{i, i, H.subs[i].nXi, 0, 0});
  for (size_t k = 0; k + 1 < H.cpair_ptr.size(); ++k) {
    const int i = H.cpair_ij[2 * k], j = H.cpair_ij[2 * k + 1];
    if (ph[i] == 0 || ph[j] == 0) continue;
    const int64_t r0 = H.cpair_ptr[k], r1 = H.cpair_ptr[k + 1];
    C.pairs.push_back(PairDesc{i, j, (int32_t)(r1 - r0), 0, (int64_t)C.pair_rows.size() / 2});
    C.pair_rows.insert(C.pair_rows.end(), H.cpair_rows.begin() + 2 * r0, H.cpair_rows.begin() + 2 * r1);
  }
  // E assembly work items: 32 x 32 output blocks of every pair (lower blocks
  // only for diagonal pairs)
  C.items.clear();
  for (size_t q = 0; q < C.pairs.size(); ++q) {
    const int pi = H.subs[C.pairs[q].i].p, pj = H.subs[C.pairs[q].j].p;
    for (int tr = 0; tr < (pj + TS - 1) / TS; ++tr)
      for (int tc = 0; tc < (pi + TS - 1) / TS; ++tc) {
        if (C.pairs[q].i == C.pairs[q].j && tc > tr) continue;
        C.items.insert(C.items.end(), {(int32_t)q, tr, tc, 0});
      }
  }
  // envelope of E: the coarse rows of subdomain j couple to the columns of
  // every subdomain i <= j it pairs with
  std::vector<int64_t> fmin(nparts, INT64_MAX);
  for (const PairDesc& pr : C.pairs) fmin[pr.j] = std::min<int64_t>(fmin[pr.j], H.subs[pr.i].cg_off);
  std::vector<int64_t> frow(C.n0tot);
  for (int64_t q = 0; q < C.n0tot; ++q) frow[q] = q;
  for (int i = 0; i < nparts; ++i)
    for (int k = 0; k < ph[i]; ++k) frow[H.subs[i].cg_off + k] = fmin[i];
  C.eF.assign(C.etiles, 0);
  C.eOff.assign(C.etiles, 0);
  C.seg_of_tile.assign(C.etiles, 0);
  for (int s = 0; s < S; ++s)
    for (int64_t t = C.segs[s].etile0; t < C.segs[s].etile0 + C.segs[s].etiles; ++t) C.seg_of_tile[t] = s;
  int64_t tiles = 0;
  for (int64_t t = 0; t < C.etiles; ++t) {
    int64_t mn = t * TS;
    for (int64_t q = t * TS; q < (t + 1) * TS; ++q) mn = std::min(mn, frow[q]);
    C.eF[t] = (int32_t)(mn / TS);
    C.eOff[t] = tiles;
    tiles += t - C.eF[t] + 1;
  }
  C.efac_tiles = tiles;
  C.pad_idx.clear();
  for (int s = 0; s < S; ++s) {
    const SegDesc& sg = C.segs[s];
    for (int64_t q = sg.c0 + sg.n0; q < sg.c0 + sg.etiles * TS; ++q) {
      const int64_t t = q / TS;
      C.pad_idx.push_back((C.eOff[t] + (t - C.eF[t])) * TT + (q % TS) * TS + q % TS);
    }
  }
  C.erows.clear();
  C.eptr.assign(C.etiles + 1, 0);
  for (int64_t J = 0; J < C.etiles; ++J) {
    const int s = C.seg_of_tile[J];
    const int64_t tend = C.segs[s].etile0 + C.segs[s].etiles;
    for (int64_t I = J + 1; I < tend; ++I)
      if (C.eF[I] <= J) C.erows.push_back((int32_t)I);
    C.eptr[J + 1] = (int64_t)C.erows.size();
  }
}

void row_order(int32_t m, int32_t n, const int32_t* rp, const int32_t* ci, RowOrder& ro) {
  auto key = [&](int32_t i) { return rp[i] < rp[i + 1] ? ci[rp[i]] : n; };
  // far descents: the first column drops by more than ROW_ORDER_JUMP (rows
  // that jitter around a slowly moving centre keep their x gathers local)
  constexpr int32_t ROW_ORDER_JUMP = 256;
  int64_t desc = 0;
  for (int32_t i = 1; i < m; ++i) desc += key(i) < key(i - 1) - ROW_ORDER_JUMP;
  ro.use = m >= 65536 && desc * 16 > m;
  if (!ro.use) return;
  std::vector<int32_t> start((size_t)n + 2, 0);
  ro.perm.resize((size_t)m);
  ro.prp.resize((size_t)m + 1);
  for (int32_t i = 0; i < m; ++i) ++start[(size_t)key(i) + 1];
  for (size_t k = 1; k < start.size(); ++k) start[k] += start[k - 1];
  for (int32_t i = 0; i < m; ++i) ro.perm[start[key(i)]++] = i;
  ro.prp[0] = 0;
  for (int32_t i = 0; i < m; ++i) ro.prp[(size_t)i + 1] = ro.prp[i] + (rp[ro.perm[i] + 1] - rp[ro.perm[i]]);
}


}  // namespace lsq2l
