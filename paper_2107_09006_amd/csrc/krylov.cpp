// The Krylov methods of Section 4.1 ("Solution phase") besides CG:
// left-preconditioned LSQR on min ||A x - b|| and right-preconditioned
// restarted GMRES on the normal equations C x = A^T b (eq. normal), both for
// many independent instances at once (per-instance scalars and convergence).
// The vector work runs in the kernels of k_krylov.hip; the small per-instance
// Hessenberg least-squares problems of GMRES are solved on the host.
//
// Also here: the symbolic count of sum_i nnz(L_i) under a fill-reducing
// order of every subdomain (the algorithmic minimum of the local solves).
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "krylov.hpp"

namespace lsq2l {

lsq2l_status krylov_alloc(lsq2l_ctx* c) {
  const int S = c->S;
  const int64_t m = c->M.m, n = c->M.n;
  if (c->opt.krylov == LSQ2L_LSQR) {
    LsqrWork& L = c->lsqr;
    TRY(c->dalloc(&L.u, m));
    TRY(c->dalloc(&L.Av, m));
    TRY(c->dalloc(&L.v, n));
    TRY(c->dalloc(&L.zh, n));
    TRY(c->dalloc(&L.w, n));
    TRY(c->dalloc(&L.q, n));
    TRY(c->dalloc(&L.s, n));
    TRY(c->dalloc(&L.sc, (int64_t)S * LSQR_NSC));
  }
  if (c->opt.krylov == LSQ2L_GMRES) {
    GmresWork& G = c->gmres;
    G.restart = c->opt.restart;
    const int ld = G.restart + 1;
    TRY(c->dalloc(&G.V, (int64_t)ld * n));
    TRY(c->dalloc(&G.w, n));
    TRY(c->dalloc(&G.z, n));
    TRY(c->dalloc(&G.t, n));
    TRY(c->dalloc(&G.part, (int64_t)S * RED_BLOCKS * ld));
    TRY(c->dalloc(&G.h, (int64_t)S * ld));
    TRY(c->dalloc(&G.y, (int64_t)S * ld));
    TRY(c->dalloc(&G.nrm, S));
    TRY(c->halloc(&G.h_h, (int64_t)S * ld + S));
    TRY(c->halloc(&G.h_y, (int64_t)S * ld));
  }
  return LSQ2L_OK;
}

// ---------------------------------------------------------------------------
// LSQR
// ---------------------------------------------------------------------------
lsq2l_status lsqr(lsq2l_ctx* c, const double* b, double* x, double tol, KrylovResult& res) {
  const hipStream_t st = c->st;
  const int S = c->S;
  const int64_t m = c->M.m, n = c->M.n;
  LsqrWork& L = c->lsqr;
  int32_t* done = c->sc.done;
  int32_t* its = c->sc.its;
  launch_fill(st, n, 0.0, x);
  // beta_1 u_1 = b
  launch_copy(st, m, b, L.u);
  launch_dot(st, S, c->d_seg_row, L.u, L.u, c->partial);
  launch_lsqr_scalar(st, LSQR_INIT_BETA, S, c->partial, L.sc, done, its, tol);
  launch_lsqr_unorm(st, m, S, c->d_seg_row, L.sc, done, L.u);
  // alpha_1: q = A^T u_1, s = M q, alpha_1 = sqrt(q^T s)
  spmv_AT(c, L.u, L.q);
  launch_lsqr_q(st, n, S, c->d_seg_col, L.sc, done, L.zh, L.q, 1);
  apply_M(c, L.q, L.s);
  launch_dot(st, S, c->d_seg_col, L.q, L.s, c->partial);
  launch_lsqr_scalar(st, LSQR_INIT_ALPHA, S, c->partial, L.sc, done, its, tol);
  launch_lsqr_update(st, n, S, c->d_seg_col, L.sc, done, L.q, L.s, L.zh, L.v, L.w, x, 1);
  std::vector<int32_t> hd(S);
  auto flags = [&](bool& all_stop, bool& brk) -> lsq2l_status {
    LSQ2L_HIP_TRY(hipMemcpyAsync(hd.data(), done, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
    LSQ2L_HIP_TRY(hipStreamSynchronize(st));
    all_stop = true;
    brk = false;
    for (int s = 0; s < S; ++s) {
      all_stop &= hd[s] != 0;
      brk |= hd[s] == 2;
    }
    return LSQ2L_OK;
  };
  bool all_stop = false, brk = false;
  TRY(flags(all_stop, brk));
  int it = 0;
  while (!all_stop && it < c->opt.max_it) {
    // beta u = A vt - alpha u
    spmv_A(c, L.v, L.Av);
    launch_lsqr_u(st, m, S, c->d_seg_row, L.sc, done, L.Av, L.u, 0);
    launch_dot(st, S, c->d_seg_row, L.u, L.u, c->partial);
    launch_lsqr_scalar(st, LSQR_BETA, S, c->partial, L.sc, done, its, tol);
    launch_lsqr_unorm(st, m, S, c->d_seg_row, L.sc, done, L.u);
    // alpha: q = A^T u - beta zh, s = M q
    spmv_AT(c, L.u, L.q);
    launch_lsqr_q(st, n, S, c->d_seg_col, L.sc, done, L.zh, L.q, 0);
    apply_M(c, L.q, L.s);
    launch_dot(st, S, c->d_seg_col, L.q, L.s, c->partial);
    launch_lsqr_scalar(st, LSQR_ALPHA, S, c->partial, L.sc, done, its, tol);
    launch_lsqr_update(st, n, S, c->d_seg_col, L.sc, done, L.q, L.s, L.zh, L.v, L.w, x, 0);
    ++it;
    if (it % std::max(1, c->opt.check_every) == 0 || it >= c->opt.max_it) TRY(flags(all_stop, brk));
  }
  TRY(flags(all_stop, brk));
  std::vector<double> hsc((size_t)S * LSQR_NSC);
  LSQ2L_HIP_TRY(hipMemcpyAsync(hsc.data(), L.sc, sizeof(double) * hsc.size(), hipMemcpyDeviceToHost, st));
  res.its.resize(S);
  LSQ2L_HIP_TRY(hipMemcpyAsync(res.its.data(), its, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  TRY(true_residual(c, x, res.relres, nullptr));
  res.relres_rec.resize(S);
  res.converged.resize(S);
  res.backward_err.assign(S, 0.0);
  for (int s = 0; s < S; ++s) {
    res.relres_rec[s] = hsc[(size_t)s * LSQR_NSC + LS_TEST];
    res.converged[s] = hd[s] == 1 || hd[s] == 3;
  }
  res.total_its = it;
  res.restarts = 0;
  if (brk) { set_error("LSQR breakdown (non-finite value or an indefinite preconditioner)"); return LSQ2L_PCG_BREAKDOWN; }
  for (int s = 0; s < S; ++s)
    if (!res.converged[s]) { set_error("LSQR did not reach the tolerance within max_it iterations"); return LSQ2L_NOT_CONVERGED; }
  return LSQ2L_OK;
}

// ---------------------------------------------------------------------------
// GMRES(restart), right preconditioning: x = x_0 + M V y minimizes
// ||rhs - C x|| over the Krylov space of C M; classical Gram-Schmidt applied
// twice, Givens rotations on the host
// ---------------------------------------------------------------------------
lsq2l_status gmres(lsq2l_ctx* c, double* x, bool adjoint, double tol, KrylovResult& res) {
  const hipStream_t st = c->st;
  const int S = c->S;
  const int64_t n = c->M.n;
  GmresWork& G = c->gmres;
  const int R = G.restart, ld = R + 1;
  launch_fill(st, n, 0.0, x);
  std::vector<double> rhs2, x2(S, 0.0), beta(S);
  launch_dot(st, S, c->d_seg_col, c->rhs, c->rhs, c->partial);
  TRY(read_seg_sums(c, c->partial, rhs2));
  std::vector<int32_t> state(S, 0);        // 0 active, 1 converged, 2 breakdown
  std::vector<int32_t> its(S, 0);
  std::vector<double> est(S, 0.0);
  std::vector<std::vector<double>> Rm(S, std::vector<double>((size_t)R * R, 0.0));
  std::vector<std::vector<double>> g(S, std::vector<double>(ld, 0.0));
  std::vector<std::vector<double>> cs(S, std::vector<double>(R, 0.0)), sn(S, std::vector<double>(R, 0.0));
  std::vector<int32_t> kcol(S, 0), stop(S, 0), hdone(S, 0);
  int total = 0, cycles = 0;
  // relative residual; an adjoint instance whose true residual stalls (less
  // than a halving over a whole cycle) is accepted on its normwise backward
  // error ||rhs - C x|| / (||C||_2 ||x|| + ||rhs||) <= tol
  auto bound = [&](int s) { return tol * std::sqrt(rhs2[s]); };
  auto bwd = [&](int s) {
    const double b = c->normC[s] * std::sqrt(x2[s]) + std::sqrt(rhs2[s]);
    return b > 0 ? beta[s] / b : 0.0;
  };
  std::vector<double> prev_beta(S, INFINITY);
  while (true) {
    // true residual w = rhs - C x of every instance
    apply_C(c, x, c->q, c->tm);
    launch_sub(st, n, c->rhs, c->q, G.w);
    std::vector<double> r2;
    launch_dot(st, S, c->d_seg_col, G.w, G.w, c->partial);
    TRY(read_seg_sums(c, c->partial, r2));
    if (adjoint) {
      launch_dot(st, S, c->d_seg_col, x, x, c->partial);
      TRY(read_seg_sums(c, c->partial, x2));
    }
    bool all_stop = true;
    for (int s = 0; s < S; ++s) {
      beta[s] = std::sqrt(r2[s]);
      if (state[s] == 2) continue;
      if (!std::isfinite(beta[s])) { state[s] = 2; continue; }
      state[s] = beta[s] <= bound(s) ? 1 : 0;
      if (adjoint && state[s] == 0 && beta[s] > 0.5 * prev_beta[s] && bwd(s) <= tol) state[s] = 1;
      prev_beta[s] = beta[s];
      all_stop &= state[s] != 0;
    }
    if (all_stop || total >= c->opt.max_it) break;
    // V_0 = w / beta on the active instances (zero elsewhere)
    for (int s = 0; s < S; ++s) hdone[s] = state[s] != 0;
    LSQ2L_HIP_TRY(hipMemcpyAsync(c->sc.done, hdone.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, st));
    launch_dot(st, S, c->d_seg_col, G.w, G.w, c->partial);
    launch_seg_sum(st, S, c->partial, G.nrm);
    launch_normalize_seg(st, n, S, c->d_seg_col, G.nrm, c->sc.done, G.w, G.V);
    for (int s = 0; s < S; ++s) {
      std::fill(g[s].begin(), g[s].end(), 0.0);
      g[s][0] = beta[s];
      kcol[s] = 0;
      stop[s] = state[s] != 0;
    }
    int j = 0;
    for (; j < R && total < c->opt.max_it; ++j) {
      const double* Vj = G.V + (int64_t)j * n;
      apply_M(c, Vj, G.z);
      apply_C(c, G.z, G.w, c->tm);
      // two passes of classical Gram-Schmidt against V_0 .. V_j
      launch_multidot(st, S, c->d_seg_col, n, j + 1, G.V, G.w, G.part, ld);
      launch_multidot_reduce(st, S, j + 1, G.part, ld, G.h, 0);
      launch_multi_axpy(st, S, c->d_seg_col, n, j + 1, G.V, G.h, ld, G.w);
      launch_multidot(st, S, c->d_seg_col, n, j + 1, G.V, G.w, G.part, ld);
      launch_multidot_reduce(st, S, j + 1, G.part, ld, G.y, 0);
      launch_multi_axpy(st, S, c->d_seg_col, n, j + 1, G.V, G.y, ld, G.w);
      launch_multidot_reduce(st, S, j + 1, G.part, ld, G.h, 1);
      launch_dot(st, S, c->d_seg_col, G.w, G.w, c->partial);
      launch_seg_sum(st, S, c->partial, G.nrm);
      launch_normalize_seg(st, n, S, c->d_seg_col, G.nrm, c->sc.done, G.w, G.V + (int64_t)(j + 1) * n);
      LSQ2L_HIP_TRY(hipMemcpyAsync(G.h_h, G.h, sizeof(double) * S * ld, hipMemcpyDeviceToHost, st));
      LSQ2L_HIP_TRY(hipMemcpyAsync(G.h_h + (size_t)S * ld, G.nrm, sizeof(double) * S, hipMemcpyDeviceToHost, st));
      LSQ2L_HIP_TRY(hipStreamSynchronize(st));
      ++total;
      bool cycle_done = true;
      for (int s = 0; s < S; ++s) {
        if (stop[s]) continue;
        std::vector<double> h(j + 2);
        for (int i = 0; i <= j; ++i) h[i] = G.h_h[(size_t)s * ld + i];
        h[j + 1] = std::sqrt(std::max(0.0, G.h_h[(size_t)S * ld + s]));
        bool finite = true;
        for (double v : h) finite &= std::isfinite(v);
        if (!finite) { state[s] = 2; stop[s] = 1; continue; }
        for (int i = 0; i < j; ++i) {               // earlier rotations
          const double t = cs[s][i] * h[i] + sn[s][i] * h[i + 1];
          h[i + 1] = -sn[s][i] * h[i] + cs[s][i] * h[i + 1];
          h[i] = t;
        }
        const double rr = std::hypot(h[j], h[j + 1]);
        cs[s][j] = rr > 0 ? h[j] / rr : 1.0;
        sn[s][j] = rr > 0 ? h[j + 1] / rr : 0.0;
        h[j] = rr;
        g[s][j + 1] = -sn[s][j] * g[s][j];
        g[s][j] = cs[s][j] * g[s][j];
        for (int i = 0; i <= j; ++i) Rm[s][(size_t)j * R + i] = h[i];
        kcol[s] = j + 1;
        its[s] += 1;
        est[s] = std::fabs(g[s][j + 1]);
        // the estimate against the bound at the start of the cycle; an
        // invariant subspace (h_{j+1,j} = 0) ends the instance's cycle too
        if (est[s] <= bound(s) || G.h_h[(size_t)S * ld + s] <= 0.0 || rr == 0.0) stop[s] = 1;
        if (!stop[s]) cycle_done = false;
      }
      if (cycle_done) { ++j; break; }
    }
    // x += M (V y), y = R^{-1} g per instance
    std::fill(G.h_y, G.h_y + (size_t)S * ld, 0.0);
    int kmax = 0;
    for (int s = 0; s < S; ++s) {
      if (state[s] != 0 || kcol[s] == 0) continue;
      const int k = kcol[s];
      double* y = G.h_y + (size_t)s * ld;
      for (int i = k - 1; i >= 0; --i) {
        double t = g[s][i];
        for (int q = i + 1; q < k; ++q) t -= Rm[s][(size_t)q * R + i] * y[q];
        const double d = Rm[s][(size_t)i * R + i];
        y[i] = d != 0.0 ? t / d : 0.0;
      }
      kmax = std::max(kmax, k);
    }
    ++cycles;
    if (kmax > 0) {
      LSQ2L_HIP_TRY(hipMemcpyAsync(G.y, G.h_y, sizeof(double) * S * ld, hipMemcpyHostToDevice, st));
      launch_multi_gemv(st, S, c->d_seg_col, n, kmax, G.V, G.y, ld, G.t);
      apply_M(c, G.t, G.z);
      launch_add(st, n, x, G.z, x);
      LSQ2L_HIP_TRY(hipStreamSynchronize(st));   // h_y is reused by the next cycle
    }
    (void)j;
  }
  res.its = its;
  res.restarts = cycles;
  res.total_its = total;
  res.relres.resize(S);
  res.relres_rec.resize(S);
  res.backward_err.assign(S, 0.0);
  res.converged.resize(S);
  bool brk = false;
  for (int s = 0; s < S; ++s) {
    const double b = std::sqrt(rhs2[s]);
    res.relres[s] = b > 0 ? beta[s] / b : 0.0;
    res.relres_rec[s] = b > 0 ? est[s] / b : 0.0;
    if (adjoint) {
      const double bd = c->normC[s] * std::sqrt(x2[s]) + b;
      res.backward_err[s] = bd > 0 ? beta[s] / bd : 0.0;
    }
    res.converged[s] = state[s] == 1;
    brk |= state[s] == 2;
  }
  if (brk) { set_error("GMRES breakdown (non-finite value)"); return LSQ2L_PCG_BREAKDOWN; }
  for (int s = 0; s < S; ++s)
    if (!res.converged[s]) { set_error("GMRES did not reach the tolerance within max_it iterations"); return LSQ2L_NOT_CONVERGED; }
  return LSQ2L_OK;
}

// ---------------------------------------------------------------------------
// sum_i nnz(L_i) under a fill-reducing order of Omega_i (the best of
// nested dissection, the global column order and [Omega_Ii, Omega_Gamma_i])
// ---------------------------------------------------------------------------
namespace {

// Nested dissection of the vertices `set` of the graph (adjacency lists
// adj over local vertices; `inset` marks membership): a BFS from a
// pseudo-peripheral vertex (the last vertex reached by a BFS from the first,
// taken twice), the middle level as separator, then both sides recursively;
// the order is side 1, side 2, separator.  Components not reached by the BFS
// are ordered on their own, first.
void nested_dissection(const std::vector<std::vector<int32_t>>& adj, std::vector<int32_t> set,
                       std::vector<char>& inset, std::vector<int32_t>& level,
                       std::vector<int32_t>& out) {
  if (set.size() <= 64) {
    std::sort(set.begin(), set.end());
    out.insert(out.end(), set.begin(), set.end());
    return;
  }
  for (int32_t v : set) inset[v] = 1;
  auto bfs = [&](int32_t root, std::vector<int32_t>& order) {
    order.clear();
    for (int32_t v : set) level[v] = -1;
    level[root] = 0;
    order.push_back(root);
    for (size_t h = 0; h < order.size(); ++h) {
      const int32_t u = order[h];
      for (int32_t w : adj[u])
        if (inset[w] && level[w] < 0) {
          level[w] = level[u] + 1;
          order.push_back(w);
        }
    }
  };
  std::vector<int32_t> order;
  int32_t root = *std::min_element(set.begin(), set.end());
  bfs(root, order);
  if (order.size() < set.size()) {
    // the component of root, then the rest
    std::vector<int32_t> comp = order, rest;
    for (int32_t v : set)
      if (level[v] < 0) rest.push_back(v);
    for (int32_t v : set) inset[v] = 0;
    nested_dissection(adj, rest, inset, level, out);
    nested_dissection(adj, comp, inset, level, out);
    return;
  }
  for (int pass = 0; pass < 2; ++pass) {
    root = order.back();
    bfs(root, order);
  }
  const int32_t nlev = level[order.back()] + 1;
  for (int32_t v : set) inset[v] = 0;
  if (nlev < 3) {                      // no useful separator: keep as is
    std::sort(set.begin(), set.end());
    out.insert(out.end(), set.begin(), set.end());
    return;
  }
  // middle level: where the cumulative count passes half
  std::vector<int64_t> cnt(nlev, 0);
  for (int32_t v : set) cnt[level[v]]++;
  int64_t acc = 0;
  int32_t mid = 1;
  for (int32_t l = 0; l < nlev; ++l) {
    acc += cnt[l];
    if (2 * acc >= (int64_t)set.size()) { mid = std::min(std::max(l, 1), nlev - 2); break; }
  }
  std::vector<int32_t> a, b, sep;
  for (int32_t v : set) {
    if (level[v] < mid) a.push_back(v);
    else if (level[v] > mid) b.push_back(v);
    else sep.push_back(v);
  }
  nested_dissection(adj, a, inset, level, out);
  nested_dissection(adj, b, inset, level, out);
  std::sort(sep.begin(), sep.end());
  out.insert(out.end(), sep.begin(), sep.end());
}

// nnz of the Cholesky factor (diagonal included) of the matrix with
// adjacency adj eliminated in the order ord: the structure of column k is
// its later neighbours merged with the structures of its children in the
// elimination tree
int64_t symbolic_nnz(const std::vector<std::vector<int32_t>>& adj, const std::vector<int32_t>& ord) {
  const int32_t nv = (int32_t)ord.size();
  std::vector<int32_t> pos(nv);
  for (int32_t k = 0; k < nv; ++k) pos[ord[k]] = k;
  std::vector<std::vector<int32_t>> st(nv), children(nv);
  std::vector<int32_t> stamp(nv, -1);
  int64_t total = 0;
  for (int32_t k = 0; k < nv; ++k) {
    std::vector<int32_t> s;
    for (int32_t w : adj[ord[k]]) {
      const int32_t p = pos[w];
      if (p > k && stamp[p] != k) { stamp[p] = k; s.push_back(p); }
    }
    for (int32_t ch : children[k]) {
      for (int32_t p : st[ch])
        if (p != k && stamp[p] != k) { stamp[p] = k; s.push_back(p); }
      std::vector<int32_t>().swap(st[ch]);
    }
    total += (int64_t)s.size() + 1;
    if (!s.empty()) children[*std::min_element(s.begin(), s.end())].push_back(k);
    st[k] = std::move(s);
  }
  return total;
}

}  // namespace

lsq2l_status factor_nnz_min(lsq2l_ctx* c) {
  if (c->fac_nnz_min >= 0) return LSQ2L_OK;
  const hipStream_t st = c->st;
  const int32_t m = c->M.m, n = c->M.n;
  const int64_t nnz = c->M.nnz;
  std::vector<int32_t> rp(m + 1), ci(nnz), trp(n + 1), tr(nnz), part(n);
  LSQ2L_HIP_TRY(hipMemcpyAsync(rp.data(), c->M.rowptr, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(ci.data(), c->M.colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(trp.data(), c->M.trowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(tr.data(), c->M.trow, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipMemcpyAsync(part.data(), c->P.part, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  LSQ2L_HIP_TRY(hipStreamSynchronize(st));
  const HostPlan& H = c->H;
  const int nsub = c->nsub;
  std::vector<int64_t> per(nsub, 0);
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nth = std::min<unsigned>(nth, (unsigned)nsub);
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t)
    pool.emplace_back([&, t]() {
      std::vector<int32_t> lpos(n, -1);
      for (int i = (int)t; i < nsub; i += (int)nth) {
        const SubDesc& d = H.subs[i];
        const int32_t ni = d.nI + d.nG;
        const int32_t* om = &H.omega[d.omega_off];
        for (int32_t a = 0; a < ni; ++a) lpos[om[a]] = a;
        // adjacency of C_ii: local columns sharing a row of A
        std::vector<std::vector<int32_t>> adj(ni);
        std::vector<int32_t> stamp(ni, -1);
        for (int32_t a = 0; a < ni; ++a) {
          const int32_t j = om[a];
          for (int32_t k = trp[j]; k < trp[j + 1]; ++k) {
            const int32_t r = tr[k];
            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
              const int32_t b = lpos[ci[e]];
              if (b >= 0 && b != a && stamp[b] != a) { stamp[b] = a; adj[a].push_back(b); }
            }
          }
        }
        for (int32_t a = 0; a < ni; ++a) lpos[om[a]] = -1;
        // the local solves may use any order of Omega_i: the fewest entries
        // among a nested-dissection order of all of Omega_i, the global
        // column order and [Omega_Ii, Omega_Gamma_i]
        std::vector<int32_t> all(ni), ord;
        for (int32_t a = 0; a < ni; ++a) all[a] = a;
        std::vector<char> inset(ni, 0);
        std::vector<int32_t> level(ni, -1);
        ord.reserve(ni);
        nested_dissection(adj, all, inset, level, ord);
        int64_t best = symbolic_nnz(adj, ord);
        best = std::min(best, symbolic_nnz(adj, all));
        std::vector<int32_t> byc(all);
        std::sort(byc.begin(), byc.end(), [&](int32_t x, int32_t y) { return om[x] < om[y]; });
        per[i] = std::min(best, symbolic_nnz(adj, byc));
      }
    });
  for (auto& th : pool) th.join();
  int64_t tot = 0;
  for (int64_t v : per) tot += v;
  c->fac_nnz_min = tot;
  c->info.factor_nnz_min = tot;
  return LSQ2L_OK;
}

}  // namespace lsq2l
