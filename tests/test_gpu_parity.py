"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars (derived in the design notes):
  * index sets, partition, coarse-space sizes p_i: bit-exact (near ties at the
    threshold, |mu - tau| <= 1e-9 tau, are reported, not asserted);
  * SpMV: |y - A x|_i <= 8 eps sum_j |A_ij x_j|;
  * preconditioner z = M r: relative error <= 1e-13 max(1, kappa(E)) (the two
    sides hold different, equally valid bases of the same coarse space, so
    the coarse solve differs at the rounding level amplified by kappa(E));
  * solution: relative error <= 1e-8 (FP64) / 1e-6 (mixed) against the oracle
    PCG at tol 1e-10, true relative residual <= tol, iterations within
    max(1, 3%) (FP64, two-level);
  * gradients: relative error <= 1e-5.
Every norm-wise comparison of a vector comes with a component-wise one
(``assert_close``): each entry's error is at most 10 tol times its own
magnitude plus the vector's root-mean-square, so that a few badly wrong
entries cannot hide under the 2-norm.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from workloads import generators as W

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="session")
def L():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need a ROCm device"
    import paper_2107_09006_amd as lib
    lib.load_library()   # raises if the HIP library is missing
    return lib


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


def assert_close(x, ref, tol):
    """||x - ref|| <= tol ||ref||, and entry-wise
    |x_i - ref_i| <= 10 tol (|ref_i| + rms(ref))."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    nrm = np.linalg.norm(ref)
    err = np.linalg.norm(x - ref)
    assert err <= tol * nrm, f"norm-wise relative error {err / nrm:.3e} > {tol:.1e}"
    rms = nrm / np.sqrt(max(ref.size, 1))
    ce = np.abs(x - ref) / (np.abs(ref) + rms)
    k = int(np.argmax(ce))
    assert ce[k] <= 10 * tol, f"component-wise error {ce[k]:.3e} at entry {k} > {10 * tol:.1e}"


PROBLEMS = {
    "worked": lambda: W.worked_example(),
    "banded_1000": lambda: W.banded_1000(),
    "banded": lambda: W.small_config("banded"),
    "grid": lambda: W.small_config("grid"),
    "irregular": lambda: W.small_config("irregular"),
    "parts32": lambda: W.random_banded(480, 960, 32, seed=232, name="parts32"),
    # interfaces of 490 columns: a non-diagonal Ct_GG (pivoted range basis)
    # and reduced problems beyond 256 (the selection's wide-interface paths)
    "wide": lambda: W.random_banded(1600, 4800, 4, seed=77, tau=0.3, half_width=160, name="wide"),
}
_cache = {}


def problem(name):
    if name not in _cache:
        _cache[name] = PROBLEMS[name]()
    return _cache[name]


def oracle(name, tau=None, variant="additive", nev_max=0):
    key = (name, tau, variant, nev_max)
    if key not in _cache:
        p = problem(name)
        _cache[key] = O.Oracle(p.scipy(), p.part, p.nparts, p.tau if tau is None else tau,
                               variant=variant, nev_max=nev_max).setup()
    return _cache[key]


def solver(L, p, **kw):
    tau = kw.pop("tau", p.tau)
    return L.Solver(p.indptr, p.indices, p.data, p.part, p.nparts, p.m, p.n, tau, **kw)


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(PROBLEMS))
def test_spmv(L, name):
    p = problem(name)
    A = p.scipy()
    s = solver(L, p, variant=L.ONE_LEVEL)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(p.n)
    y = rng.standard_normal(p.m)
    ax = _np(s.spmv(_t(x)))
    aty = _np(s.spmv(_t(y), trans=True))
    absA = abs(A)
    assert np.all(np.abs(ax - A @ x) <= 8 * EPS * (absA @ np.abs(x)) + 1e-300)
    assert np.all(np.abs(aty - A.T @ y) <= 8 * EPS * (absA.T @ np.abs(y)) + 1e-300)
    s.close()


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_index_sets_bit_exact(L, name):
    p = problem(name)
    s = solver(L, p, variant=L.ONE_LEVEL)
    sets = O.index_sets(p.scipy(), p.part, p.nparts)
    for i, st in enumerate(sets):
        d = s.subdomain(i)
        np.testing.assert_array_equal(d["I"], st.I)
        np.testing.assert_array_equal(d["Xi"], st.Xi)
        np.testing.assert_array_equal(d["G"], st.G)
    s.close()


def _near_ties(p, tau):
    """Subdomains whose interior pencil has an eigenvalue within 1e-9 tau of tau."""
    A = p.scipy()
    out = set()
    for i, st in enumerate(O.index_sets(A, p.part, p.nparts)):
        Cii, Ctii = O.local_matrices(A, st)
        _, mu = O.selection_count_schur(Cii, Ctii, st.nI, tau)
        if np.any(np.abs(mu - tau) <= 1e-9 * tau):
            out.add(i)
    return out


@pytest.mark.parametrize("name,tau", [("worked", 0.6), ("worked", 0.7), ("banded_1000", 0.1),
                                      ("banded_1000", 0.4), ("banded", 0.1), ("grid", 0.1),
                                      ("grid", 0.02), ("irregular", 0.05), ("irregular", 0.3),
                                      ("parts32", 0.1), ("wide", 0.3)])
def test_selection_count_bit_exact(L, name, tau):
    p = problem(name)
    orc = oracle(name, tau)
    s = solver(L, p, tau=tau)
    ties = _near_ties(p, tau)
    gp = [s.subdomain(i)["p"] for i in range(p.nparts)]
    for i in range(p.nparts):
        if i in ties:
            continue
        assert gp[i] == orc.p[i], (i, gp[i], orc.p[i])
    assert s.info()["n0"] == sum(gp)
    s.close()


def span_tolerance(Cii, Ctii, nI, tau):
    """Bound on the principal angle between two computed selected subspaces.

    Both sides reach the interface pencil through Ct_GG = A_IG^T A_IG and a
    factorization of C_I, so errors of eps / lambda_r (lambda_r: smallest
    retained eigenvalue of the diagonally scaled Ct_GG) and eps kappa(C_I)
    (diagonally scaled) enter the reduced matrix; the invariant subspace moves
    by that over the gap between selected and unselected mu."""
    G = Ctii[nI:, nI:]
    d = 1.0 / np.sqrt(np.diag(G))
    ev = sla.eigvalsh(G * d[:, None] * d[None, :])
    lam_r = ev[ev > G.shape[0] * EPS * ev.max()].min()
    CI = Cii[:nI, :nI]
    s = 1.0 / np.sqrt(np.diag(CI))
    kI = np.linalg.cond(CI * s[:, None] * s[None, :])
    _, mu = O.selection_count_schur(Cii, Ctii, nI, tau)
    sel, uns = mu[mu < tau], mu[mu >= tau]
    gap = (uns.min() - sel.max()) if sel.size and uns.size else 1.0
    return max(1e-10, 10 * EPS * (kI + 1.0 / lam_r) / gap)


@pytest.mark.parametrize("name", ["banded_1000", "grid", "parts32", "wide"])
def test_coarse_span_parity(L, name):
    """The GPU basis spans the same space as the oracle's (principal angles)
    and is C_I-orthonormal, within the conditioning bound of each subdomain."""
    p = problem(name)
    orc = oracle(name)
    s = solver(L, p)
    A = p.scipy()
    for i, st in enumerate(orc.sets):
        Xg = s.coarse_basis(i)
        Xo = orc.X[i]
        assert Xg.shape == Xo.shape
        if Xg.shape[1] == 0:
            continue
        Cii, Ctii = O.local_matrices(A, st)
        tol = span_tolerance(Cii, Ctii, st.nI, p.tau)
        ang = sla.subspace_angles(Xg, Xo)
        assert ang.max() <= tol, (i, ang.max(), tol)
        CI = Cii[:st.nI, :st.nI]
        G = Xg.T @ CI @ Xg
        assert np.abs(G - np.eye(G.shape[0])).max() <= max(1e-8, tol), i
    s.close()


def max_local_condition(name):
    """Largest condition number of the diagonally scaled local matrices C_ii
    (the local solves are backward stable: error ~ eps kappa)."""
    key = ("kloc", name)
    if key not in _cache:
        p = problem(name)
        A = p.scipy()
        k = 1.0
        for st in O.index_sets(A, p.part, p.nparts):
            Cii, _ = O.local_matrices(A, st)
            d = 1.0 / np.sqrt(np.diag(Cii))
            k = max(k, np.linalg.cond(Cii * d[:, None] * d[None, :]))
        _cache[key] = k
    return _cache[key]


def max_span_tolerance(name):
    """Largest span_tolerance over the subdomains that hold coarse vectors."""
    key = ("spantol", name)
    if key not in _cache:
        p = problem(name)
        orc = oracle(name)
        A = p.scipy()
        t = 0.0
        for i, st in enumerate(orc.sets):
            if orc.p[i] > 0:
                Cii, Ctii = O.local_matrices(A, st)
                t = max(t, span_tolerance(Cii, Ctii, st.nI, p.tau))
        _cache[key] = t
    return _cache[key]


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("variant", ["additive", "one_level"])
def test_preconditioner_parity(L, name, variant):
    """z = M r against the oracle.  The coarse part carries the rounding of the
    coarse solve (kappa(E) eps) and the difference between the two computed
    coarse spaces (bounded per subdomain by span_tolerance)."""
    p = problem(name)
    orc = oracle(name, variant=variant)
    s = solver(L, p, variant=L.ADDITIVE if variant == "additive" else L.ONE_LEVEL)
    r = np.random.default_rng(3).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    zr = orc.apply(r)
    tol = 10 * EPS * max_local_condition(name)
    if variant == "additive" and orc.E is not None:
        tol = max(tol, 1e-13 * np.linalg.cond(orc.E), max_span_tolerance(name))
    assert_close(z, zr, tol)
    s.close()


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("variant", ["additive", "one_level"])
def test_solve_parity_fp64(L, name, variant):
    p = problem(name)
    orc = oracle(name, variant=variant)
    ref = orc.solve(p.b, tol=1e-10)
    s = solver(L, p, tol=1e-10, variant=L.ADDITIVE if variant == "additive" else L.ONE_LEVEL)
    x, info, st = s.solve(_t(p.b))
    x = _np(x)
    assert info[0]["relres"] <= 1e-10
    assert_close(x, ref["x"], 1e-8)
    # Rounding differences (summation order) shift the iteration count of a
    # run once its Krylov basis has lost orthogonality: a few steps for the
    # two-level method, more for one-level runs of 100+ iterations, whose
    # count in finite precision is not a stable quantity.
    slack = 0.03 if variant == "additive" else 0.10
    assert abs(info[0]["iterations"] - ref["its"]) <= max(1, math.ceil(slack * ref["its"]))
    s.close()


@pytest.mark.parametrize("name", ["banded_1000", "grid", "irregular", "parts32", "wide"])
def test_solve_parity_mixed(L, name):
    p = problem(name)
    ref = oracle(name).solve(p.b, tol=1e-10)
    for flexible in (0, 1):
        s = solver(L, p, tol=1e-10, precision=L.MIXED, flexible=flexible)
        x, info, _ = s.solve(_t(p.b))
        assert info[0]["relres"] <= 1e-10
        assert_close(_np(x), ref["x"], 1e-6)
        s.close()


def test_solve_matches_dense_least_squares(L):
    p = W.banded_1000()
    s = solver(L, p, tol=1e-12)
    x, info, _ = s.solve(_t(p.b))
    xs = np.linalg.lstsq(p.scipy().toarray(), p.b, rcond=None)[0]
    assert_close(_np(x), xs, 1e-9)
    s.close()


@pytest.mark.parametrize("name", ["banded_1000", "grid", "banded"])
def test_backward_parity(L, name):
    """The adjoint converges on its backward-error rule (status OK, no
    warning) and the gradients match the oracle's within 1e-5."""
    p = problem(name)
    orc = oracle(name)
    xstar = np.random.default_rng(11).standard_normal(p.n)
    xo = orc.solve(p.b, tol=1e-11)["x"]
    go = orc.backward(p.b, xo, xo - xstar, tol=1e-11)
    s = solver(L, p, tol=1e-11)
    x, _, _ = s.solve(_t(p.b))
    dLdb, dLdv, info = s.backward(x - _t(xstar))
    assert info[0]["relres"] <= 1e-11 or info[0]["backward_err"] <= 1e-11
    assert_close(_np(dLdb), go["dLdb"], 1e-5)
    assert_close(_np(dLdv), go["dLdvals"], 1e-5)
    s.close()


def test_backward_central_differences(L):
    """Gradient of L = 1/2 ||x - x*||^2 against central differences (h = 1e-6),
    each perturbed problem set up and solved on the GPU."""
    p = W.random_banded(120, 360, 4, seed=8, k=3, half_width=8)
    xstar = np.random.default_rng(1).standard_normal(p.n)

    def loss(data, b):
        s = L.Solver(p.indptr, p.indices, data, p.part, p.nparts, p.m, p.n, 0.3, tol=1e-14,
                     max_it=1000)
        x, _, _ = s.solve(_t(b), allow_not_converged=True)
        s.close()
        return 0.5 * np.sum((_np(x) - xstar) ** 2)

    s = L.Solver(p.indptr, p.indices, p.data, p.part, p.nparts, p.m, p.n, 0.3, tol=1e-14,
                 max_it=1000)
    x, _, _ = s.solve(_t(p.b), allow_not_converged=True)
    dLdb, dLdv, _ = s.backward(x - _t(xstar))
    dLdb, dLdv = _np(dLdb), _np(dLdv)
    rng = np.random.default_rng(4001)
    h = 1e-6
    gmax = max(np.abs(dLdb).max(), np.abs(dLdv).max())
    for k in rng.choice(p.nnz, 6, replace=False):
        dp = p.data.copy(); dp[k] += h
        dm = p.data.copy(); dm[k] -= h
        fd = (loss(dp, p.b) - loss(dm, p.b)) / (2 * h)
        assert abs(fd - dLdv[k]) <= 1e-5 * max(abs(dLdv[k]), 1e-3 * gmax)
    for k in rng.choice(p.m, 6, replace=False):
        bp = p.b.copy(); bp[k] += h
        bm = p.b.copy(); bm[k] -= h
        fd = (loss(p.data, bp) - loss(p.data, bm)) / (2 * h)
        assert abs(fd - dLdb[k]) <= 1e-5 * max(abs(dLdb[k]), 1e-3 * gmax)
    s.close()


def test_autograd_function(L):
    """torch.autograd through lstsq gives the library's adjoint gradients."""
    import torch
    p = problem("banded_1000")
    s = solver(L, p, tol=1e-12)
    vals = s.vals.clone().requires_grad_(True)
    b = _t(p.b).requires_grad_(True)
    xstar = _t(np.random.default_rng(2).standard_normal(p.n))
    x = L.lstsq(vals, b, s)
    loss = 0.5 * torch.sum((x - xstar) ** 2)
    loss.backward()
    orc = oracle("banded_1000")
    xo = orc.solve(p.b, tol=1e-12)["x"]
    go = orc.backward(p.b, xo, xo - _np(xstar), tol=1e-12)
    assert_close(_np(b.grad), go["dLdb"], 1e-6)
    assert_close(_np(vals.grad), go["dLdvals"], 1e-6)
    s.close()


def test_batched_instances(L):
    probs = [W.random_banded(300 + 70 * k, 600 + 140 * k, 3 + k, seed=40 + k, name=f"b{k}")
             for k in range(5)]
    s = L.Solver.batched([(q.indptr, q.indices, q.data, q.part, q.nparts, q.m, q.n) for q in probs],
                         0.1, tol=1e-10)
    b = np.concatenate([q.b for q in probs])
    x, infos, st = s.solve(_t(b))
    x = _np(x)
    assert len(infos) == len(probs)
    off = sub = 0
    for k, q in enumerate(probs):
        orc = O.Oracle(q.scipy(), q.part, q.nparts, 0.1).setup()
        ref = orc.solve(q.b, tol=1e-10)
        assert infos[k]["relres"] <= 1e-10
        assert_close(x[off:off + q.n], ref["x"], 1e-8)
        assert abs(infos[k]["iterations"] - ref["its"]) <= 1
        for i in range(q.nparts):
            d = s.subdomain(sub + i)
            np.testing.assert_array_equal(d["I"], orc.sets[i].I + off)
            assert d["p"] == orc.p[i]
        off += q.n
        sub += q.nparts
    s.close()


def test_deterministic(L):
    p = problem("grid")
    xs = []
    for _ in range(2):
        s = solver(L, p, tol=1e-10)
        x1, _, _ = s.solve(_t(p.b))
        x2, _, _ = s.solve(_t(p.b))
        assert np.array_equal(_np(x1), _np(x2))
        xs.append(_np(x1))
        s.close()
    assert np.array_equal(xs[0], xs[1])


# ---------------------------------------------------------------------------
# special and degenerate cases
# ---------------------------------------------------------------------------

def test_single_subdomain_is_direct_solve(L):
    p = W.random_banded(200, 400, 1, seed=3)
    s = solver(L, p, tol=1e-12)
    assert s.info()["n0"] == 0
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["iterations"] == 1
    xs = np.linalg.lstsq(p.scipy().toarray(), p.b, rcond=None)[0]
    assert_close(_np(x), xs, 1e-10)
    s.close()


def test_tiny_tau_is_one_level(L):
    p = problem("banded_1000")
    s1 = solver(L, p, tau=1e-12)
    s2 = solver(L, p, variant=L.ONE_LEVEL)
    assert s1.info()["n0"] == 0
    r = _t(np.random.default_rng(5).standard_normal(p.n))
    assert np.array_equal(_np(s1.apply_preconditioner(r)), _np(s2.apply_preconditioner(r)))
    s1.close(); s2.close()


def test_tau_near_one_and_nev_cap(L):
    """tau close to 1 (tau = 1 itself sits on the multiple eigenvalue mu = 1 of
    every subdomain, a tie) and a cap on the number of vectors per subdomain."""
    p = problem("banded_1000")
    s = solver(L, p, tau=0.99)
    orc = oracle("banded_1000", tau=0.99)
    assert [s.subdomain(i)["p"] for i in range(p.nparts)] == list(orc.p)
    s.close()
    s = solver(L, p, tau=0.4, nev_max=1)
    orc = oracle("banded_1000", tau=0.4, nev_max=1)
    assert [s.subdomain(i)["p"] for i in range(p.nparts)] == list(orc.p)
    r = np.random.default_rng(6).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    assert_close(z, orc.apply(r), 1e-10)
    s.close()


def test_not_converged_returns_last_iterate(L):
    p = problem("grid")
    s = solver(L, p, max_it=2)
    x, info, st = s.solve(_t(p.b), allow_not_converged=True)
    assert st == L.NOT_CONVERGED
    assert info[0]["iterations"] == 2
    assert np.all(np.isfinite(_np(x))) and 0 < info[0]["relres"] < 1
    s.close()


def test_graph_replay_matches_eager(L):
    """A solve that replays the captured PCG iteration gives the bits and the
    iteration count of the eager loop: for two right-hand sides in a row on
    one handle (a new graph per call, eager work and a synchronisation in
    between), for the flexible variant, and with the residual read back
    every third iteration."""
    p = problem("grid")
    rng = np.random.default_rng(17)
    bs = [p.b, rng.standard_normal(p.m)]
    for kw in ({}, {"flexible": 1}, {"check_every": 3}):
        se = solver(L, p, **kw)
        sg = solver(L, p, use_graph=1, **kw)
        for b in bs:
            xe, ie, _ = se.solve(_t(b))
            xe = _np(xe).copy()
            xg, ig, _ = sg.solve(_t(b))
            xg = _np(xg).copy()
            assert ig[0]["iterations"] == ie[0]["iterations"] and ig[0]["restarts"] == ie[0]["restarts"]
            assert np.array_equal(xg, xe), kw
        se.close()
        sg.close()


def test_graph_replay_batched_matches_eager(L):
    """Batched instances with per-instance scalars and done flags: replaying
    the captured iteration gives the eager loop's bits for every instance."""
    probs = [W.random_banded(300 + 70 * k, 600 + 140 * k, 3 + k, seed=60 + k, name=f"g{k}")
             for k in range(4)]
    args = [(q.indptr, q.indices, q.data, q.part, q.nparts, q.m, q.n) for q in probs]
    b = _t(np.concatenate([q.b for q in probs]))
    se = L.Solver.batched(args, 0.1, tol=1e-10)
    sg = L.Solver.batched(args, 0.1, tol=1e-10, use_graph=1)
    xe, ie, _ = se.solve(b)
    xg, ig, _ = sg.solve(b)
    assert [i["iterations"] for i in ig] == [i["iterations"] for i in ie]
    assert np.array_equal(_np(xg), _np(xe))
    se.close()
    sg.close()


def test_csr_validation_rejects_corrupt_input(L):
    """Bad CSR input ends in EINVAL with the failing row named, for a small
    matrix (serial check) and one with more than 65536 rows (parallel
    check).  The first case has a row start beyond nnz in the middle of
    rowptr, which must not be followed into colind."""
    big = W.grid_gradient(200, 4, seed=3, tau=0.1, tol=1e-8, name="g200")
    assert big.m > 65536
    for p in (problem("banded_1000"), big):
        rp = p.indptr.copy()
        rp[len(rp) // 2] = p.indices.size + 100
        ci_range = p.indices.copy()
        ci_range[-1] = p.n
        ci_order = p.indices.copy()
        r = int(np.flatnonzero(np.diff(p.indptr) >= 2)[-1])
        a = int(p.indptr[r])
        ci_order[a], ci_order[a + 1] = ci_order[a + 1], ci_order[a]
        for rr, cc, msg in [(rp, p.indices, "monotone"), (p.indptr, ci_range, "out of range"),
                            (p.indptr, ci_order, "increasing")]:
            with pytest.raises(L.Lsq2lError) as e:
                L.Solver(rr, cc, p.data, p.part, p.nparts, p.m, p.n, 0.1)
            assert e.value.status == L.EINVAL and msg in str(e.value)


def test_device_memory_cache_reuse_is_bitwise_neutral(L):
    """Handles built on device memory taken from the cache left by destroyed
    handles give the same bits as handles on fresh allocations."""
    p = problem("grid")
    L.release_cache()
    xs = []
    for k in range(3):
        s = solver(L, p)
        x, info, _ = s.solve(_t(p.b))
        xs.append(_np(x).copy())
        s.close()
        if k == 1:
            L.release_cache()
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])


def test_error_paths(L):
    p = problem("banded_1000")
    bad = p.part.copy(); bad[0] = p.nparts
    with pytest.raises(L.Lsq2lError) as e:
        L.Solver(p.indptr, p.indices, p.data, bad, p.nparts, p.m, p.n, 0.1)
    assert e.value.status == L.EINVAL
    empty = p.part.copy(); empty[empty == 3] = 2
    with pytest.raises(L.Lsq2lError):
        L.Solver(p.indptr, p.indices, p.data, empty, p.nparts, p.m, p.n, 0.1)
    for tau in (0.0, 1.5, -1.0):
        with pytest.raises(L.Lsq2lError):
            L.Solver(p.indptr, p.indices, p.data, p.part, p.nparts, p.m, p.n, tau)
    with pytest.raises(L.Lsq2lError):
        L.Solver(p.indptr, p.indices, p.data, p.part, p.nparts, p.m, p.n, 0.1, overlap=2)
    unsorted = p.indices.copy(); unsorted[[0, 1]] = unsorted[[1, 0]]
    with pytest.raises(L.Lsq2lError):
        L.Solver(p.indptr, unsorted, p.data, p.part, p.nparts, p.m, p.n, 0.1)
    # rank deficiency: a column with no stored entry makes C singular
    keep = p.indices != 5
    rows = np.repeat(np.arange(p.m), np.diff(p.indptr))[keep]
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=p.m))]).astype(np.int32)
    with pytest.raises(L.Lsq2lError) as e:
        L.Solver(rp, p.indices[keep], p.data[keep], p.part, p.nparts, p.m, p.n, 0.1)
    assert e.value.status == L.CHOL_BREAKDOWN
    # a NaN right-hand side is a breakdown, not a silent result
    s = solver(L, p)
    b = p.b.copy(); b[7] = np.nan
    with pytest.raises(L.Lsq2lError) as e:
        s.solve(_t(b))
    assert e.value.status == L.PCG_BREAKDOWN
    s.close()


# ---------------------------------------------------------------------------
# full-size workloads in the benchmark's launch configuration
# ---------------------------------------------------------------------------

def test_full_size_grid(L):
    """The 1000 x 1000 grid with 256 patches, as timed by bench.py: both
    precisions reach 1e-8; sampled subdomains match the oracle exactly."""
    p = W.grid_1000()
    A = p.scipy()
    dev = [_t(p.data)]
    results = {}
    for prec in (L.FP64, L.MIXED):
        s = L.Solver(p.indptr, p.indices, dev[0], p.part, p.nparts, p.m, p.n, p.tau,
                     precision=prec, tol=1e-8)
        x, info, _ = s.solve(_t(p.b))
        assert info[0]["relres"] <= 1e-8
        xn = _np(x)
        r = A.T @ (p.b - A @ xn)
        rhs = A.T @ p.b
        assert np.linalg.norm(r) <= 1.5e-8 * np.linalg.norm(rhs)
        results[prec] = (s, xn, info[0])
    s = results[L.FP64][0]
    xv = np.random.default_rng(9).standard_normal(p.n)
    ax = _np(s.spmv(_t(xv)))
    assert np.all(np.abs(ax - A @ xv) <= 8 * EPS * (abs(A) @ np.abs(xv)) + 1e-300)
    picks = (0, 119, 255)      # corner, interior (four-sided interface) and last patch
    sets = dict(zip(picks, O.index_sets(A, p.part, p.nparts, subdomains=picks)))
    for i in picks:
        d = s.subdomain(i)
        np.testing.assert_array_equal(d["I"], sets[i].I)
        np.testing.assert_array_equal(d["Xi"], sets[i].Xi)
        np.testing.assert_array_equal(d["G"], sets[i].G)
    assert sets[119].nG == 252
    for i in (0, 119):          # the oracle's eigenproblem on sampled subdomains
        d = s.subdomain(i)
        Cii, Ctii = O.local_matrices(A, sets[i])
        res = O.coarse_vectors(Cii, Ctii, sets[i].nI, p.tau)
        assert d["p"] == res["p"], (i, d["p"], res["p"])
        ang = sla.subspace_angles(s.coarse_basis(i), res["X"])
        assert ang.max() <= span_tolerance(Cii, Ctii, sets[i].nI, p.tau)
    for prec in results:
        results[prec][0].close()
