"""Local factors from thin QR factorizations and the principal-angle coarse
selection (Remarks 3.1 and 3.2: no C_ii formed), against the oracle's QR
route (``Oracle(local_factor="qr")``):

  * the selection counts p_i, bit-exact (angles within 1e-9 tau of tau skipped);
  * the coarse spans, by principal angles, and C_I-orthonormality;
  * z = M r element by element (one-level and additive), in both orders of the
    solve factors, and in the mixed path (FP64 QR factors rounded to float);
  * the PCG solve;
  * a subdomain above the streaming local solve's 12,544 unknowns (checked
    against the Cholesky oracle: both factor the same C_ii);
  * the balanced, RAS and deflated forms, LSQR and GMRES, and a batch of
    instances in one handle;
  * the option's restrictions.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from tests.test_gpu_parity import (L, _np, _t, assert_close, max_local_condition,  # noqa: F401
                                   problem, span_tolerance, solver)
from tests.test_gpu_solve_order import _above_cap

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)
NAMES = ["worked", "banded_1000", "banded", "grid", "irregular", "parts32", "wide"]
_qcache = {}


def qr_oracle(name, tau=None, variant="additive"):
    key = (name, tau, variant)
    if key not in _qcache:
        p = problem(name)
        _qcache[key] = O.Oracle(p.scipy(), p.part, p.nparts, p.tau if tau is None else tau,
                                variant=variant, local_factor="qr").setup()
    return _qcache[key]


def _angle_ties(p, tau):
    A = p.scipy()
    out = set()
    for i, st in enumerate(O.index_sets(A, p.part, p.nparts)):
        mu = O.coarse_vectors_angles(A, st, tau)["mu"]
        if np.any(np.abs(mu - tau) <= 1e-9 * tau):
            out.add(i)
    return out


def _qr_tol(name, orc):
    tol = 10 * EPS * max_local_condition(name)
    if orc.E is not None:
        p = problem(name)
        A = p.scipy()
        st = 0.0
        for i, s in enumerate(orc.sets):
            if orc.p[i] > 0:
                Cii, Ctii = O.local_matrices(A, s)
                st = max(st, span_tolerance(Cii, Ctii, s.nI, p.tau))
        tol = max(tol, 1e-13 * np.linalg.cond(orc.E), st)
    return tol


@pytest.mark.parametrize("name,tau", [("worked", 0.6), ("worked", 0.7), ("banded_1000", 0.1),
                                      ("banded_1000", 0.4), ("banded", 0.1), ("grid", 0.1),
                                      ("grid", 0.02), ("irregular", 0.05), ("irregular", 0.3),
                                      ("parts32", 0.1), ("wide", 0.3)])
def test_qr_selection_count_bit_exact(L, name, tau):
    p = problem(name)
    orc = qr_oracle(name, tau)
    s = solver(L, p, tau=tau, local_factor=L.FACTOR_QR)
    ties = _angle_ties(p, tau)
    gp = [s.subdomain(i)["p"] for i in range(p.nparts)]
    for i in range(p.nparts):
        if i not in ties:
            assert gp[i] == orc.p[i], (i, gp[i], orc.p[i])
    assert s.info()["n0"] == sum(gp)
    s.close()


@pytest.mark.parametrize("name", ["banded_1000", "grid", "parts32", "wide"])
def test_qr_coarse_span(L, name):
    p = problem(name)
    orc = qr_oracle(name)
    s = solver(L, p, local_factor=L.FACTOR_QR)
    A = p.scipy()
    for i, st in enumerate(orc.sets):
        Xg = s.coarse_basis(i)
        Xo = orc.X[i]
        assert Xg.shape == Xo.shape
        if Xg.shape[1] == 0:
            continue
        Cii, Ctii = O.local_matrices(A, st)
        tol = span_tolerance(Cii, Ctii, st.nI, p.tau)
        assert sla.subspace_angles(Xg, Xo).max() <= tol, i
        CI = Cii[:st.nI, :st.nI]
        G = Xg.T @ CI @ Xg
        assert np.abs(G - np.eye(G.shape[0])).max() <= max(1e-8, tol), i
    s.close()


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("order", ["split", "global", "auto"])
@pytest.mark.parametrize("variant", ["one_level", "additive"])
def test_qr_preconditioner(L, name, order, variant):
    p = problem(name)
    orc = qr_oracle(name, variant=variant)
    opts = {"split": L.ORDER_SPLIT, "global": L.ORDER_GLOBAL, "auto": L.ORDER_AUTO}
    s = solver(L, p, variant=L.ADDITIVE if variant == "additive" else L.ONE_LEVEL,
               local_factor=L.FACTOR_QR, solve_order=opts[order])
    inf = s.info()
    if order == "split":
        assert inf["solve_permuted"] == 0
    elif order == "global":
        assert inf["solve_permuted"] == p.nparts
    r = np.random.default_rng(5).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    tol = 10 * EPS * max_local_condition(name) if variant == "one_level" else _qr_tol(name, orc)
    assert_close(z, orc.apply(r), tol)
    s.close()


@pytest.mark.parametrize("name", NAMES)
def test_qr_solve(L, name):
    p = problem(name)
    ref = qr_oracle(name).solve(p.b, tol=1e-10)
    s = solver(L, p, tol=1e-10, local_factor=L.FACTOR_QR)
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-8)
    s.close()


@pytest.mark.parametrize("name", ["banded_1000", "grid", "irregular", "wide"])
def test_qr_mixed(L, name):
    """FP32 solve factors rounded from the FP64 QR factors: M_ASM r within
    10 eps_32 kappa, and the flexible mixed solve within 1e-6."""
    p = problem(name)
    orc = qr_oracle(name, variant="one_level")
    s = solver(L, p, variant=L.ONE_LEVEL, precision=L.MIXED, local_factor=L.FACTOR_QR)
    assert s.info()["mixed_fallback"] == 0
    r = np.random.default_rng(6).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    assert_close(z, orc.apply(r), 10 * EPS32 * max_local_condition(name))
    s.close()
    ref = qr_oracle(name).solve(p.b, tol=1e-10)
    s = solver(L, p, tol=1e-10, precision=L.MIXED, flexible=1, local_factor=L.FACTOR_QR)
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-6)
    s.close()


@pytest.mark.parametrize("order", ["split", "global"])
def test_qr_block_above_streaming_cap(L, order):
    """Two parts of 13,000 and 2,000 columns: the first has more than 12,544
    local unknowns (local solve with y in global memory).  C_ii^{-1} r is the
    same whichever way C_ii is factored, so the Cholesky oracle checks it."""
    p, orc, kap = _above_cap()
    s = L.Solver(p.indptr, p.indices, p.data, p.part, 2, p.m, p.n, p.tau, variant=L.ONE_LEVEL,
                 tol=1e-10, local_factor=L.FACTOR_QR,
                 solve_order=L.ORDER_SPLIT if order == "split" else L.ORDER_GLOBAL)
    assert s.info()["max_ni"] > 12544
    r = np.random.default_rng(13).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    assert_close(z, orc.apply(r), 10 * EPS * kap)
    ref = orc.solve(p.b, tol=1e-10)
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-8)
    s.close()


def test_qr_option_restrictions(L):
    p = problem("banded")
    with pytest.raises(L.Lsq2lError) as e:
        solver(L, p, local_factor=L.FACTOR_QR, diag_shift_rel=1e-10)
    assert e.value.status == L.EINVAL
    with pytest.raises(L.Lsq2lError) as e:
        solver(L, p, local_factor=7)
    assert e.value.status == L.EINVAL


def test_qr_deterministic(L):
    p = problem("grid")
    out = []
    for _ in range(2):
        s = solver(L, p, local_factor=L.FACTOR_QR)
        x, _, _ = s.solve(_t(p.b))
        out.append(_np(x))
        s.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("name", ["banded_1000", "grid", "wide"])
@pytest.mark.parametrize("variant", ["balanced", "ras", "deflated"])
def test_qr_other_forms(L, name, variant):
    """The balanced, RAS and deflated forms on the QR factors and the
    principal-angle coarse space: z = M r against the oracle's QR route
    (tolerances as for the Cholesky route; C amplifies the coarse error once
    more in the deflated form)."""
    p = problem(name)
    orc = qr_oracle(name, variant=variant)
    var = {"balanced": L.BALANCED, "ras": L.RAS, "deflated": L.DEFLATED}[variant]
    kry = L.GMRES if variant in ("ras", "deflated") else L.PCG
    s = solver(L, p, variant=var, krylov=kry, local_factor=L.FACTOR_QR)
    r = np.random.default_rng(7).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    tol = 10 * EPS * max_local_condition(name)
    if variant != "ras" and orc.E is not None:
        tol = max(tol, _qr_tol(name, orc))
        if variant == "deflated":
            tol *= 10
    assert_close(z, orc.apply(r), tol)
    s.close()


@pytest.mark.parametrize("method", ["lsqr", "gmres"])
def test_qr_krylov_methods(L, method):
    """LSQR (additive) and GMRES(100) (deflated) on the QR route against the
    oracle's QR route with the same method."""
    p = problem("banded_1000")
    variant = "additive" if method == "lsqr" else "deflated"
    ref = qr_oracle("banded_1000", variant=variant).solve(p.b, tol=1e-10, method=method)
    s = solver(L, p, tol=1e-10, local_factor=L.FACTOR_QR,
               variant=L.ADDITIVE if method == "lsqr" else L.DEFLATED,
               krylov=L.LSQR if method == "lsqr" else L.GMRES)
    x, info, st = s.solve(_t(p.b))
    assert st == L.OK
    if method == "lsqr":
        assert info[0]["relres_rec"] <= 1e-10
        assert_close(_np(x), ref["x"], 1e-7)
    else:
        assert info[0]["relres"] <= 1e-10
        assert_close(_np(x), ref["x"], 1e-8)
    s.close()


def test_qr_batched(L):
    """Five instances in one handle on the QR route: per-instance solutions
    and selection counts against the oracle's QR route."""
    from workloads import generators as W
    probs = [W.random_banded(300 + 70 * k, 600 + 140 * k, 3 + k, seed=40 + k, name=f"qb{k}")
             for k in range(5)]
    s = L.Solver.batched([(q.indptr, q.indices, q.data, q.part, q.nparts, q.m, q.n) for q in probs],
                         0.1, tol=1e-10, local_factor=L.FACTOR_QR)
    x, infos, _ = s.solve(_t(np.concatenate([q.b for q in probs])))
    x = _np(x)
    off = sub = 0
    for k, q in enumerate(probs):
        orc = O.Oracle(q.scipy(), q.part, q.nparts, 0.1, local_factor="qr").setup()
        ref = orc.solve(q.b, tol=1e-10)
        assert infos[k]["relres"] <= 1e-10
        assert_close(x[off:off + q.n], ref["x"], 1e-8)
        for i in range(q.nparts):
            assert s.subdomain(sub + i)["p"] == orc.p[i]
        off += q.n
        sub += q.nparts
    s.close()
