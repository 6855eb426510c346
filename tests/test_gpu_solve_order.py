"""Local solves with factors in the global-column order of each subdomain.

C_ii^{-1} r does not depend on the order of Omega_i.  The library may factor
C_ii a second time for the per-iteration solves, in the order of the columns
of A, which avoids the dense interface rows that the coarse selection's
order [Omega_Ii, Omega_Gamma_i] creates; in mixed precision that factor is
computed in FP32.  Checked here against the oracle:
  * z = M r entry by entry with either order forced (FP64);
  * the mixed-precision z within the FP32 rounding of a backward-stable local
    solve, and the mixed solve within 1e-6, in every order;
  * the automatic choice on a banded problem (global order, fewer tiles);
  * a subdomain above the streaming kernel's 12,544 local unknowns (y in
    global memory), both orders, both precisions.
"""
import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import (L, _np, _t, assert_close, max_local_condition,  # noqa: F401
                                   max_span_tolerance, oracle, problem, solver)
from workloads import generators as W

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
EPS32 = float(np.finfo(np.float32).eps)
NAMES = ["banded", "grid", "irregular", "parts32", "wide"]


def _order(L, name):
    return {"split": L.ORDER_SPLIT, "global": L.ORDER_GLOBAL, "auto": L.ORDER_AUTO}[name]


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("order", ["split", "global"])
@pytest.mark.parametrize("variant", ["one_level", "additive"])
def test_preconditioner_both_orders(L, name, order, variant):
    p = problem(name)
    orc = oracle(name, variant=variant)
    s = solver(L, p, variant=L.ADDITIVE if variant == "additive" else L.ONE_LEVEL,
               solve_order=_order(L, order))
    inf = s.info()
    assert inf["solve_permuted"] == (p.nparts if order == "global" else 0)
    r = np.random.default_rng(11).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    tol = 10 * EPS * max_local_condition(name)
    if variant == "additive" and orc.E is not None:
        tol = max(tol, 1e-13 * np.linalg.cond(orc.E), max_span_tolerance(name))
    assert_close(z, orc.apply(r), tol)
    s.close()


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("order", ["split", "global", "auto"])
def test_mixed_float_factors(L, name, order):
    """FP32 solve factors: M_ASM r within 10 eps_32 kappa of the oracle (unless
    the float factorization broke down and the double one was rounded,
    which the setup reports), and the flexible mixed solve within 1e-6."""
    p = problem(name)
    orc = oracle(name, variant="one_level")
    s = solver(L, p, variant=L.ONE_LEVEL, precision=L.MIXED, solve_order=_order(L, order))
    inf = s.info()
    if order != "auto":
        assert inf["solve_permuted"] == (p.nparts if order == "global" else 0)
    # the float factorization holds wherever FP32 resolves C_ii comfortably
    if max_local_condition(name) < 1e5:
        assert inf["mixed_fallback"] == 0
    assert inf["mixed_fallback"] in (0, 1)
    assert inf["factor_bytes"] == inf["factor_tiles"] * 1024 * 4
    r = np.random.default_rng(12).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    assert_close(z, orc.apply(r), 10 * EPS32 * max_local_condition(name))
    s.close()
    ref = oracle(name).solve(p.b, tol=1e-10)
    s = solver(L, p, tol=1e-10, precision=L.MIXED, flexible=1, solve_order=_order(L, order))
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-6)
    s.close()


def test_auto_order_on_banded_rows(L):
    """Banded columns: the global order avoids the dense interface rows of
    every subdomain with an interface on its left, so the automatic choice
    takes it there (all but the first subdomain, whose interface already
    comes last) and stores fewer tiles."""
    p = W.random_banded(6000, 12000, 6, seed=41, half_width=20, name="banded_auto")
    s = L.Solver(p.indptr, p.indices, p.data, p.part, p.nparts, p.m, p.n, p.tau)
    inf = s.info()
    assert inf["solve_permuted"] == p.nparts - 1
    assert inf["factor_tiles"] < 0.85 * inf["split_tiles"]
    orc = O.Oracle(p.scipy(), p.part, p.nparts, p.tau).setup()
    ref = orc.solve(p.b, tol=1e-10)
    s.close()
    s = L.Solver(p.indptr, p.indices, p.data, p.part, p.nparts, p.m, p.n, p.tau, tol=1e-10)
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-8)
    s.close()


_big = {}


def _above_cap():
    """Two parts of 13,000 and 2,000 columns: the first has more than 12,544
    local unknowns in either order."""
    if "p" not in _big:
        p = W.random_banded(15000, 30000, 2, seed=93, tau=0.1, half_width=20, name="above_cap")
        p.part = np.concatenate([np.zeros(13000, np.int32), np.ones(2000, np.int32)])
        orc = O.Oracle(p.scipy(), p.part, 2, p.tau, variant="one_level").setup()
        A = p.scipy()
        kap = 1.0
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        for st in orc.sets:
            Ac = A[:, st.Omega]
            C = (Ac.T @ Ac).tocsc()
            d = 1.0 / np.sqrt(C.diagonal())
            Cs = sp.diags(d) @ C @ sp.diags(d)
            hi = spla.eigsh(Cs, k=1, which="LA", return_eigenvectors=False)[0]
            lo = spla.eigsh(Cs, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
            kap = max(kap, hi / lo)
        _big["p"] = (p, orc, kap)
    return _big["p"]


@pytest.mark.parametrize("order", ["split", "global"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_block_above_streaming_cap(L, order, precision):
    p, orc, kap = _above_cap()
    prec = L.FP64 if precision == "fp64" else L.MIXED
    s = L.Solver(p.indptr, p.indices, p.data, p.part, 2, p.m, p.n, p.tau, variant=L.ONE_LEVEL,
                 precision=prec, tol=1e-10, solve_order=_order(L, order))
    assert s.info()["max_ni"] > 12544
    r = np.random.default_rng(13).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    u = EPS if precision == "fp64" else EPS32
    assert_close(z, orc.apply(r), 10 * u * kap)
    ref = orc.solve(p.b, tol=1e-10)
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-8 if precision == "fp64" else 1e-6)
    s.close()
