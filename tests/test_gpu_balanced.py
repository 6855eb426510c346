"""GPU parity of the balanced two-level preconditioner (eq. balanced) with
M_ASM as first level: M = Q + (I - C Q)^T M_ASM (I - C Q), Q = R_0^T E^{-1} R_0.

Through the C ABI (variant LSQ2L_BALANCED) against the oracle's balanced
form, on the same seeded inputs as the other parity tests."""
import math

import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import (EPS, L, _np, _t, assert_close, max_local_condition,  # noqa: F401
                                   max_span_tolerance, oracle, problem, solver)

pytestmark = pytest.mark.gpu

NAMES = ["banded_1000", "banded", "grid", "irregular", "parts32", "wide"]


_consts = {}


def _constants(name):
    """k_c (greedy colouring of the subdomain graph) and kappa(M C) of the
    oracle's balanced preconditioner, from the dense M (n <= 2000)."""
    if name not in _consts:
        p = problem(name)
        A = p.scipy()
        orc = oracle(name, variant="balanced")
        _, kc = O.greedy_colouring(A, orc.sets)
        Lc = np.linalg.cholesky((A.T @ A).toarray())
        ev = np.linalg.eigvalsh(Lc.T @ O.dense_preconditioner(orc) @ Lc)
        _consts[name] = (kc, ev.max() / ev.min())
    return _consts[name]


def _cnorm(A, v):
    return float(np.linalg.norm(A @ v))


@pytest.mark.parametrize("name", NAMES)
def test_balanced_preconditioner_parity(L, name):
    """z = M r against the oracle.

    The local and coarse parts carry the same rounding and coarse-space
    differences as the additive form (relative size t).  In the C inner
    product P = Q C is the orthogonal projector onto the coarse space and
    ||M_ASM C||_C <= k_c + 1, so M C = P + (I - P) M_ASM C (I - P) moves by at
    most t (3 + 2 k_c) when P and M_ASM do by t; z = (M C)(C^{-1} r) then
    moves by at most that times kappa(M C), relative to ||z||_C.  Without a
    coarse space M = M_ASM and the additive bound t applies as it stands."""
    p = problem(name)
    A = p.scipy()
    orc = oracle(name, variant="balanced")
    s = solver(L, p, variant=L.BALANCED)
    assert s.info()["n0"] == orc.n0
    r = np.random.default_rng(3).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    zr = orc.apply(r)
    tol = 10 * EPS * max_local_condition(name)
    if orc.E is None:
        err = np.linalg.norm(z - zr) / np.linalg.norm(zr)
    else:
        kc, kap = _constants(name)
        tol = max(tol, 1e-13 * np.linalg.cond(orc.E), max_span_tolerance(name))
        tol *= (3 + 2 * kc) * kap
        err = _cnorm(A, z - zr) / _cnorm(A, zr)
    print(f"{name}: n0 {orc.n0} relative error {err:.3e} bound {tol:.3e}")
    assert err <= tol, f"relative error {err:.3e} > {tol:.3e}"
    s.close()


@pytest.mark.parametrize("name", ["banded_1000", "grid", "parts32", "wide"])
def test_balanced_coarse_space_is_unit_eigenspace(L, name):
    """With the library's own coarse basis X_i: M C v = v for every coarse
    vector v = R_0^T e_k (E = R_0 C R_0^T makes Q C the C-orthogonal projector
    onto the coarse space).  The computed E differs from R_0 C R_0^T by
    rounding, so Q C v = v + d with ||d||_C / ||v||_C of order eps kappa(E);
    d passes through (I - P) M_ASM C (I - P) and P, which in the C norm are
    bounded by k_c + 1 and 1: the error bound is 100 eps kappa(E) (3 + 2 k_c)."""
    p = problem(name)
    orc = oracle(name, variant="balanced")
    if orc.n0 == 0:
        pytest.skip("no coarse space")
    A = p.scipy()
    s = solver(L, p, variant=L.BALANCED)
    kc, _ = _constants(name)
    tol = 100 * EPS * np.linalg.cond(orc.E) * (3 + 2 * kc)
    worst = 0.0
    for i, st in enumerate(orc.sets):
        Xg = s.coarse_basis(i)
        for k in range(min(Xg.shape[1], 2)):
            v = np.zeros(p.n)
            v[st.I] = Xg[:, k]
            z = _np(s.apply_preconditioner(_t(A.T @ (A @ v))))
            worst = max(worst, _cnorm(A, z - v) / _cnorm(A, v))
    print(f"{name}: worst {worst:.3e} bound {tol:.3e}")
    assert worst <= tol
    s.close()


@pytest.mark.parametrize("name", NAMES)
def test_balanced_solve_parity(L, name):
    """FP64: x within 1e-8 of the oracle's balanced PCG at tol 1e-10, and the
    iteration count within 3%.  MIXED (flexible): x within 1e-6."""
    p = problem(name)
    orc = oracle(name, variant="balanced")
    ref = orc.solve(p.b, tol=1e-10)
    s = solver(L, p, tol=1e-10, variant=L.BALANCED)
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-8)
    assert abs(info[0]["iterations"] - ref["its"]) <= max(1, math.ceil(0.03 * ref["its"]))
    s.close()
    s = solver(L, p, tol=1e-10, variant=L.BALANCED, precision=L.MIXED, flexible=1)
    x, info, _ = s.solve(_t(p.b))
    assert info[0]["relres"] <= 1e-10
    assert_close(_np(x), ref["x"], 1e-6)
    s.close()


def test_balanced_in_place_and_graph_replay(L):
    """z = M r with z aliasing r gives the same bits; a solve with the PCG
    iteration captured as a HIP graph gives the eager solve's bits."""
    p = problem("banded_1000")
    s = solver(L, p, variant=L.BALANCED)
    r = np.random.default_rng(4).standard_normal(p.n)
    z = _np(s.apply_preconditioner(_t(r)))
    rt = _t(r)
    s.apply_preconditioner(rt, out=rt)
    assert np.array_equal(_np(rt), z)
    x0, i0, _ = s.solve(_t(p.b))
    s.close()
    s = solver(L, p, variant=L.BALANCED, use_graph=1)
    for _ in range(2):
        x1, i1, _ = s.solve(_t(p.b))
        assert np.array_equal(_np(x1), _np(x0))
        assert i1[0]["iterations"] == i0[0]["iterations"]
    s.close()
