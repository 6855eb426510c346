"""Parity on a problem whose rows start at unrelated columns (clustered random
rows, 65,536 rows, 16 BFS parts).  On such inputs the library forms
C p = A^T (A p) with a copy of A whose rows are sorted by their first column;
C, and so every result, is the same as with A's own row order.  Solve and
adjoint against the oracle, for every preconditioner form that applies C
inside (the additive and balanced two-level forms, the one-level form) and
with the PCG iteration replayed from a captured graph; the true residual of
every returned x is recomputed on the host with A's own row order."""
import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import L, _np, _t, assert_close, solver  # noqa: F401
from workloads import generators as W

pytestmark = pytest.mark.gpu

_cache = {}


def _problem(variant="one_level"):
    if "p" not in _cache:
        p = W.irregular_clustered(16384, 49152, 16, seed=21, tau=0.05, tol=1e-8, name="irregular_16k")
        A = p.scipy()
        # the row order the library reorders: many far drops of the first column
        key = np.where(np.diff(A.indptr) > 0, A.indices[np.minimum(A.indptr[:-1], A.nnz - 1)], p.n)
        assert p.m >= 65536 and 16 * int((key[1:] < key[:-1] - 256).sum()) > p.m
        _cache["p"] = p
    p = _cache["p"]
    if variant not in _cache:
        _cache[variant] = O.Oracle(p.scipy(), p.part, p.nparts, p.tau, variant=variant).setup()
    return p, _cache[variant]


def _host_residual(p, x):
    A = p.scipy()
    rhs = A.T @ p.b
    return np.linalg.norm(rhs - A.T @ (A @ x)) / np.linalg.norm(rhs)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_parity_row_permuted_products(L, precision):
    p, orc = _problem()
    ref = orc.solve(p.b, tol=1e-10)
    prec = L.FP64 if precision == "fp64" else L.MIXED
    s = solver(L, p, tol=1e-10, variant=L.ONE_LEVEL, precision=prec)
    x, info, _ = s.solve(_t(p.b))
    x = _np(x)
    assert info[0]["relres"] <= 1e-10
    assert_close(x, ref["x"], 1e-8 if precision == "fp64" else 1e-6)
    if precision == "fp64":
        assert abs(info[0]["iterations"] - ref["its"]) <= 1
    assert _host_residual(p, x) <= 1.5e-10
    s.close()


@pytest.mark.parametrize("variant", ["additive", "balanced"])
@pytest.mark.parametrize("use_graph", [0, 1])
def test_two_level_forms_row_permuted_products(L, variant, use_graph):
    """The two-level forms (balanced applies C = A^T A twice inside M) with the
    row-permuted copy, eager and graph-replayed: x against the oracle and the
    true residual in A's own row order."""
    p, orc = _problem(variant)
    ref = orc.solve(p.b, tol=1e-10, flexible=(variant == "balanced"))
    var = L.ADDITIVE if variant == "additive" else L.BALANCED
    s = solver(L, p, tol=1e-10, variant=var, use_graph=use_graph,
               flexible=int(variant == "balanced"))
    x, info, _ = s.solve(_t(p.b))
    x = _np(x)
    assert info[0]["relres"] <= 1e-10
    assert_close(x, ref["x"], 1e-8)
    assert _host_residual(p, x) <= 1.5e-10
    s.close()


def test_backward_parity_row_permuted_products(L):
    """dL/db in A's own row order and dL/dvals in A's CSR order, for
    L = 1/2 ||x - x*||^2, within the 1e-5 gradient tolerance; the adjoint
    returns OK on its backward-error rule."""
    p, orc = _problem()
    xstar = np.random.default_rng(7).standard_normal(p.n)
    xo = orc.solve(p.b, tol=1e-11)["x"]
    go = orc.backward(p.b, xo, xo - xstar, tol=1e-11)
    s = solver(L, p, tol=1e-11, variant=L.ONE_LEVEL)
    x, _, _ = s.solve(_t(p.b))
    dLdb, dLdv, info = s.backward(x - _t(xstar))
    assert info[0]["relres"] <= 1e-11 or info[0]["backward_err"] <= 1e-11
    assert_close(_np(dLdb), go["dLdb"], 1e-5)
    assert_close(_np(dLdv), go["dLdvals"], 1e-5)
    s.close()
