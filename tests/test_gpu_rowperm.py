"""Parity on a problem whose rows start at unrelated columns (clustered random
rows, 65,536 rows, 16 BFS parts).  On such inputs the library forms
C p = A^T (A p) with a copy of A whose rows are sorted by their first column;
C, and so every result, is the same as with A's own row order.  Solve and
adjoint against the oracle's one-level preconditioned solve (eq.
one_level_schwarz), whose setup stays cheap at this size."""
import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import L, _np, _t, solver  # noqa: F401
from workloads import generators as W

pytestmark = pytest.mark.gpu

_cache = {}


def _problem():
    if "p" not in _cache:
        p = W.irregular_clustered(16384, 49152, 16, seed=21, tau=0.05, tol=1e-8, name="irregular_16k")
        A = p.scipy()
        # the row order the library reorders: many descents of the first column
        key = np.where(np.diff(A.indptr) > 0, A.indices[np.minimum(A.indptr[:-1], A.nnz - 1)], p.n)
        assert p.m >= 65536 and 16 * int((key[1:] < key[:-1]).sum()) > p.m
        orc = O.Oracle(A, p.part, p.nparts, p.tau, variant="one_level").setup()
        _cache["p"] = (p, orc)
    return _cache["p"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_parity_row_permuted_products(L, precision):
    p, orc = _problem()
    ref = orc.solve(p.b, tol=1e-10)
    prec = L.FP64 if precision == "fp64" else L.MIXED
    s = solver(L, p, tol=1e-10, variant=L.ONE_LEVEL, precision=prec)
    x, info, _ = s.solve(_t(p.b))
    x = _np(x)
    assert info[0]["relres"] <= 1e-10
    tol = 1e-8 if precision == "fp64" else 1e-6
    assert np.linalg.norm(x - ref["x"]) <= tol * np.linalg.norm(ref["x"])
    if precision == "fp64":
        assert abs(info[0]["iterations"] - ref["its"]) <= 1
    # the true residual of the returned x, on the host
    A = p.scipy()
    rhs = A.T @ p.b
    assert np.linalg.norm(rhs - A.T @ (A @ x)) <= 1e-10 * np.linalg.norm(rhs) * 1.5
    s.close()


def test_backward_parity_row_permuted_products(L):
    """dL/db in A's own row order and dL/dvals in A's CSR order, for
    L = 1/2 ||x - x*||^2, within the 1e-5 gradient tolerance."""
    p, orc = _problem()
    xstar = np.random.default_rng(7).standard_normal(p.n)
    xo = orc.solve(p.b, tol=1e-11)["x"]
    go = orc.backward(p.b, xo, xo - xstar, tol=1e-11)
    s = solver(L, p, tol=1e-11, variant=L.ONE_LEVEL)
    x, _, _ = s.solve(_t(p.b))
    dLdb, dLdv, _ = s.backward(x - _t(xstar))
    assert np.linalg.norm(_np(dLdb) - go["dLdb"]) <= 1e-5 * np.linalg.norm(go["dLdb"])
    assert np.linalg.norm(_np(dLdv) - go["dLdvals"]) <= 1e-5 * np.linalg.norm(go["dLdvals"])
    s.close()
