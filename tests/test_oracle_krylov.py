"""CPU pins of the oracle's Krylov methods, preconditioner variants and
options beyond the additive two-level CG: left-preconditioned LSQR and
right-preconditioned restarted GMRES (Section 4.1, "Solution phase";
Section 4.2), the restricted additive and deflated forms (eqs. RAS,
deflated), the global diagonal shift of Section 4.1 ("Setup phase"), the cap
on coarse vectors, and the colouring constant of the worked example.

Each pin compares against something other than the oracle itself: a
library routine on an equivalent problem, a closed form, brute force over
an explicit basis, or an identity the paper's definitions imply.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from workloads import generators as W


def _small(n=60, m=150, parts=4, seed=5, **kw):
    return W.random_banded(n, m, parts, seed=seed, half_width=6, **kw)


# ---------------------------------------------------------------------------
# LSQR
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 5, 12, 30])
def test_lsqr_identity_preconditioner_matches_library_lsqr(k):
    """With M = I the oracle's LSQR is Paige and Saunders' LSQR: its k-th
    iterate equals scipy's after k iterations."""
    p = _small()
    A = p.scipy()
    x = O.lsqr(A, p.b, lambda v: v.copy(), tol=0.0, maxit=k)["x"]
    ref = spla.lsqr(A, p.b, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("k", [1, 3, 6, 10])
def test_lsqr_preconditioned_is_lsqr_on_transformed_operator(k):
    """For M = W^{-1} W^{-T}, the k-th iterate is W^{-1} y_k with y_k the
    library LSQR iterate on A W^{-1} (the paper's left preconditioning)."""
    p = _small(seed=9)
    A = p.scipy()
    rng = np.random.default_rng(3)
    n = p.n
    Wm = np.triu(rng.standard_normal((n, n)) * 0.1) + np.diag(1.0 + rng.uniform(size=n))
    Wi = sla.solve_triangular(Wm, np.eye(n))
    Mm = Wi @ Wi.T
    x = O.lsqr(A, p.b, lambda v: Mm @ v, tol=0.0, maxit=k)["x"]
    y = spla.lsqr(A.toarray() @ Wi, p.b, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
    ref = Wi @ y
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_lsqr_exact_preconditioner_converges_in_one_step():
    """M = C^{-1} = W^{-1} W^{-T} with C = W^T W: A W^{-1} has orthonormal
    columns, so one LSQR step gives the least-squares solution."""
    p = _small(seed=2)
    A = p.scipy()
    C = (A.T @ A).toarray()
    Ci = np.linalg.inv(C)
    res = O.lsqr(A, p.b, lambda v: Ci @ v, tol=1e-12, maxit=50)
    xs = np.linalg.lstsq(A.toarray(), p.b, rcond=None)[0]
    assert res["its"] == 1
    assert np.linalg.norm(res["x"] - xs) <= 1e-10 * np.linalg.norm(xs)


@pytest.mark.parametrize("variant", ["additive", "balanced", "one_level"])
def test_lsqr_with_schwarz_preconditioner_reaches_least_squares(variant):
    """Preconditioned LSQR stops on its normal-equation test and the result
    is the least-squares solution within the conditioning of the test."""
    p = W.banded_1000()
    A = p.scipy()
    orc = O.Oracle(A, p.part, p.nparts, p.tau, variant=variant).setup()
    res = orc.solve(p.b, tol=1e-12, method="lsqr")
    assert res["test"] <= 1e-12
    xs = np.linalg.lstsq(A.toarray(), p.b, rcond=None)[0]
    assert np.linalg.norm(res["x"] - xs) <= 1e-8 * np.linalg.norm(xs)
    # the test quantity is LSQR's estimate of ||(A W^-1)^T r|| / (||A W^-1||_F ||r||);
    # at the solution the true normal residual is small too
    r = p.b - A @ res["x"]
    assert np.linalg.norm(A.T @ r) <= 1e-9 * np.linalg.norm(A.T @ p.b)


# ---------------------------------------------------------------------------
# GMRES
# ---------------------------------------------------------------------------

def _tiny_gmres_problem():
    p = W.random_banded(30, 70, 3, seed=11, half_width=4)
    A = p.scipy()
    orc = O.Oracle(A, p.part, p.nparts, 0.3, variant="ras").setup()
    return p, A, orc


@pytest.mark.parametrize("k", [1, 2, 4, 7, 10])
def test_gmres_iterate_minimizes_residual_over_krylov_space(k):
    """After k steps of the first cycle, ||rhs - C x_k|| is the minimum over
    x in M K_k(C M, rhs): brute force over an explicit Krylov basis."""
    p, A, orc = _tiny_gmres_problem()
    C = (A.T @ A).toarray()
    rhs = A.T @ p.b
    M = orc.apply
    x = O.gmres(A, rhs, M, tol=0.0, maxit=k, restart=50)["x"]
    K = [rhs]
    for _ in range(k - 1):
        K.append(C @ M(K[-1]))
    Q = sla.orth(np.column_stack(K))
    CMQ = np.column_stack([C @ M(Q[:, j]) for j in range(Q.shape[1])])
    y = np.linalg.lstsq(CMQ, rhs, rcond=None)[0]
    best = np.linalg.norm(rhs - CMQ @ y)
    got = np.linalg.norm(rhs - C @ x)
    assert abs(got - best) <= 1e-8 * np.linalg.norm(rhs)


def test_gmres_restart_one_is_minimal_residual_steepest_descent():
    """GMRES(1): each cycle takes x += a M r with the closed-form step
    a = (r^T C M r) / ||C M r||^2."""
    p, A, orc = _tiny_gmres_problem()
    C = (A.T @ A).toarray()
    rhs = A.T @ p.b
    M = orc.apply
    x = np.zeros(p.n)
    for _ in range(5):
        r = rhs - C @ x
        v = C @ M(r)
        x = x + (r @ v) / (v @ v) * M(r)
    got = O.gmres(A, rhs, M, tol=0.0, maxit=5, restart=1)["x"]
    assert np.linalg.norm(got - x) <= 1e-10 * np.linalg.norm(x)


def test_gmres_full_space_reaches_least_squares():
    """Without restarts GMRES on the n x n system ends within n steps at the
    solution of the normal equations (dense least squares)."""
    p, A, orc = _tiny_gmres_problem()
    res = O.gmres(A, A.T @ p.b, orc.apply, tol=1e-12, maxit=200, restart=200)
    xs = np.linalg.lstsq(A.toarray(), p.b, rcond=None)[0]
    assert res["its"] <= p.n
    assert np.linalg.norm(res["x"] - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("variant", ["ras", "deflated", "additive"])
def test_gmres_with_schwarz_preconditioners_reaches_least_squares(variant):
    p = W.banded_1000()
    A = p.scipy()
    orc = O.Oracle(A, p.part, p.nparts, p.tau, variant=variant).setup()
    res = orc.solve(p.b, tol=1e-12, method="gmres")
    assert res["relres"] <= 1e-12
    xs = np.linalg.lstsq(A.toarray(), p.b, rcond=None)[0]
    assert np.linalg.norm(res["x"] - xs) <= 1e-8 * np.linalg.norm(xs)


# ---------------------------------------------------------------------------
# RAS and the deflated form
# ---------------------------------------------------------------------------

def test_ras_partition_of_unity_restores_identity():
    """sum_i R_i^T D_i R_i = I: every column is interior to exactly one subdomain."""
    p = _small(parts=5, seed=4)
    A = p.scipy()
    sets = O.index_sets(A, p.part, p.nparts)
    S = sum((O.restriction(s, p.n).T @ sp.diags(O.partition_of_unity(s)) @ O.restriction(s, p.n))
            for s in sets)
    assert np.array_equal(S.toarray(), np.eye(p.n))


def test_ras_single_subdomain_is_exact_inverse():
    p = W.random_banded(40, 90, 1, seed=6, half_width=5)
    A = p.scipy()
    orc = O.Oracle(A, p.part, 1, 0.1, variant="ras").setup()
    C = (A.T @ A).toarray()
    r = np.random.default_rng(1).standard_normal(p.n)
    z = orc.apply(r)
    assert np.linalg.norm(z - np.linalg.solve(C, r)) <= 1e-10 * np.linalg.norm(z)


def test_ras_equals_asm_without_overlap():
    """With decoupled column blocks (A block diagonal) there is no interface:
    D_i = I on every subdomain, M_RAS = M_ASM = C^{-1}."""
    blocks = [W.random_banded(20, 45, 1, seed=20 + k, half_width=3).scipy() for k in range(3)]
    A = sp.block_diag(blocks, format="csr")
    part = np.repeat(np.arange(3), 20).astype(np.int32)
    ras = O.Oracle(A, part, 3, 0.1, variant="ras").setup()
    asm = O.Oracle(A, part, 3, 0.1, variant="one_level").setup()
    r = np.random.default_rng(2).standard_normal(60)
    C = (A.T @ A).toarray()
    assert all(s.nG == 0 for s in ras.sets)
    assert np.linalg.norm(ras.apply(r) - asm.apply(r)) <= 1e-12 * np.linalg.norm(asm.apply(r))
    assert np.linalg.norm(ras.apply(r) - np.linalg.solve(C, r)) <= 1e-10 * np.linalg.norm(r)


def test_ras_differs_from_asm_with_overlap():
    p = _small(parts=4, seed=8)
    A = p.scipy()
    ras = O.Oracle(A, p.part, p.nparts, 0.1, variant="ras").setup()
    asm = O.Oracle(A, p.part, p.nparts, 0.1, variant="one_level").setup()
    r = np.random.default_rng(4).standard_normal(p.n)
    zr, za = ras.apply(r), asm.apply(r)
    assert np.linalg.norm(zr - za) > 1e-3 * np.linalg.norm(za)
    # on each interior, RAS keeps exactly the owner's local solution
    for s, F in zip(ras.sets, ras.chol):
        zi = sla.cho_solve(F, r[s.Omega])
        assert np.allclose(zr[s.I], zi[:s.nI], rtol=1e-12, atol=1e-14)


def test_deflated_coarse_space_is_unit_eigenspace():
    """M_deflated C R_0^T = R_0^T: Q C R_0^T = R_0^T and (I - C Q) C R_0^T = 0."""
    p = W.banded_1000()
    A = p.scipy()
    orc = O.Oracle(A, p.part, p.nparts, 0.4, variant="deflated").setup()
    assert orc.n0 > 0
    R0T = orc.R0T.toarray()
    for j in range(R0T.shape[1]):
        v = R0T[:, j]
        got = orc.apply(A.T @ (A @ v))
        assert np.linalg.norm(got - v) <= 1e-8 * np.linalg.norm(v)


def test_deflated_without_coarse_space_is_ras():
    p = W.banded_1000()
    A = p.scipy()
    d = O.Oracle(A, p.part, p.nparts, 1e-12, variant="deflated").setup()
    r = O.Oracle(A, p.part, p.nparts, 1e-12, variant="ras").setup()
    assert d.n0 == 0
    v = np.random.default_rng(7).standard_normal(p.n)
    assert np.array_equal(d.apply(v), r.apply(v))


# ---------------------------------------------------------------------------
# diagonal shift (Section 4.1, "Setup phase")
# ---------------------------------------------------------------------------

def test_frobenius_of_normal_matrix_against_dense():
    p = _small(seed=12)
    A = p.scipy()
    C = A.toarray().T @ A.toarray()
    assert abs(O.frobenius_normal(A) - np.linalg.norm(C, "fro")) <= 1e-12 * np.linalg.norm(C, "fro")


def test_shift_single_subdomain_is_shifted_inverse():
    """N = 1: M = (C + s I)^{-1}, s = diag_shift_rel ||C||_F."""
    p = W.random_banded(40, 90, 1, seed=6, half_width=5)
    A = p.scipy()
    rel = 1e-3
    orc = O.Oracle(A, p.part, 1, 0.1, variant="one_level", diag_shift_rel=rel).setup()
    C = (A.T @ A).toarray()
    s = rel * np.linalg.norm(C, "fro")
    assert abs(orc.shift - s) <= 1e-12 * s
    r = np.random.default_rng(1).standard_normal(p.n)
    ref = np.linalg.solve(C + s * np.eye(p.n), r)
    assert np.linalg.norm(orc.apply(r) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_shift_keeps_theorem26_bound_for_shifted_matrix():
    """The shifted preconditioner is the two-level preconditioner of
    [A; sqrt(s) I], so Theorem 2.6 bounds kappa(M (C + s I)) with the
    constants of that matrix (each added row lies in one Xi_i: k_m unchanged)."""
    p = _small(n=80, m=200, parts=6, seed=3)
    A = p.scipy()
    orc = O.Oracle(A, p.part, p.nparts, 0.2, diag_shift_rel=1e-2).setup()
    Ab = orc.Ab
    C = (Ab.T @ Ab).toarray()
    Mm = O.dense_preconditioner(orc)
    ev = np.sort(np.real(sla.eigvals(Mm @ C)))
    _, kc = O.greedy_colouring(Ab, orc.sets)
    _, km = O.multiplicity(Ab, orc.sets)
    _, km0 = O.multiplicity(A, O.index_sets(A, p.part, p.nparts))
    assert km == km0
    assert ev[-1] / ev[0] <= O.theorem26_bound(kc, km, 0.2) * (1 + 1e-10)


def test_shift_zero_is_unshifted():
    p = W.banded_1000()
    A = p.scipy()
    a = O.Oracle(A, p.part, p.nparts, p.tau).setup()
    b = O.Oracle(A, p.part, p.nparts, p.tau, diag_shift_rel=0.0).setup()
    r = np.random.default_rng(0).standard_normal(p.n)
    assert np.array_equal(a.apply(r), b.apply(r))


# ---------------------------------------------------------------------------
# nev_max and the colouring constant
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cap", [1, 2, 3])
def test_nev_max_keeps_the_smallest_schur_eigenvalues(cap):
    """coarse_vectors with nev_max keeps the directions of the nev_max
    smallest mu of the Schur pencil S x = mu C_I x (route (i), a library
    generalized eigensolver): principal angles against those eigenvectors."""
    p = W.banded_1000()
    A = p.scipy()
    sets = O.index_sets(A, p.part, p.nparts)
    for st in sets[:4]:
        Cii, Ctii = O.local_matrices(A, st)
        nI = st.nI
        CI = Cii[:nI, :nI]
        CIG = Ctii[:nI, nI:]
        S = CI - CIG @ sla.pinvh(Ctii[nI:, nI:]) @ CIG.T
        mu, V = sla.eigh(0.5 * (S + S.T), CI)
        res = O.coarse_vectors(Cii, Ctii, nI, 0.6, nev_max=cap)
        k = min(cap, int((mu < 0.6).sum()))
        assert res["p"] == k
        if k:
            ang = sla.subspace_angles(res["X"], V[:, :k])
            assert ang.max() <= 1e-7
            assert np.allclose(res["X"].T @ CI @ res["X"], np.eye(k), atol=1e-10)


def test_worked_example_colouring_constant():
    """The two subdomains of the worked example share a row, so k_c = 2."""
    p = W.worked_example()
    A = p.scipy()
    sets = O.index_sets(A, p.part, p.nparts)
    colour, kc = O.greedy_colouring(A, sets)
    assert kc == 2 and colour[0] != colour[1]


# ---------------------------------------------------------------------------
# direct reference solves for full-size checks
# ---------------------------------------------------------------------------

def test_direct_normal_solve_matches_dense_least_squares():
    """Within the forward error eps kappa(C) = eps kappa(A)^2 of a backward
    stable solve of the normal equations (the grid's kappa(A) is 1.6e5)."""
    p = W.small_config("grid")
    A = p.scipy()
    x = O.normal_solve_direct(A, A.T @ p.b)
    xs = np.linalg.lstsq(A.toarray(), p.b, rcond=None)[0]
    kappa = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - xs) <= 10 * np.finfo(float).eps * kappa ** 2 * np.linalg.norm(xs)


def test_gradient_formula_matches_oracle_adjoint_and_differences():
    """gradients() with the direct adjoint equals the oracle's PCG adjoint,
    and central differences of L = 1/2 ||x - x*||^2 in b."""
    p = W.banded_1000()
    A = p.scipy()
    xstar = np.random.default_rng(5).standard_normal(p.n)
    x = O.normal_solve_direct(A, A.T @ p.b)
    lam = O.normal_solve_direct(A, x - xstar)
    g = O.gradients(A, p.b, x, lam)
    orc = O.Oracle(A, p.part, p.nparts, p.tau).setup()
    go = orc.backward(p.b, x, x - xstar, tol=1e-13)
    assert np.linalg.norm(g["dLdb"] - go["dLdb"]) <= 1e-9 * np.linalg.norm(go["dLdb"])
    assert np.linalg.norm(g["dLdvals"] - go["dLdvals"]) <= 1e-9 * np.linalg.norm(go["dLdvals"])
    h = 1e-6
    for k in (3, 500, 2900):
        bp, bm = p.b.copy(), p.b.copy()
        bp[k] += h
        bm[k] -= h
        lp = 0.5 * np.sum((O.normal_solve_direct(A, A.T @ bp) - xstar) ** 2)
        lm = 0.5 * np.sum((O.normal_solve_direct(A, A.T @ bm) - xstar) ** 2)
        assert abs((lp - lm) / (2 * h) - g["dLdb"][k]) <= 1e-6 * max(1.0, abs(g["dLdb"][k]))
