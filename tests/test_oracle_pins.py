"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks it against
values printed in the paper (the worked example of Section 3), closed forms
derived by hand from that example, library routines (principal angles,
dense least squares), the inequalities of Lemmas 2.2, 2.4, 3.1 and
Theorem 2.6, or central finite differences.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
from workloads import generators as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":")
            out[k.strip()] = np.array([float(t) for t in v.split()])
    return out


# ---------------------------------------------------------------------------
# worked example (Section 3)
# ---------------------------------------------------------------------------

def test_worked_example_index_sets_match_paper():
    g = _golden()
    A_dense = np.stack([g[f"A_row{r}"] for r in range(5)])
    p = W.worked_example()
    A = p.scipy()
    np.testing.assert_array_equal(A.toarray(), A_dense)
    np.testing.assert_array_equal(p.part, g["part"].astype(int))
    sets = O.index_sets(A, p.part, p.nparts)
    for i, s in enumerate(sets):
        np.testing.assert_array_equal(s.Xi, g[f"Xi_{i}"].astype(int))
        np.testing.assert_array_equal(s.G, g[f"Gamma_{i}"].astype(int))
        np.testing.assert_array_equal(s.Omega, g[f"Omega_{i}"].astype(int))
        np.testing.assert_array_equal(O.partition_of_unity(s), g[f"D_{i}"])
        # R_i = I_4(Omega_i, :)
        R = O.restriction(s, 4).toarray()
        np.testing.assert_array_equal(R, np.eye(4)[g[f"Omega_{i}"].astype(int)])
        # the permuted matrix A([Xi, Xi_c], [Omega_I, Omega_Gamma, Omega_c])
        Xc = np.setdiff1d(np.arange(5), s.Xi)
        Oc = g[f"Omega_c_{i}"].astype(int)
        perm = A_dense[np.concatenate([s.Xi, Xc])][:, np.concatenate([s.I, s.G, Oc])]
        np.testing.assert_array_equal(perm, np.stack([g[f"permuted_{i}_row{r}"] for r in range(5)]))


def test_worked_example_partition_of_unity_sums_to_identity():
    p = W.worked_example()
    sets = O.index_sets(p.scipy(), p.part, p.nparts)
    tot = sum((O.restriction(s, 4).T @ sp.diags(O.partition_of_unity(s)) @ O.restriction(s, 4)).toarray()
              for s in sets)
    np.testing.assert_array_equal(tot, np.eye(4))


# Hand-derived closed forms from the printed A (exact integers): with
# Omega_1 = [1,3,2] and Omega_2 = [2,4,1] (1-based), C_ii is the Gram matrix of
# the columns, and Ct_ii the Gram matrix restricted to the rows Xi_i.
C11 = np.array([[14, 6, 8], [6, 36, 0], [8, 0, 41]], dtype=float)
Ct11 = np.array([[14, 6, 8], [6, 36, 0], [8, 0, 16]], dtype=float)
C22 = np.array([[41, 35, 8], [35, 113, 0], [8, 0, 14]], dtype=float)
Ct22 = np.array([[41, 35, 8], [35, 113, 0], [8, 0, 4]], dtype=float)


def test_worked_example_local_matrices_closed_form():
    p = W.worked_example()
    A = p.scipy()
    sets = O.index_sets(A, p.part, p.nparts)
    for s, (C, Ct) in zip(sets, [(C11, Ct11), (C22, Ct22)]):
        Cii, Ctii = O.local_matrices(A, s)
        np.testing.assert_array_equal(Cii, C)
        np.testing.assert_array_equal(Ctii, Ct)


def test_worked_example_eigenvalues_closed_form():
    """eq. (gevp) on the example: lambda in {0, 1, 13/9} and {0, 1, 213/100}.

    Subdomain 1: eliminating Gamma gives C_I - S = diag(4, 0), so
    1 - mu = 4 (C_I^{-1})_11 = 4/13 and lambda = 1/mu = 13/9; subdomain 2:
    C_I - S = diag(16, 0), 1 - mu = 16 * 113 / 3408 = 113/213, lambda = 213/100.
    """
    p = W.worked_example()
    A = p.scipy()
    sets = O.index_sets(A, p.part, p.nparts)
    expected = [np.array([0.0, 1.0, 13 / 9]), np.array([0.0, 1.0, 213 / 100])]
    for s, ev in zip(sets, expected):
        Cii, Ctii = O.local_matrices(A, s)
        res = O.coarse_vectors(Cii, Ctii, s.nI, 0.6)
        np.testing.assert_allclose(np.sort(res["lam"]), ev, atol=1e-13, rtol=1e-13)


@pytest.mark.parametrize("tau,expect", [(0.6, (0, 1)), (0.70, (1, 1)), (0.69, (0, 1)),
                                        (0.47, (0, 1)), (0.46, (0, 0))])
def test_worked_example_selection_thresholds(tau, expect):
    """Subdomain 1 is selected iff tau > 9/13 = 0.6923, subdomain 2 iff tau > 100/213 = 0.4695."""
    p = W.worked_example()
    orc = O.Oracle(p.scipy(), p.part, p.nparts, tau).setup()
    assert tuple(orc.p) == expect


def test_worked_example_coarse_vector_direction():
    """At tau = 0.6 the coarse space is spanned by (0, 113, 0, -35): the interior
    part C_I^{-1} e_1 of subdomain 2 (order [2, 4])."""
    p = W.worked_example()
    orc = O.Oracle(p.scipy(), p.part, p.nparts, 0.6).setup()
    assert orc.n0 == 1
    v = orc.R0T.toarray()[:, 0]
    ref = np.array([0.0, 113.0, 0.0, -35.0])
    cos = abs(v @ ref) / (np.linalg.norm(v) * np.linalg.norm(ref))
    assert cos == pytest.approx(1.0, abs=1e-14)
    # C_I-normalised: x^T C_I x = 1 with C_I = [[41, 35], [35, 113]]
    x = v[[1, 3]]
    assert x @ C22[:2, :2] @ x == pytest.approx(1.0, rel=1e-13)


def test_worked_example_multiplicity():
    p = W.worked_example()
    A = p.scipy()
    sets = O.index_sets(A, p.part, p.nparts)
    mj, km = O.multiplicity(A, sets)
    np.testing.assert_array_equal(mj, [1, 2, 1, 1, 1])
    assert km == 2
    # Section 3: sum_i Ct_i - C is the outer product of row 2 of A
    C = (A.T @ A).toarray()
    St = sum((A[s.Xi, :].T @ A[s.Xi, :]).toarray() for s in sets)
    a2 = np.array([2.0, 4.0, 0.0, 0.0])
    np.testing.assert_array_equal(St - C, np.outer(a2, a2))


# ---------------------------------------------------------------------------
# splitting invariants (Section 2.1, eq. spsd_normal_eq, Lemma 3.1)
# ---------------------------------------------------------------------------

def _small_problems():
    return [W.random_banded(240, 480, 6, seed=11, name="rb"),
            W.small_config("grid"),
            W.random_banded(300, 600, 5, seed=12, k=6, half_width=30, name="rb6")]


@pytest.mark.parametrize("prob", _small_problems(), ids=lambda p: p.name)
def test_local_splitting_invariants(prob):
    A = prob.scipy()
    n = prob.n
    C = (A.T @ A).toarray()
    sets = O.index_sets(A, prob.part, prob.nparts)
    mj, km = O.multiplicity(A, sets)
    tot = np.zeros((n, n))
    scale = np.abs(C).max()
    for s in sets:
        Cii, Ctii = O.local_matrices(A, s)
        R = O.restriction(s, n).toarray()
        Ct_glob = R.T @ Ctii @ R
        # C_ii = R_i C R_i^T (eq. one_level_schwarz)
        np.testing.assert_allclose(Cii, R @ C @ R.T, atol=1e-12 * scale)
        # C = Ct_i + A(Xi_c,:)^T A(Xi_c,:) (proof of Lemma 3.1 / eq. spsd_normal_eq)
        Xc = np.setdiff1d(np.arange(prob.m), s.Xi)
        Ac = A[Xc, :].toarray()
        np.testing.assert_allclose(C - Ct_glob, Ac.T @ Ac, atol=1e-12 * scale)
        # 0 <= u^T Ct_i u <= u^T C u (definition of a local SPSD splitting)
        assert sla.eigvalsh(Ct_glob).min() >= -1e-10 * scale
        assert sla.eigvalsh(C - Ct_glob).min() >= -1e-10 * scale
        # Ct_i vanishes outside Omega_i (the 2x2 block structure)
        out = np.setdiff1d(np.arange(n), s.Omega)
        assert np.all(Ct_glob[out, :] == 0) and np.all(Ct_glob[:, out] == 0)
        tot += Ct_glob
    Ad = A.toarray()
    np.testing.assert_allclose(tot, Ad.T @ (mj[:, None] * Ad), atol=1e-11 * scale)
    # eq. (sum C-tildeC_ge_0) with k_m from Lemma 3.1
    assert sla.eigvalsh(km * C - tot).min() >= -1e-9 * scale
    # Lemma 3.1: k_m <= max_i k_Omega_i
    kOm = [sum(1 for t in sets if np.intersect1d(s.Omega, t.Omega).size) for s in sets]
    assert km <= max(kOm)


def test_multiplicity_one_gives_exact_splitting():
    """If every row touches one interior only (m_j = 1), sum_i Ct_i = C."""
    # block-diagonal A: parts aligned with the blocks, so no row is shared
    blocks = [W.random_banded(40, 80, 1, seed=20 + k).scipy() for k in range(3)]
    A = sp.block_diag(blocks).tocsr()
    part = np.repeat(np.arange(3), 40).astype(np.int32)
    sets = O.index_sets(A, part, 3)
    mj, km = O.multiplicity(A, sets)
    assert km == 1
    C = (A.T @ A).toarray()
    tot = sum((A[s.Xi, :].T @ A[s.Xi, :]).toarray() for s in sets)
    np.testing.assert_allclose(tot, C, atol=1e-13 * np.abs(C).max())


# ---------------------------------------------------------------------------
# coarse selection: independent routes and Lemma 2.4
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prob", [W.banded_1000(), W.small_config("grid"),
                                  W.small_config("banded"),
                                  W.random_banded(480, 960, 32, seed=232, name="rb32")],
                         ids=lambda p: p.name)
@pytest.mark.parametrize("tau", [0.05, 0.1, 0.3, 0.6])
def test_selection_count_four_routes(prob, tau):
    A = prob.scipy()
    sets = O.index_sets(A, prob.part, prob.nparts)
    for s in sets:
        Cii, Ctii = O.local_matrices(A, s)
        res = O.coarse_vectors(Cii, Ctii, s.nI, tau)
        cs, mu = O.selection_count_schur(Cii, Ctii, s.nI, tau)
        ca, mua = O.selection_count_angles(A, s, tau)
        if np.any(np.abs(mu - tau) <= 1e-9 * tau):
            pytest.skip("near tie at the threshold")
        assert res["p"] == cs == ca
        ci = O.selection_count_inertia(Cii, Ctii, s.nI, tau)
        assert ci == res["p"]


def _stability_ratio(Cii, Ctii, nI, Z, w):
    """tau-stability quantity of Lemma 2.4 for the local vector w = R_i u:
    u_i^T C_ii u_i / (w^T Ct_ii w) with u_i = D (I - Pi) w, Pi the orthogonal
    projection onto span(Z)."""
    d = np.concatenate([np.ones(nI), np.zeros(Cii.shape[0] - nI)])
    if Z.shape[1]:
        Q, _ = np.linalg.qr(Z)
        w_perp = w - Q @ (Q.T @ w)
    else:
        w_perp = w
    ui = d * w_perp
    return (ui @ Cii @ ui) / (w @ Ctii @ w)


@pytest.mark.parametrize("tau", [0.1, 0.4])
def test_lemma24_stable_and_minimal(tau):
    """tau u_i^T C_ii u_i <= u^T Ct_i u for every u (Lemma 2.4), and dropping any
    selected vector breaks it for some u (minimality)."""
    prob = W.banded_1000()
    A = prob.scipy()
    sets = O.index_sets(A, prob.part, prob.nparts)
    rng = np.random.default_rng(5)
    checked_minimal = 0
    for s in sets:
        Cii, Ctii = O.local_matrices(A, s)
        res = O.coarse_vectors(Cii, Ctii, s.nI, tau)
        Z = res["Z"]
        for _ in range(20):
            w = rng.standard_normal(s.ni)
            assert tau * _stability_ratio(Cii, Ctii, s.nI, Z, w) <= 1 + 1e-9
        # minimality: without the k-th selected vector, that vector itself
        # (or a mix of the selected ones) violates the inequality
        for k in range(Z.shape[1]):
            Zk = np.delete(Z, k, axis=1)
            worst = 0.0
            for w in [Z[:, k]] + [Z @ rng.standard_normal(Z.shape[1]) for _ in range(5)]:
                worst = max(worst, tau * _stability_ratio(Cii, Ctii, s.nI, Zk, w))
            assert worst > 1 + 1e-9
            checked_minimal += 1
    assert checked_minimal > 0


# ---------------------------------------------------------------------------
# Theorem 2.6 and Lemma 2.2 on dense small problems
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_theorem26_condition_bound(N):
    prob = W.random_banded(480, 960, N, seed=100 + N, name=f"bound{N}")
    A = prob.scipy()
    tau = 0.1
    orc = O.Oracle(A, prob.part, N, tau).setup()
    M = O.dense_preconditioner(orc)
    C = (A.T @ A).toarray()
    # eigenvalues of M C = those of the symmetric C^{1/2} M C^{1/2}
    Lc = np.linalg.cholesky(C)
    ev = sla.eigvalsh(Lc.T @ M @ Lc)
    kappa = ev.max() / ev.min()
    _, km = O.multiplicity(A, orc.sets)
    _, kc = O.greedy_colouring(A, orc.sets)
    assert ev.min() > 0
    assert kappa <= O.theorem26_bound(kc, km, tau)
    # Lemma 2.2: the upper end c_u = k_c + 1
    assert ev.max() <= (kc + 1) * (1 + 1e-10)


def test_theorem26_bound_on_grid_needs_the_coarse_space():
    """On a grid Laplacian-like problem one-level ASM is far outside the
    Theorem 2.6 bound while the two-level operator is inside it.  The additive
    coarse term is positive semidefinite, so by Weyl's inequalities every
    eigenvalue of M_additive C is at least the matching one of M_ASM C."""
    prob = W.small_config("grid")
    A = prob.scipy()
    C = (A.T @ A).toarray()
    Lc = np.linalg.cholesky(C)
    ev = {}
    for variant in ["additive", "one_level"]:
        orc = O.Oracle(A, prob.part, prob.nparts, prob.tau, variant=variant).setup()
        ev[variant] = sla.eigvalsh(Lc.T @ O.dense_preconditioner(orc) @ Lc)
    _, km = O.multiplicity(A, orc.sets)
    _, kc = O.greedy_colouring(A, orc.sets)
    bound = O.theorem26_bound(kc, km, prob.tau)
    add, one = ev["additive"], ev["one_level"]
    assert add.min() > 0 and add.max() / add.min() <= bound
    assert one.max() / one.min() > bound
    # the coarse term is PSD up to rounding amplified by kappa(E): 1e-6 slack
    assert np.all(add >= one - 1e-6 * one.max())


# ---------------------------------------------------------------------------
# special cases and brute force
# ---------------------------------------------------------------------------

def test_single_subdomain_is_exact_solve():
    """N = 1: Gamma is empty, M = C^{-1}, one PCG step reaches the LS solution."""
    prob = W.random_banded(200, 400, 1, seed=3)
    A = prob.scipy()
    orc = O.Oracle(A, prob.part, 1, 0.1).setup()
    assert orc.sets[0].nG == 0 and orc.n0 == 0
    sol = orc.solve(prob.b, tol=1e-10)
    assert sol["its"] == 1
    xs = np.linalg.lstsq(A.toarray(), prob.b, rcond=None)[0]
    np.testing.assert_allclose(sol["x"], xs, rtol=0, atol=1e-10 * np.abs(xs).max())


def test_tiny_tau_gives_one_level_asm():
    """tau -> 0 selects nothing, so M_additive = M_ASM (eq. one_level_schwarz)."""
    prob = W.random_banded(150, 300, 4, seed=4)
    A = prob.scipy()
    orc = O.Oracle(A, prob.part, 4, 1e-12).setup()
    assert orc.n0 == 0
    Cd = (A.T @ A).toarray()
    n = prob.n
    Masm = np.zeros((n, n))
    for s in orc.sets:
        Om = s.Omega
        Masm[np.ix_(Om, Om)] += np.linalg.inv(Cd[np.ix_(Om, Om)])
    np.testing.assert_allclose(O.dense_preconditioner(orc), Masm, rtol=1e-9,
                               atol=1e-12 * np.abs(Masm).max())


@pytest.mark.parametrize("variant", ["additive", "one_level", "balanced"])
def test_pcg_matches_dense_least_squares(variant):
    prob = W.banded_1000()
    A = prob.scipy()
    orc = O.Oracle(A, prob.part, prob.nparts, prob.tau, variant=variant).setup()
    sol = orc.solve(prob.b, tol=1e-12)
    xs = np.linalg.lstsq(A.toarray(), prob.b, rcond=None)[0]
    assert np.linalg.norm(sol["x"] - xs) <= 1e-9 * np.linalg.norm(xs)
    assert sol["relres"] <= 1e-12


# ---------------------------------------------------------------------------
# balanced two-level form (eq. balanced): properties fixed by C, Q and E
# ---------------------------------------------------------------------------

def _balanced_small():
    prob = W.random_banded(240, 480, 6, seed=5)
    A = prob.scipy()
    orc = O.Oracle(A, prob.part, prob.nparts, 0.3, variant="balanced").setup()
    assert orc.n0 > 0
    return A, orc


def test_balanced_coarse_space_is_unit_eigenspace():
    """M C R_0^T = R_0^T: with E = R_0 C R_0^T, (I - C Q) C R_0^T = 0 and
    Q C R_0^T = R_0^T, so every coarse vector is an eigenvector of M C with
    eigenvalue 1."""
    A, orc = _balanced_small()
    CR0T = (A.T @ (A @ orc.R0T)).toarray()
    R0T = orc.R0T.toarray()
    MC = np.column_stack([orc.apply(CR0T[:, k]) for k in range(orc.n0)])
    np.testing.assert_allclose(MC, R0T, atol=1e-9 * np.abs(R0T).max())


def test_balanced_correction_is_C_orthogonal_to_coarse_space():
    """R_0 C (M r - Q r) = 0: the first-level part leaves the coarse space
    C-orthogonally, since R_0 C (I - Q C) = 0."""
    A, orc = _balanced_small()
    rng = np.random.default_rng(1)
    C = (A.T @ A).toarray()
    for _ in range(3):
        r = rng.standard_normal(orc.n)
        d = orc.apply(r) - orc.apply_coarse(r)
        lhs = orc.R0T.T @ (C @ d)
        scale = np.abs(orc.R0T.T @ (C @ np.abs(d))).max()
        assert np.abs(lhs).max() <= 1e-11 * scale


def test_balanced_is_symmetric_positive_definite():
    """Symmetric when M_ASM is (the paper states it), and positive definite:
    the eigenvalues of L^T M L (C = L L^T) are those of M C, all positive,
    with the n_0 unit ones of the coarse space among them."""
    A, orc = _balanced_small()
    M = O.dense_preconditioner(orc)
    np.testing.assert_allclose(M, M.T, atol=1e-12 * np.abs(M).max())
    Lc = np.linalg.cholesky((A.T @ A).toarray())
    ev = sla.eigvalsh(Lc.T @ M @ Lc)
    assert ev.min() > 0
    assert np.sum(np.abs(ev - 1.0) < 1e-8) >= orc.n0


def test_balanced_without_coarse_space_is_one_level():
    """n_0 = 0 (tau tiny): Q = 0, so the balanced form is M_ASM."""
    prob = W.random_banded(240, 480, 6, seed=5)
    A = prob.scipy()
    bal = O.Oracle(A, prob.part, prob.nparts, 1e-12, variant="balanced").setup()
    one = O.Oracle(A, prob.part, prob.nparts, 1e-12, variant="one_level").setup()
    assert bal.n0 == 0
    r = np.random.default_rng(2).standard_normal(bal.n)
    np.testing.assert_allclose(bal.apply(r), one.apply(r), rtol=0, atol=0)


def test_balanced_needs_no_more_iterations_than_additive():
    """The balanced form converges at least as fast as the additive one on the
    banded 1000-column problem (its spectrum clusters the coarse space at 1)."""
    prob = W.banded_1000()
    A = prob.scipy()
    its = {v: O.Oracle(A, prob.part, prob.nparts, prob.tau, variant=v).setup()
           .solve(prob.b, tol=1e-8)["its"] for v in ["additive", "balanced"]}
    assert its["balanced"] <= its["additive"]


def test_flexible_pcg_same_solution():
    prob = W.banded_1000()
    A = prob.scipy()
    orc = O.Oracle(A, prob.part, prob.nparts, prob.tau).setup()
    a = orc.solve(prob.b, tol=1e-10)
    b = orc.solve(prob.b, tol=1e-10, flexible=True)
    assert abs(a["its"] - b["its"]) <= 1
    assert np.linalg.norm(a["x"] - b["x"]) <= 1e-8 * np.linalg.norm(a["x"])


def test_two_level_bound_independent_of_N():
    """Iteration counts stay bounded as N grows (Theorem 2.6): two-level PCG on
    the same matrix with N = 4 .. 32 parts."""
    its = []
    for N in [4, 8, 16, 32]:
        prob = W.random_banded(960, 1920, N, seed=9)
        orc = O.Oracle(prob.scipy(), prob.part, N, 0.1).setup()
        its.append(orc.solve(prob.b, tol=1e-8)["its"])
    assert max(its) <= 40


# ---------------------------------------------------------------------------
# adjoint against central finite differences
# ---------------------------------------------------------------------------

def test_adjoint_against_central_differences():
    prob = W.random_banded(60, 180, 3, seed=8, k=3, half_width=6)
    A = prob.scipy()
    rng = np.random.default_rng(1)
    xstar = rng.standard_normal(prob.n)
    orc = O.Oracle(A, prob.part, 3, 0.3).setup()
    x = orc.solve(prob.b, tol=1e-14)["x"]
    g = x - xstar
    grads = orc.backward(prob.b, x, g, tol=1e-14)

    def loss(data, b):
        Ad = sp.csr_matrix((data, prob.indices, prob.indptr), shape=(prob.m, prob.n)).toarray()
        xx = np.linalg.lstsq(Ad, b, rcond=None)[0]
        return 0.5 * np.sum((xx - xstar) ** 2)

    h = 1e-6
    for k in rng.choice(prob.nnz, 8, replace=False):
        dp = prob.data.copy(); dp[k] += h
        dm = prob.data.copy(); dm[k] -= h
        fd = (loss(dp, prob.b) - loss(dm, prob.b)) / (2 * h)
        assert abs(fd - grads["dLdvals"][k]) <= 1e-6 * max(1.0, abs(fd))
    for k in rng.choice(prob.m, 8, replace=False):
        bp = prob.b.copy(); bp[k] += h
        bm = prob.b.copy(); bm[k] -= h
        fd = (loss(prob.data, bp) - loss(prob.data, bm)) / (2 * h)
        assert abs(fd - grads["dLdb"][k]) <= 1e-6 * max(1.0, abs(fd))


def test_generators_are_deterministic():
    a = W.banded_1000()
    b = W.banded_1000()
    for f in ["indptr", "indices", "data", "b", "part"]:
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert a.m == 3000 and a.n == 1000 and a.nnz == 9000
    g = W.grid_gradient(10, 2, seed=1)
    assert g.m == 2 * 10 * 9 + 100 and g.nnz == 4 * 10 * 9 + 100
    # every row of the random part has distinct, sorted columns
    for r in range(a.m):
        cols = a.indices[a.indptr[r]:a.indptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


# ---------------------------------------------------------------------------
# Remarks 3.1 and 3.2: QR local factors and principal-angle selection
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prob", _small_problems() + [W.worked_example()], ids=lambda p: p.name)
def test_qr_factor_is_the_cholesky_factor(prob):
    """Remark 3.1: R of a thin QR of A(:, Omega_i) with a positive diagonal
    is the Cholesky factor of C_ii (uniqueness of both); checked against the
    library Cholesky of the formed C_ii."""
    A = prob.scipy()
    for s in O.index_sets(A, prob.part, prob.nparts):
        Cii, _ = O.local_matrices(A, s)
        L = O.local_factor_qr(A, s)
        Lc = np.linalg.cholesky(Cii)
        assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
        kap = np.linalg.cond(Cii)
        np.testing.assert_allclose(L, Lc, atol=1e2 * kap ** 0.5 * np.finfo(float).eps * np.abs(Lc).max())


def test_qr_factor_where_cholesky_breaks_down():
    """Closed form: A = G [[1, 1], [0, d]] with a plane rotation G has
    R = [[1, 1], [0, d]].  At d = 1e-10, C = A^T A = [[1, 1], [1, 1 + d^2]]
    rounds to a singular matrix and its Cholesky factorization fails, while
    the QR route recovers d to about eps / d."""
    d, th = 1e-10, 0.7
    c, sn = np.cos(th), np.sin(th)
    Ad = np.array([[c, c - sn * d], [sn, sn + c * d]])
    A = sp.csr_matrix(Ad)
    s = O.Subdomain(np.array([0, 1]), np.array([0, 1]), np.array([], dtype=np.int64))
    L = O.local_factor_qr(A, s)
    assert L[0, 0] == pytest.approx(1.0, rel=1e-15)
    assert L[1, 0] == pytest.approx(1.0, rel=1e-14)
    assert L[1, 1] == pytest.approx(d, rel=1e-4)
    C = Ad.T @ Ad
    try:
        Lc = np.linalg.cholesky(C)
    except np.linalg.LinAlgError:
        return
    assert not (abs(Lc[1, 1] - d) <= 1e-4 * d)


@pytest.mark.parametrize("prob", [W.banded_1000(), W.small_config("grid"),
                                  W.small_config("banded"),
                                  W.random_banded(480, 960, 32, seed=232, name="rb32")],
                         ids=lambda p: p.name)
@pytest.mark.parametrize("tau", [0.05, 0.1, 0.3, 0.6])
def test_angle_selection_matches_library_angles_and_lemma24(prob, tau):
    """Remark 3.2 / route (iii) as the production route: sin^2 of the
    Bjorck-Golub angles equal those of the library routine
    (scipy.linalg.subspace_angles), the count equals the Lemma 2.4 count,
    and X_i spans the same space as Lemma 2.4's, C_I-orthonormal."""
    A = prob.scipy()
    for s in O.index_sets(A, prob.part, prob.nparts):
        res = O.coarse_vectors_angles(A, s, tau)
        ca, mua = O.selection_count_angles(A, s, tau)
        if np.any(np.abs(mua - tau) <= 1e-9 * tau):
            pytest.skip("near tie at the threshold")
        k = min(res["mu"].size, mua.size)
        np.testing.assert_allclose(np.sort(res["mu"])[:k], np.sort(mua)[:k], atol=1e-12)
        Cii, Ctii = O.local_matrices(A, s)
        ref = O.coarse_vectors(Cii, Ctii, s.nI, tau)
        assert res["p"] == ca == ref["p"]
        X = res["X"]
        if X.shape[1] == 0:
            continue
        CI = Cii[:s.nI, :s.nI]
        np.testing.assert_allclose(X.T @ CI @ X, np.eye(X.shape[1]), atol=1e-9)
        # principal angles between the two spans, in the C_I inner product
        Lc = np.linalg.cholesky(CI)
        Qa, _ = np.linalg.qr(Lc.T @ X)
        Qb, _ = np.linalg.qr(Lc.T @ ref["X"])
        sv = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
        assert sv.min() >= 1.0 - 1e-10


@pytest.mark.parametrize("tau,expect", [(0.6, (0, 1)), (0.70, (1, 1)), (0.69, (0, 1)),
                                        (0.47, (0, 1)), (0.46, (0, 0))])
def test_worked_example_angle_selection_thresholds(tau, expect):
    """The printed example through the QR route: subdomain 1 is selected iff
    tau > 9/13, subdomain 2 iff tau > 100/213 (sin^2 theta = 9/13 and
    100/213, the reciprocals of the closed-form eigenvalues), and the coarse
    vector at tau = 0.6 is (0, 113, 0, -35)."""
    p = W.worked_example()
    orc = O.Oracle(p.scipy(), p.part, p.nparts, tau, local_factor="qr").setup()
    assert tuple(orc.p) == expect
    sets = O.index_sets(p.scipy(), p.part, p.nparts)
    mus = [np.sort(O.coarse_vectors_angles(p.scipy(), s, tau)["mu"]) for s in sets]
    assert mus[0][0] == pytest.approx(9 / 13, rel=1e-13)
    assert mus[1][0] == pytest.approx(100 / 213, rel=1e-13)
    if tau == 0.6:
        v = orc.R0T.toarray()[:, 0]
        ref = np.array([0.0, 113.0, 0.0, -35.0])
        assert abs(v @ ref) / (np.linalg.norm(v) * np.linalg.norm(ref)) == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("variant", ["additive", "one_level"])
def test_qr_route_pcg_matches_dense_least_squares(variant):
    prob = W.banded_1000()
    A = prob.scipy()
    orc = O.Oracle(A, prob.part, prob.nparts, prob.tau, variant=variant, local_factor="qr").setup()
    ref = O.Oracle(A, prob.part, prob.nparts, prob.tau, variant=variant).setup()
    assert np.array_equal(orc.p, ref.p)
    r = np.random.default_rng(3).standard_normal(prob.n)
    z, zr = orc.apply(r), ref.apply(r)
    assert np.linalg.norm(z - zr) <= 1e-8 * np.linalg.norm(zr)
    sol = orc.solve(prob.b, tol=1e-12)
    xs = np.linalg.lstsq(A.toarray(), prob.b, rcond=None)[0]
    assert np.linalg.norm(sol["x"] - xs) <= 1e-9 * np.linalg.norm(xs)
