"""Planted mistakes in the CPU oracle must make a pin fail.

Each test replaces one oracle function by a version with a plausible slip:
a transposed operand, a dropped term or factor, a threshold read the wrong
way, or a wrong sign.  It then runs an existing pin from test_oracle_pins.py
and expects it to fail.  The mistakes are planted only here, on the CPU, and
only for the duration of one test.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import oracle.lsq2l_oracle as OM
from tests import test_oracle_pins as P
from workloads import generators as W


def plant(monkeypatch, name, fn):
    """Replace oracle function ``name`` in the package and in its module (the
    module-internal callers look it up there)."""
    monkeypatch.setattr(O, name, fn)
    monkeypatch.setattr(OM, name, fn)


def test_xi_from_column_indices_is_caught(monkeypatch):
    """Transposed operand: Xi_i read from the CSR column indices of A(:, Omega_I)."""
    def bad(A, part, nparts):
        A = sp.csr_matrix(A)
        out = []
        for i in range(nparts):
            I = np.flatnonzero(np.asarray(part) == i).astype(np.int64)
            Xi = np.unique(A[:, I].indices).astype(np.int64)
            cols = np.unique(A[Xi, :].indices).astype(np.int64)
            out.append(OM.Subdomain(I, Xi, np.setdiff1d(cols, I, assume_unique=True)))
        return out
    plant(monkeypatch, "index_sets", bad)
    with pytest.raises(AssertionError):
        P.test_worked_example_index_sets_match_paper()


def test_partition_of_unity_without_zero_block_is_caught(monkeypatch):
    plant(monkeypatch, "partition_of_unity", lambda s: np.ones(s.ni))
    with pytest.raises(AssertionError):
        P.test_worked_example_partition_of_unity_sums_to_identity()


def test_splitting_over_all_rows_is_caught(monkeypatch):
    """Dropped restriction: Ct_ii built from every row of A instead of Xi_i."""
    def bad(A, s):
        A = sp.csr_matrix(A)
        Ac = A[:, s.Omega]
        C = (Ac.T @ Ac).toarray()
        return C, C.copy()
    plant(monkeypatch, "local_matrices", bad)
    with pytest.raises(AssertionError):
        P.test_worked_example_local_matrices_closed_form()


def test_pencil_without_partition_of_unity_is_caught(monkeypatch):
    """Dropped factor: C_ii v = lambda Ct_ii v instead of D C D v = lambda Ct v."""
    good = OM.coarse_vectors

    def bad(Cii, Ctii, nI, tau, nev_max=0):
        return good(Cii, Ctii, Cii.shape[0], tau, nev_max)
    plant(monkeypatch, "coarse_vectors", bad)
    with pytest.raises(AssertionError):
        P.test_worked_example_eigenvalues_closed_form()


def test_threshold_tau_instead_of_inverse_is_caught(monkeypatch):
    """Threshold read the wrong way: lambda > tau instead of lambda > 1 / tau."""
    good = OM.coarse_vectors

    def bad(Cii, Ctii, nI, tau, nev_max=0):
        return good(Cii, Ctii, nI, 1.0 / tau, nev_max)
    plant(monkeypatch, "coarse_vectors", bad)
    with pytest.raises(AssertionError):
        P.test_worked_example_selection_thresholds(0.46, (0, 0))


def test_schur_route_without_correction_is_caught(monkeypatch):
    """Dropped term in route (i): S = C_I instead of the generalized Schur complement."""
    def bad(Cii, Ctii, nI, tau):
        CI = Cii[:nI, :nI]
        mu = sla.eigh(CI, CI, eigvals_only=True)
        return int((mu < tau).sum()), mu
    plant(monkeypatch, "selection_count_schur", bad)
    prob = W.random_banded(480, 960, 32, seed=232, name="rb32")
    with pytest.raises(AssertionError):
        P.test_selection_count_four_routes(prob, 0.6)


def test_coarse_correction_with_wrong_sign_is_caught(monkeypatch):
    def bad(self, r):
        z = np.zeros(self.n)
        for s, F in zip(self.sets, self.chol):
            z[s.Omega] += sla.cho_solve(F, r[s.Omega])
        if self.cholE is not None:
            z -= self.R0T @ sla.cho_solve(self.cholE, self.R0T.T @ r)
        return z
    monkeypatch.setattr(O.Oracle, "apply", bad)
    with pytest.raises(AssertionError):
        P.test_theorem26_bound_on_grid_needs_the_coarse_space()


def test_adjoint_with_wrong_sign_is_caught(monkeypatch):
    def bad(self, b, x, g, tol=1e-12, maxit=10000):
        A = self.A
        lam = OM.pcg(A, g, self.apply, tol, maxit)["x"]
        Alam = A @ lam
        r = b - A @ x
        rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
        dvals = r[rows] * lam[A.indices] + Alam[rows] * x[A.indices]
        return {"dLdb": Alam, "dLdvals": dvals, "lam": lam, "its": 0}
    monkeypatch.setattr(O.Oracle, "backward", bad)
    with pytest.raises(AssertionError):
        P.test_adjoint_against_central_differences()


def test_balanced_without_first_coarse_term_is_caught(monkeypatch):
    """Dropped term: M r = (I - Q C) M_ASM (I - C Q) r without the leading Q r."""
    def bad(self, r):
        A = self.A
        Qr = self.apply_coarse(r)
        y = self.apply_one_level(r - A.T @ (A @ Qr))
        return y - self.apply_coarse(A.T @ (A @ y))
    monkeypatch.setattr(OM.Oracle, "apply", bad)
    with pytest.raises(AssertionError):
        P.test_balanced_coarse_space_is_unit_eigenspace()


def test_balanced_with_untransposed_left_factor_is_caught(monkeypatch):
    """Transposed operand: (I - C Q) on the left instead of (I - C Q)^T."""
    def bad(self, r):
        A = self.A
        Qr = self.apply_coarse(r)
        y = self.apply_one_level(r - A.T @ (A @ Qr))
        return Qr + y - A.T @ (A @ self.apply_coarse(y))
    monkeypatch.setattr(OM.Oracle, "apply", bad)
    with pytest.raises(AssertionError):
        P.test_balanced_correction_is_C_orthogonal_to_coarse_space()
    with pytest.raises(AssertionError):
        P.test_balanced_is_symmetric_positive_definite()


# ---------------------------------------------------------------------------
# planted mistakes in the Krylov methods, the RAS / deflated forms and the
# shift: one edit of the oracle's source each, checked against the pins of
# test_oracle_krylov.py
# ---------------------------------------------------------------------------
import inspect  # noqa: E402
import textwrap  # noqa: E402

from tests import test_oracle_krylov as PK  # noqa: E402


def mutant(fn, old, new):
    """The oracle function ``fn`` with one source fragment replaced."""
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, old
    ns = dict(vars(OM))
    exec(compile(src.replace(old, new), OM.__file__, "exec"), ns)
    return ns[fn.__name__]


def test_lsqr_rotation_sign_is_caught(monkeypatch):
    plant(monkeypatch, "lsqr", mutant(OM.lsqr, "rhobar = -c * alpha", "rhobar = c * alpha"))
    with pytest.raises(AssertionError):
        PK.test_lsqr_identity_preconditioner_matches_library_lsqr(5)


def test_lsqr_missing_preconditioner_in_alpha_is_caught(monkeypatch):
    """alpha from ||q|| instead of sqrt(q^T M q)."""
    plant(monkeypatch, "lsqr", mutant(OM.lsqr, "alpha = float(np.sqrt(q @ s))\n        # plane",
                                      "alpha = float(np.linalg.norm(q))\n        # plane"))
    with pytest.raises(AssertionError):
        PK.test_lsqr_preconditioned_is_lsqr_on_transformed_operator(3)


def test_gmres_update_without_preconditioner_is_caught(monkeypatch):
    """x += V y instead of x += M V y (right preconditioning dropped)."""
    plant(monkeypatch, "gmres", mutant(OM.gmres, "x = x + M(np.column_stack(V[:k]) @ y)",
                                       "x = x + np.column_stack(V[:k]) @ y"))
    with pytest.raises(AssertionError):
        PK.test_gmres_iterate_minimizes_residual_over_krylov_space(4)


def test_ras_without_partition_of_unity_is_caught(monkeypatch):
    bad = mutant(OM.Oracle.apply_one_level, "zi = partition_of_unity(s) * zi", "zi = 1.0 * zi")
    monkeypatch.setattr(OM.Oracle, "apply_one_level", bad)
    with pytest.raises(AssertionError):
        PK.test_ras_differs_from_asm_with_overlap()


def test_deflated_wrong_sign_is_caught(monkeypatch):
    bad = mutant(OM.Oracle.apply, "r - A.T @ (A @ Qr), restricted=True",
                 "r + A.T @ (A @ Qr), restricted=True")
    monkeypatch.setattr(OM.Oracle, "apply", bad)
    with pytest.raises(AssertionError):
        PK.test_deflated_coarse_space_is_unit_eigenspace()


def test_shift_on_squared_norm_is_caught(monkeypatch):
    plant(monkeypatch, "frobenius_normal", lambda A: float(np.sum((A.T @ A).tocsr().data ** 2)))
    with pytest.raises(AssertionError):
        PK.test_shift_single_subdomain_is_shifted_inverse()


# ---------------------------------------------------------------------------
# Remarks 3.1 and 3.2 (QR factors, principal-angle selection)
# ---------------------------------------------------------------------------

def test_qr_factor_over_xi_rows_only_is_caught(monkeypatch):
    """Dropped rows: the QR taken over Xi_i only gives the factor of the
    splitting matrix Ct_ii, not of C_ii."""
    def bad(A, s):
        A = sp.csr_matrix(A)
        R = np.linalg.qr(A[s.Xi, :][:, s.Omega].toarray(), mode="r")
        sg = np.where(np.diag(R) < 0.0, -1.0, 1.0)
        return (sg[:, None] * R).T
    plant(monkeypatch, "local_factor_qr", bad)
    with pytest.raises(AssertionError):
        P.test_qr_factor_is_the_cholesky_factor(W.small_config("grid"))


def test_qr_factor_without_sign_fix_is_caught(monkeypatch):
    def bad(A, s):
        A = sp.csr_matrix(A)
        Ac = A[:, s.Omega].tocsr()
        rows = np.flatnonzero(np.diff(Ac.indptr))
        return np.linalg.qr(Ac[rows].toarray(), mode="r").T
    plant(monkeypatch, "local_factor_qr", bad)
    with pytest.raises(AssertionError):
        P.test_qr_factor_is_the_cholesky_factor(W.worked_example())


def test_angle_threshold_on_cosines_is_caught(monkeypatch):
    """Threshold read the wrong way: cos^2 theta < tau instead of sin^2."""
    good = OM.coarse_vectors_angles

    def bad(A, s, tau, nev_max=0):
        return good(A, s, 1.0 - tau, nev_max)
    plant(monkeypatch, "coarse_vectors_angles", bad)
    with pytest.raises(AssertionError):
        P.test_worked_example_angle_selection_thresholds(0.70, (1, 1))


def test_angle_vectors_without_inverse_factor_are_caught(monkeypatch):
    """Inverted operand: X = R_I U instead of R_I^{-1} U."""
    good = OM.coarse_vectors_angles

    def bad(A, s, tau, nev_max=0):
        res = good(A, s, tau, nev_max)
        _, RI = np.linalg.qr(sp.csr_matrix(A)[s.Xi, :][:, s.I].toarray())
        res["X"] = RI @ (RI @ res["X"])      # R_I U with U = R_I X
        return res
    plant(monkeypatch, "coarse_vectors_angles", bad)
    with pytest.raises(AssertionError):
        P.test_angle_selection_matches_library_angles_and_lemma24(W.small_config("grid"), 0.1)
