"""Plain FP64 CPU oracle of the two-level Schwarz preconditioned normal equations.

TEST INFRASTRUCTURE.  This module exists to check the GPU library; only the
tests, the smoke entry point and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the library (no kernels, headers, helpers
or constants); both are fed by the seeded generators in ``workloads``.

What it computes (Al Daas, Jolivet, Scott, "A robust algebraic domain
decomposition preconditioner for sparse normal equations"):

* ``index_sets``        -- Section 3, eq. (reorderedA) and Algorithm 1:
                           Xi_i, Omega_Gamma_i, Omega_i = [Omega_Ii, Omega_Gamma_i];
* ``partition_of_unity``-- Section 3, the 0/1 matrices D_i of the worked
                           example and Section 3.3.1;
* ``local_matrices``    -- C_ii = A(:,Omega_i)^T A(:,Omega_i) (Section 3.1) and
                           the local SPSD splitting
                           Ct_ii = A(Xi_i,Omega_i)^T A(Xi_i,Omega_i) (eq. spsd_normal_eq);
* ``coarse_vectors``    -- Lemma 2.4 / eq. (gevp) with its 0 and infinity
                           conventions (Section 3.3.2): Z_i = L_i^perp (+)
                           span{v : lambda > 1/tau}, returned as the interior
                           part X_i of D_i Z_i;
* ``Oracle.setup``      -- Algorithm 1 steps in order: index sets, D_i, R_i,
                           Cholesky of C_ii, Z_i, R_0^T = [R_1^T D_1 Z_1, ...],
                           Cholesky of C_00 = (A R_0^T)^T (A R_0^T);
* ``local_factor_qr``, ``coarse_vectors_angles`` -- Remarks 3.1 and 3.2
                           (``Oracle(local_factor="qr")``): L_i from a thin QR
                           of A(:,Omega_i), and the selection from the
                           principal angles between range(A(Xi_i,Omega_Ii))
                           and range(A(Xi_i,Omega_Gamma_i)) (Bjorck-Golub),
                           sin^2 theta < tau;
* ``Oracle.apply``      -- M_additive = R_0^T C_00^{-1} R_0 + sum_i R_i^T C_ii^{-1} R_i
                           (eq. two_level_schwarz), the one-level M_ASM
                           (eq. one_level_schwarz), M_RAS (eq. RAS), and the
                           balanced and deflated second levels (eqs. balanced,
                           deflated);
* ``diag_shift_rel``    -- Section 4.1 "Setup phase": the preconditioner is
                           built for C + s I, s = diag_shift_rel ||C||_F (the
                           least-squares matrix [A; sqrt(s) I]) and applied to C;
* ``pcg``               -- preconditioned conjugate gradients on C x = A^T b
                           (eq. normal), x_0 = 0, C applied as A^T (A p);
* ``lsqr``              -- left-preconditioned LSQR (Section 4.1, "Solution
                           phase"): Golub-Kahan bidiagonalization of A W^{-1}
                           for M = W^{-1} W^{-T}, carried with products by M
                           only; stops on LSQR's estimate of
                           ||(A W^{-1})^T r|| / (||A W^{-1}||_F ||r||);
* ``gmres``             -- right-preconditioned restarted GMRES on C x = A^T b
                           (Section 4.2), stopping on the unpreconditioned
                           residual;
* ``Oracle.backward``   -- adjoint of x = C^{-1} A^T b: lambda = C^{-1} g,
                           dL/db = A lambda, dL/dA_ij = r_i lambda_j - (A lambda)_i x_j
                           on the stored pattern (differentiation of eq. normal);
* ``normal_solve_direct``, ``gradients`` -- the solution of eq. (normal) by a
                           sparse direct factorization of C, and the adjoint
                           gradient formula, for full-size checks;
* pin helpers           -- multiplicity m_j and k_m (Lemma 3.1), greedy colouring
                           k_c (Lemma 2.2), the bound of Theorem 2.6, and three
                           independent routes to the selection count (Schur
                           pencil, principal angles, inertia).

Readings of points the paper leaves open (all listed in the design notes):
nonzero means structurally stored; overlap is one layer; the eigenproblem is
solved exactly (no shift s) and selection is strict lambda > 1/tau; the
numerical rank of Ct_ii is decided after a symmetric diagonal scaling to unit
diagonal (a congruence that commutes with D_i and leaves the eigenvalues of
eq. gevp unchanged) with relative tolerance n_i * eps, a kernel direction is
infinite (in L^perp) when its interior part exceeds 1e-8, and the number of
coarse vectors p_i is the rank of D_i Z_i; no cap on the number
of eigenpairs unless ``nev_max`` is given; PCG stops on the recurrence
residual ||r_k|| <= tol ||A^T b|| and then checks the true residual,
restarting from it at most three times.

Parity status: every function here is pinned by a CPU test against values
the paper prints, closed forms, library routines or the paper's lemmas;
iteration counts have no published counterpart (parity unpinned against the
paper, the tables' data files are absent).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

EPS = np.finfo(np.float64).eps

__all__ = [
    "Subdomain", "index_sets", "partition_of_unity", "restriction",
    "local_matrices", "coarse_vectors", "selection_count_schur",
    "selection_count_angles", "selection_count_inertia", "multiplicity",
    "greedy_colouring", "theorem26_bound", "Oracle", "pcg", "lsqr", "gmres", "csr_matrix",
    "dense_preconditioner", "spmv", "spmv_t", "frobenius_normal", "gradients",
    "normal_solve_direct", "local_factor_qr", "coarse_vectors_angles",
]


def csr_matrix(m, n, indptr, indices, data) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(data, dtype=np.float64),
                          np.asarray(indices), np.asarray(indptr)), shape=(m, n))


def spmv(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = A x, y_i = sum_k A_ik x_k (library sparse product)."""
    return A @ x


def spmv_t(A: sp.csr_matrix, y: np.ndarray) -> np.ndarray:
    """x = A^T y (library sparse product on the transpose)."""
    return A.T @ y


# ---------------------------------------------------------------------------
# Section 3: index sets, restriction, partition of unity
# ---------------------------------------------------------------------------

@dataclass
class Subdomain:
    I: np.ndarray    # Omega_Ii, sorted column indices (0-based)
    Xi: np.ndarray   # Xi_i, sorted row indices of the nonzero rows of A(:, Omega_Ii)
    G: np.ndarray    # Omega_Gamma_i, sorted

    @property
    def Omega(self) -> np.ndarray:
        return np.concatenate([self.I, self.G])

    @property
    def nI(self) -> int:
        return int(self.I.size)

    @property
    def nG(self) -> int:
        return int(self.G.size)

    @property
    def ni(self) -> int:
        return self.nI + self.nG


def index_sets(A: sp.csr_matrix, part: np.ndarray, nparts: int,
               subdomains=None) -> list[Subdomain]:
    """Section 3 (eq. reorderedA), Algorithm 1 (FindNonzeroRows, FindNonzeroColumns).

    Xi_i     = rows of A with a stored entry in some column of Omega_Ii;
    Gamma_i  = columns with a stored entry in some row of Xi_i, minus Omega_Ii;
    Omega_i  = [Omega_Ii, Omega_Gamma_i], each part in ascending order.
    ``subdomains`` restricts the list to those indices (in that order).
    """
    A = sp.csr_matrix(A)
    Acsc = A.tocsc()
    out = []
    for i in (range(nparts) if subdomains is None else subdomains):
        I = np.flatnonzero(np.asarray(part) == i).astype(np.int64)
        Xi = np.unique(Acsc[:, I].indices).astype(np.int64)
        cols = np.unique(A[Xi, :].indices).astype(np.int64)
        G = np.setdiff1d(cols, I, assume_unique=True)
        out.append(Subdomain(I, Xi, G))
    return out


def partition_of_unity(s: Subdomain) -> np.ndarray:
    """Diagonal of D_i: one on the n_Ii interior entries, zero on Gamma (Section 3,
    worked example; Section 3.3.1)."""
    return np.concatenate([np.ones(s.nI), np.zeros(s.nG)])


def restriction(s: Subdomain, n: int) -> sp.csr_matrix:
    """R_i = I_n(Omega_i, :) (Section 2)."""
    Om = s.Omega
    return sp.csr_matrix((np.ones(Om.size), (np.arange(Om.size), Om)), shape=(Om.size, n))


def local_matrices(A: sp.csr_matrix, s: Subdomain) -> tuple[np.ndarray, np.ndarray]:
    """C_ii = A(:,Omega_i)^T A(:,Omega_i) (Section 3.1) and
    Ct_ii = A(Xi_i,Omega_i)^T A(Xi_i,Omega_i) (eq. spsd_normal_eq), both dense."""
    A = sp.csr_matrix(A)
    Ac = A[:, s.Omega]
    Cii = (Ac.T @ Ac).toarray()
    At = A[s.Xi, :][:, s.Omega]
    Ctii = (At.T @ At).toarray()
    return Cii, Ctii


# ---------------------------------------------------------------------------
# Lemma 2.4: local filtering eigenproblem and the coarse vectors
# ---------------------------------------------------------------------------

def coarse_vectors(Cii: np.ndarray, Ctii: np.ndarray, nI: int, tau: float,
                   nev_max: int = 0) -> dict:
    """Z_i of Lemma 2.4 with the conventions of eq. (gevp), restricted by D_i.

    The pencil D_i C_ii D_i v = lambda Ct_ii v is solved on range(Ct_ii);
    Ct_ii's kernel is split into L_i = ker(D C D) cap ker(Ct) (lambda = 0) and
    its complement L_i^perp inside ker(Ct) (lambda = infinity).  Selected:
    L_i^perp and every finite lambda > 1/tau.  Returns the interior block X_i
    of D_i Z_i, orthonormalised in the C_I = C_ii(I,I) inner product, plus the
    finite eigenvalues and counts.
    """
    ni = Cii.shape[0]
    d = np.concatenate([np.ones(nI), np.zeros(ni - nI)])
    DCD = d[:, None] * Cii * d[None, :]
    # symmetric diagonal scaling S Ct S, S = diag(Ct)^(-1/2); D S = S D.
    sc = 1.0 / np.sqrt(np.diag(Ctii))
    Ct_s = sc[:, None] * Ctii * sc[None, :]
    DCD_s = sc[:, None] * DCD * sc[None, :]
    lam_t, Q = sla.eigh(Ct_s)
    tol = ni * EPS * max(float(lam_t.max()), 0.0)
    in_range = lam_t > tol
    Qr, Qk = Q[:, in_range], Q[:, ~in_range]
    # finite eigenvalues: restrict to range(Ct) (the projection P_0 of Lemma 2.4)
    Wr = Qr / np.sqrt(lam_t[in_range])[None, :]
    H = Wr.T @ DCD_s @ Wr
    H = 0.5 * (H + H.T)
    lam, Y = sla.eigh(H)
    fin_vecs = Wr @ Y
    # infinite eigenvalues: L^perp in ker(Ct), L = {v in ker(Ct): D v = 0}
    if Qk.shape[1] > 0:
        # the kernel basis is orthonormal; a direction belongs to L^perp when
        # its interior part is not zero, decided at 1e-8 (the computed kernel
        # basis carries eps / gap noise in the interior rows of L)
        KI = Qk[:nI, :]
        _, sv, Vt = np.linalg.svd(KI, full_matrices=False)
        rk = int((sv > 1e-8).sum())
        inf_vecs = Qk @ Vt[:rk].T
    else:
        rk = 0
        inf_vecs = np.zeros((ni, 0))
    order_fin = np.argsort(-lam, kind="stable")          # largest lambda first
    sel_fin = [k for k in order_fin if lam[k] > 1.0 / tau]
    Z = np.concatenate([inf_vecs, fin_vecs[:, sel_fin]], axis=1)
    if nev_max and Z.shape[1] > nev_max:
        Z = Z[:, :nev_max]
    Z = sc[:, None] * Z                                  # undo the scaling: v = S w
    # The coarse space takes D_i Z_i (the columns R_i^T D_i Z_i of R_0^T).  A
    # vector of L^perp and a finite eigenvector of the range-restricted pencil
    # can share their D-part, so p_i is the rank of D_i Z_i: an orthonormal
    # basis of its span in the C_I inner product is kept.
    X = Z[:nI, :]                                        # D_i Z_i restricted to Omega_Ii
    p = 0
    if X.shape[1] > 0:
        CI = Cii[:nI, :nI]
        Gm = X.T @ CI @ X
        Gm = 0.5 * (Gm + Gm.T)
        w, U = sla.eigh(Gm)
        keep = w > ni * EPS * max(float(w.max()), 0.0)
        X = X @ (U[:, keep] / np.sqrt(w[keep])[None, :])
        p = int(keep.sum())
    return {"X": X, "Z": Z, "p": p, "lam": lam, "n_inf": rk, "n_fin": len(sel_fin),
            "rank_ct": int(in_range.sum())}


def selection_count_schur(Cii, Ctii, nI, tau) -> tuple[int, np.ndarray]:
    """Route (i): S x = mu C_I x with S = C_I - C_IG Ct_GG^+ C_GI; count mu < tau.

    Eliminating the Gamma block from eq. (gevp) gives C_I x = lambda S x, so
    lambda = 1/mu and lambda > 1/tau is mu < tau.
    """
    CI = Cii[:nI, :nI]
    CIG = Ctii[:nI, nI:]
    CtGG = Ctii[nI:, nI:]
    if CtGG.shape[0]:
        S = CI - CIG @ sla.pinvh(CtGG) @ CIG.T
    else:
        S = CI.copy()
    mu = sla.eigh(0.5 * (S + S.T), CI, eigvals_only=True)
    return int((mu < tau).sum()), mu


def selection_count_angles(A: sp.csr_matrix, s: Subdomain, tau) -> tuple[int, np.ndarray]:
    """Route (iii): principal angles theta between range(A(Xi,Omega_I)) and
    range(A(Xi,Omega_Gamma)) (library routine); mu = sin^2 theta < tau."""
    A = sp.csr_matrix(A)
    AI = A[s.Xi, :][:, s.I].toarray()
    AG = A[s.Xi, :][:, s.G].toarray()
    if AG.shape[1] == 0:
        return 0, np.zeros(0)
    th = sla.subspace_angles(AI, AG)
    mu = np.sin(th) ** 2
    return int((mu < tau).sum()), mu


def selection_count_inertia(Cii, Ctii, nI, tau) -> int:
    """Route (iv): number of negative eigenvalues of Ct_ii - tau D C_ii D
    (with a tolerance n_i eps ||.||), i.e. directions where lambda > 1/tau."""
    ni = Cii.shape[0]
    d = np.concatenate([np.ones(nI), np.zeros(ni - nI)])
    Mx = Ctii - tau * (d[:, None] * Cii * d[None, :])
    ev = sla.eigvalsh(Mx)
    return int((ev < -ni * EPS * np.abs(ev).max()).sum())


# ---------------------------------------------------------------------------
# Remarks 3.1 and 3.2: local factors and coarse selection without C_ii
# ---------------------------------------------------------------------------

def local_factor_qr(A: sp.csr_matrix, s: Subdomain) -> np.ndarray:
    """Remark 3.1: the Cholesky factor of C_ii from a thin QR factorization
    of A(:, Omega_i), without forming C_ii.  Rows of A with no stored entry in
    Omega_i are zero rows of A(:, Omega_i) and are left out.  R is made unique
    by a positive diagonal; returns L_i = R^T, so that C_ii = L_i L_i^T."""
    A = sp.csr_matrix(A)
    Ac = A[:, s.Omega].tocsr()
    rows = np.flatnonzero(np.diff(Ac.indptr))
    R = np.linalg.qr(Ac[rows].toarray(), mode="r")
    sg = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return (sg[:, None] * R).T


def coarse_vectors_angles(A: sp.csr_matrix, s: Subdomain, tau: float,
                          nev_max: int = 0) -> dict:
    """Lemma 2.4's selection read through principal angles (Remark 3.2: no
    C_ii or Ct_ii is formed).

    With A_I = A(Xi_i, Omega_Ii) and A_G = A(Xi_i, Omega_Gamma_i), eliminating
    the interface block from eq. (gevp) leaves S x = mu C_I x with
    S = A_I^T (I - P_G) A_I, P_G the orthogonal projector onto range(A_G), and
    lambda = 1/mu.  Written with orthonormal bases, the eigenvalues mu are
    sin^2 theta for the principal angles theta between range(A_I) and
    range(A_G) (and 1 for the directions of range(A_I) orthogonal to
    range(A_G)); theta = 0 covers the infinite eigenvalues of L_i^perp.
    Selected: sin^2 theta < tau, i.e. cos^2 theta > 1 - tau.

    The angles are those of Bjorck and Golub:
      Q_I R_I = A_I                (thin QR; A_I has full column rank, C_I
                                    being positive definite);
      A_G S P = Q R                (QR with column pivoting of A_G with unit
                                    columns, S = diag of inverse column norms;
                                    numerical rank r = #{k : |R_kk| > n_G eps},
                                    Q_G = Q(:, :r) spans range(A_G));
      U diag(cos theta) V^T = Q_I^T Q_G   (SVD, angles ascending).
    The interior part of the eigenvector of angle theta_k is proportional to
    C_I^{-1} C_IG y = R_I^{-1} Q_I^T A_G y with A_G y = Q_G v_k, that is to
    R_I^{-1} u_k; X_i = R_I^{-1} U(:, selected) is C_I-orthonormal.  With
    ``nev_max`` the nev_max smallest angles are kept."""
    A = sp.csr_matrix(A)
    AXi = A[s.Xi, :]
    AI = AXi[:, s.I].toarray()
    AG = AXi[:, s.G].toarray()
    nI, nG = AI.shape[1], AG.shape[1]
    QI, RI = np.linalg.qr(AI)
    if nG == 0:
        return {"X": np.zeros((nI, 0)), "p": 0, "mu": np.zeros(0), "rank_g": 0}
    cn = np.sqrt((AG * AG).sum(axis=0))
    sc = np.zeros(nG)
    sc[cn > 0] = 1.0 / cn[cn > 0]
    Q, R, _ = sla.qr(AG * sc[None, :], mode="economic", pivoting=True)
    r = int((np.abs(np.diag(R)) > nG * EPS).sum())
    if r == 0:
        return {"X": np.zeros((nI, 0)), "p": 0, "mu": np.zeros(0), "rank_g": 0}
    U, cos, _ = np.linalg.svd(QI.T @ Q[:, :r], full_matrices=False)
    cos = np.minimum(cos, 1.0)
    mu = 1.0 - cos * cos
    sel = np.flatnonzero(cos * cos > 1.0 - tau)
    if nev_max and sel.size > nev_max:
        sel = sel[:nev_max]
    X = sla.solve_triangular(RI, U[:, sel], lower=False)
    return {"X": X, "p": int(sel.size), "mu": mu, "rank_g": r}


# ---------------------------------------------------------------------------
# constants of the condition-number bound
# ---------------------------------------------------------------------------

def multiplicity(A: sp.csr_matrix, sets: list[Subdomain]) -> tuple[np.ndarray, int]:
    """m_j = #{i : j in Xi_i} and k_m = max_j m_j (Lemma 3.1)."""
    mj = np.zeros(A.shape[0], dtype=np.int64)
    for s in sets:
        mj[s.Xi] += 1
    return mj, int(mj.max(initial=0))


def greedy_colouring(A: sp.csr_matrix, sets: list[Subdomain]) -> tuple[np.ndarray, int]:
    """Colours of subdomains such that two subdomains with a stored coupling
    C(Omega_i, Omega_j) != 0 get different colours (Lemma 2.2); greedy in
    index order, so k_c is an upper bound on the minimum."""
    A = sp.csr_matrix(A)
    C = (A.T @ A).tocsr()
    C.data[:] = 1.0
    N = len(sets)
    member = sp.csr_matrix((np.ones(sum(s.ni for s in sets)),
                            (np.concatenate([np.full(s.ni, i) for i, s in enumerate(sets)]),
                             np.concatenate([s.Omega for s in sets]))),
                           shape=(N, A.shape[1]))
    adj = (member @ C @ member.T).tocsr()
    colour = -np.ones(N, dtype=np.int64)
    for i in range(N):
        nb = adj.indices[adj.indptr[i]:adj.indptr[i + 1]]
        used = set(int(colour[j]) for j in nb if j != i and colour[j] >= 0)
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour, int(colour.max(initial=-1) + 1)


def theorem26_bound(kc: int, km: int, tau: float) -> float:
    """kappa(M_additive C) <= (k_c + 1)(2 + (2 k_c + 1) k_m / tau) (Theorem 2.6)."""
    return (kc + 1) * (2.0 + (2 * kc + 1) * km / tau)


# ---------------------------------------------------------------------------
# Algorithm 1 and the preconditioned solve
# ---------------------------------------------------------------------------

@dataclass
class Oracle:
    A: sp.csr_matrix
    part: np.ndarray
    nparts: int
    tau: float
    variant: str = "additive"          # or "one_level", "balanced", "ras", "deflated"
    nev_max: int = 0
    diag_shift_rel: float = 0.0
    local_factor: str = "cholesky"     # or "qr" (Remarks 3.1 and 3.2)
    shift: float = 0.0
    sets: list = field(default_factory=list)
    chol: list = field(default_factory=list)
    X: list = field(default_factory=list)
    p: np.ndarray = None
    R0T: sp.csr_matrix = None
    E: np.ndarray = None
    cholE: tuple = None

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def n0(self) -> int:
        return int(self.p.sum()) if self.p is not None else 0

    def setup(self, subdomains=None) -> "Oracle":
        """Algorithm 1.  ``subdomains`` restricts the per-subdomain work to a
        list of indices (used to time a bounded sample; the result is then not
        a usable preconditioner)."""
        A = self.A = sp.csr_matrix(self.A)
        # the preconditioner is built for C + s I, i.e. for [A; sqrt(s) I]
        # (Section 4.1, "Setup phase"); the solve still uses A
        self.shift = self.diag_shift_rel * frobenius_normal(A) if self.diag_shift_rel > 0 else 0.0
        if self.shift > 0:
            n = A.shape[1]
            Ab = sp.vstack([A, np.sqrt(self.shift) * sp.identity(n, format="csr")]).tocsr()
        else:
            Ab = A
        self.Ab = Ab
        self.sets = index_sets(Ab, self.part, self.nparts)
        todo = range(self.nparts) if subdomains is None else subdomains
        self.chol = [None] * self.nparts
        self.X = [np.zeros((s.nI, 0)) for s in self.sets]
        self.info = [None] * self.nparts
        two_level = self.variant in ("additive", "balanced", "deflated")
        for i in todo:
            s = self.sets[i]
            if self.local_factor == "qr":
                # Remark 3.1: L_i from a QR of A(:, Omega_i); Remark 3.2: the
                # selection by principal angles, no C_ii or Ct_ii formed
                self.chol[i] = (local_factor_qr(Ab, s), True)
                if two_level:
                    res = coarse_vectors_angles(Ab, s, self.tau, self.nev_max)
                    self.X[i] = res["X"]
                    self.info[i] = res
                continue
            Cii, Ctii = local_matrices(Ab, s)
            self.chol[i] = sla.cho_factor(Cii, lower=True)
            if two_level:
                res = coarse_vectors(Cii, Ctii, s.nI, self.tau, self.nev_max)
                self.X[i] = res["X"]
                self.info[i] = res
        self.p = np.array([x.shape[1] for x in self.X], dtype=np.int64)
        if subdomains is not None:
            return self
        n0 = self.n0
        if n0 > 0:
            rows, cols, vals = [], [], []
            off = 0
            for s, X in zip(self.sets, self.X):
                pi = X.shape[1]
                if pi == 0:
                    continue
                rr, cc = np.meshgrid(s.I, np.arange(pi) + off, indexing="ij")
                rows.append(rr.ravel()); cols.append(cc.ravel()); vals.append(X.ravel())
                off += pi
            self.R0T = sp.csr_matrix((np.concatenate(vals),
                                      (np.concatenate(rows), np.concatenate(cols))),
                                     shape=(self.n, n0))
            W = (Ab @ self.R0T).toarray()
            self.E = W.T @ W
            self.cholE = sla.cho_factor(self.E, lower=True)
        return self

    def apply_one_level(self, r: np.ndarray, restricted: bool = False) -> np.ndarray:
        """M_ASM r = sum_{i >= 1} R_i^T C_ii^{-1} R_i r (eq. one_level_schwarz),
        or with ``restricted`` M_RAS r = sum_i R_i^T D_i C_ii^{-1} R_i r (eq. RAS)."""
        z = np.zeros(self.n)
        for s, F in zip(self.sets, self.chol):
            Om = s.Omega
            zi = sla.cho_solve(F, r[Om])
            if restricted:
                zi = partition_of_unity(s) * zi
            z[Om] += zi
        return z

    def apply_coarse(self, r: np.ndarray) -> np.ndarray:
        """Q r with Q = R_0^T C_00^{-1} R_0 and C_00 = E = R_0 C R_0^T."""
        if self.cholE is None:
            return np.zeros(self.n)
        return self.R0T @ sla.cho_solve(self.cholE, self.R0T.T @ r)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = M r.

        additive (eq. two_level_schwarz): M = M_ASM + Q.
        one_level: M = M_ASM.
        balanced (eq. balanced, with M_ASM as the first level):
        M = Q + (I - C Q)^T M_ASM (I - C Q); C and Q are symmetric, so
        (I - C Q)^T = I - Q C.
        ras (eq. RAS): M = M_RAS.
        deflated (eq. deflated, with M_RAS as the first level):
        M = Q + M_RAS (I - C Q).
        C is applied as A^T (A .); it is the matrix of the least-squares
        problem (unshifted), the factors come from the shifted one."""
        A = self.A
        if self.variant == "ras":
            return self.apply_one_level(r, restricted=True)
        if self.variant == "deflated":
            Qr = self.apply_coarse(r)
            return Qr + self.apply_one_level(r - A.T @ (A @ Qr), restricted=True)
        if self.variant == "balanced":
            Qr = self.apply_coarse(r)
            v = r - A.T @ (A @ Qr)                  # (I - C Q) r
            y = self.apply_one_level(v)             # M_ASM (I - C Q) r
            return Qr + y - self.apply_coarse(A.T @ (A @ y))
        z = self.apply_one_level(r)
        if self.variant == "additive":
            z += self.apply_coarse(r)
        return z

    def solve(self, b: np.ndarray, tol: float = 1e-8, maxit: int = 10000,
              flexible: bool = False, method: str = "pcg", restart: int = 100) -> dict:
        if method == "lsqr":
            return lsqr(self.A, b, self.apply, tol, maxit)
        if method == "gmres":
            return gmres(self.A, self.A.T @ b, self.apply, tol, maxit, restart)
        return pcg(self.A, self.A.T @ b, self.apply, tol, maxit, flexible)

    def backward(self, b: np.ndarray, x: np.ndarray, g: np.ndarray,
                 tol: float = 1e-12, maxit: int = 10000) -> dict:
        """lambda = C^{-1} g; dL/db = A lambda; dL/dvals = r_i lambda_j - (A lambda)_i x_j."""
        A = self.A
        sol = pcg(A, g, self.apply, tol, maxit)
        lam = sol["x"]
        out = gradients(A, b, x, lam)
        out.update({"lam": lam, "its": sol["its"]})
        return out


def pcg(A: sp.csr_matrix, rhs: np.ndarray, M, tol: float, maxit: int,
        flexible: bool = False) -> dict:
    """Preconditioned CG on C x = rhs, C = A^T A applied as A^T (A p), x_0 = 0.

    Stops when ||r_k|| <= tol ||rhs|| on the recurrence residual, then forms
    the true residual rhs - C x; if that misses tol the iteration restarts from
    it (at most three restarts).  ``flexible`` uses
    beta = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k).
    """
    n = A.shape[1]
    x = np.zeros(n)
    nrm0 = float(np.linalg.norm(rhs))
    hist = []
    if nrm0 == 0.0:
        return {"x": x, "its": 0, "relres": 0.0, "hist": hist, "restarts": 0}
    r = rhs.copy()
    its = 0
    restarts = 0
    while True:
        z = M(r)
        rz = float(r @ z)
        p = z.copy()
        while its < maxit:
            q = A.T @ (A @ p)
            pq = float(p @ q)
            alpha = rz / pq
            x = x + alpha * p
            r_old = r
            r = r - alpha * q
            its += 1
            rel = float(np.linalg.norm(r)) / nrm0
            hist.append(rel)
            if rel <= tol:
                break
            z_new = M(r)
            rz_new = float(r @ z_new)
            beta = (float(z_new @ (r - r_old)) if flexible else rz_new) / rz
            rz = rz_new
            p = z_new + beta * p
        true_r = rhs - A.T @ (A @ x)
        relt = float(np.linalg.norm(true_r)) / nrm0
        if relt <= tol or restarts == 3 or its >= maxit:
            return {"x": x, "its": its, "relres": relt, "hist": hist, "restarts": restarts}
        r = true_r
        restarts += 1


def dense_preconditioner(orc: Oracle) -> np.ndarray:
    """The matrix M of ``orc.apply`` (small problems only)."""
    n = orc.n
    return np.column_stack([orc.apply(e) for e in np.eye(n)])


def frobenius_normal(A: sp.csr_matrix) -> float:
    """||C||_F for C = A^T A (library sparse product)."""
    C = (A.T @ A).tocsr()
    return float(np.sqrt(np.sum(C.data ** 2)))


def lsqr(A: sp.csr_matrix, b: np.ndarray, M, tol: float, maxit: int) -> dict:
    """Left-preconditioned LSQR on min ||A x - b||_2 (Section 4.1).

    With M = W^{-1} W^{-T} symmetric positive definite, LSQR (Paige and
    Saunders) runs on the operator A W^{-1}; its right vectors v are kept as
    vt = W^{-1} v and zh = W^T v, so that
        beta u = A vt - alpha u,
        alpha v = W^{-T} A^T u - beta v   becomes
        q = A^T u - beta zh,  s = M q,  alpha = sqrt(q^T s),
        zh = q / alpha,  vt = s / alpha,
    and the iterate x = W^{-1} y is updated with wt = W^{-1} w.  Stops when
    the estimate alpha |tau| / (anorm phibar) of
    ||(A W^{-1})^T r|| / (||A W^{-1}||_F ||r||) is at most tol, anorm the
    Frobenius norm of the bidiagonal matrix so far.
    """
    n = A.shape[1]
    x = np.zeros(n)
    u = b.copy()
    beta = float(np.linalg.norm(u))
    hist = []
    if beta == 0.0:
        return {"x": x, "its": 0, "test": 0.0, "hist": hist}
    u /= beta
    q = A.T @ u
    s = M(q)
    alpha = float(np.sqrt(q @ s))
    if alpha == 0.0:
        return {"x": x, "its": 0, "test": 0.0, "hist": hist}
    zh = q / alpha
    vt = s / alpha
    wt = vt.copy()
    rhobar, phibar = alpha, beta
    anorm2 = 0.0
    its = 0
    test = 1.0
    while its < maxit:
        u = A @ vt - alpha * u
        beta = float(np.linalg.norm(u))
        anorm2 += alpha * alpha + beta * beta
        if beta > 0:
            u /= beta
        q = A.T @ u - beta * zh
        s = M(q)
        alpha = float(np.sqrt(q @ s))
        # plane rotation eliminating beta below the diagonal
        rho = float(np.hypot(rhobar, beta))
        c, sn = rhobar / rho, beta / rho
        theta = sn * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = sn * phibar
        tau = sn * phi
        x = x + (phi / rho) * wt
        if alpha > 0:
            zh = q / alpha
            vt = s / alpha
        else:
            zh = np.zeros(n)
            vt = np.zeros(n)
        wt = vt - (theta / rho) * wt
        its += 1
        test = 0.0 if phibar == 0.0 else alpha * abs(tau) / (np.sqrt(anorm2) * phibar)
        hist.append(test)
        if test <= tol or alpha == 0.0:
            break
    return {"x": x, "its": its, "test": test, "hist": hist}


def gmres(A: sp.csr_matrix, rhs: np.ndarray, M, tol: float, maxit: int,
          restart: int = 100) -> dict:
    """Right-preconditioned restarted GMRES on C x = rhs, C = A^T A (Section 4.2).

    Each cycle builds an orthonormal basis V of the Krylov space of C M from
    the true residual (Arnoldi, modified Gram-Schmidt), minimizes the residual
    over x_0 + M V y by the Hessenberg least-squares problem (library
    lstsq), and restarts.  Stops when ||rhs - C x|| <= tol ||rhs|| (the
    unpreconditioned residual), checked on the Arnoldi estimate inside a cycle
    and on the true residual between cycles.
    """
    n = A.shape[1]
    x = np.zeros(n)
    nrm0 = float(np.linalg.norm(rhs))
    its = 0
    cycles = 0
    hist = []
    while True:
        r = rhs - A.T @ (A @ x)
        beta = float(np.linalg.norm(r))
        if beta <= tol * nrm0 or its >= maxit:
            return {"x": x, "its": its, "relres": beta / nrm0 if nrm0 else 0.0,
                    "cycles": cycles, "hist": hist}
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        k = 0
        for j in range(restart):
            if its >= maxit:
                break
            w = A.T @ (A @ M(V[j]))
            for i in range(j + 1):
                H[i, j] = float(V[i] @ w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            its += 1
            k = j + 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
            est = float(np.linalg.norm(e1 - H[:k + 1, :k] @ y))
            hist.append(est / nrm0)
            if est <= tol * nrm0 or H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
        x = x + M(np.column_stack(V[:k]) @ y)
        cycles += 1


def gradients(A: sp.csr_matrix, b: np.ndarray, x: np.ndarray, lam: np.ndarray) -> dict:
    """Implicit differentiation of x = C^{-1} A^T b for L(x) with lam = C^{-1} dL/dx:
    dL/db = A lam and dL/dA_ij = r_i lam_j - (A lam)_i x_j, r = b - A x, on the
    stored pattern of A (CSR order)."""
    Alam = A @ lam
    r = b - A @ x
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    dvals = r[rows] * lam[A.indices] - Alam[rows] * x[A.indices]
    return {"dLdb": Alam, "dLdvals": dvals}


def normal_solve_direct(A: sp.csr_matrix, rhs: np.ndarray) -> np.ndarray:
    """C x = rhs, C = A^T A, by a sparse direct factorization of C (library
    LU); used where an iterative oracle solve would take too long."""
    import scipy.sparse.linalg as spla
    C = (A.T @ A).tocsc()
    return spla.spsolve(C, rhs)

