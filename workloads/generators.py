"""Deterministic generators for the synthetic least-squares problems.

Every problem is min ||Ax - b||_2 with A (m x n, m >= n) sparse.  The paper's
own test matrices come from the SuiteSparse collection (Section 4, Table 1)
and are not available here; these generators stand in for them with the
shapes, value distributions and structure described for each workload:

* ``random_banded``     -- rows with k distinct columns near the diagonal
                           (N(0,1) values) plus ``reg * e_j`` rows
                           (the tiny plain workload and the batched instances);
* ``grid_gradient``     -- forward-difference operator of a G x G grid with
                           weights 10^U(-2,2) plus ``reg * e_j`` rows, split
                           into P x P square patches;
* ``irregular_clustered`` -- geometric row lengths, clustered column indices,
                           column scaling 10^U(-3,3), BFS partition of the
                           A^T A graph.

The partition is an *input* of the method (Algorithm 1 takes the partition as
its first step; here it is supplied, not computed by the library), so the
partitioners live here too.  Nothing in this module computes any part of the
preconditioner.

All index arrays are int32, values float64, CSR rows have strictly increasing
column indices.  Random draws come from ``numpy.random.default_rng(seed)`` in a
fixed order, so a (function, arguments, seed) triple always yields the same
bytes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Problem:
    """One least-squares instance plus the parameters of its solve."""

    name: str
    m: int
    n: int
    indptr: np.ndarray      # int32 [m+1]
    indices: np.ndarray     # int32 [nnz]
    data: np.ndarray        # float64 [nnz]
    b: np.ndarray           # float64 [m]
    part: np.ndarray        # int32 [n], values in [0, nparts)
    nparts: int
    tau: float
    tol: float
    extra: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def scipy(self):
        """A as a ``scipy.sparse.csr_matrix`` (float64)."""
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr),
                             shape=(self.m, self.n))


# ---------------------------------------------------------------------------
# helpers (structure only)
# ---------------------------------------------------------------------------

def _csr_from_rows(row_of_entry: np.ndarray, cols: np.ndarray, vals: np.ndarray,
                   m: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Build CSR arrays from entries already grouped by row with sorted columns."""
    counts = np.bincount(row_of_entry, minlength=m).astype(np.int64)
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    assert indptr[-1] < 2**31
    return indptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def _distinct_rows(rng, row_len: np.ndarray, draw_cols) -> tuple[np.ndarray, np.ndarray]:
    """Draw column indices row by row and redraw repeated ones.

    ``draw_cols(row_ids) -> cols`` draws one column for each listed entry.  A
    column that repeats an earlier entry of the same row (after a stable sort
    by (row, column)) is redrawn, until every row holds distinct columns.
    Returns (row_of_entry, cols) with columns sorted inside each row.
    """
    nrows = row_len.shape[0]
    row_of_entry = np.repeat(np.arange(nrows, dtype=np.int64), row_len)
    cols = draw_cols(row_of_entry)
    n_big = np.int64(1) << 32
    while True:
        key = row_of_entry * n_big + cols
        order = np.argsort(key, kind="stable")
        sk = key[order]
        dup_sorted = np.zeros(sk.shape[0], dtype=bool)
        dup_sorted[1:] = sk[1:] == sk[:-1]
        if not dup_sorted.any():
            break
        dup_pos = np.sort(order[dup_sorted])
        cols[dup_pos] = draw_cols(row_of_entry[dup_pos])
    order = np.argsort(row_of_entry * n_big + cols, kind="stable")
    return row_of_entry[order], cols[order]


def _append_diag_rows(row_of_entry, cols, vals, m_rows: int, n: int, reg: float):
    """Append the n rows reg * e_j^T (j = 0..n-1) after the first m_rows rows."""
    row_of_entry = np.concatenate([row_of_entry, m_rows + np.arange(n, dtype=np.int64)])
    cols = np.concatenate([cols, np.arange(n, dtype=np.int64)])
    vals = np.concatenate([vals, np.full(n, reg, dtype=np.float64)])
    return row_of_entry, cols, vals, m_rows + n


def contiguous_partition(n: int, nparts: int) -> np.ndarray:
    """Column j belongs to part k when floor(k n / N) <= j < floor((k+1) n / N)."""
    bounds = (np.arange(nparts + 1, dtype=np.int64) * n) // nparts
    part = np.empty(n, dtype=np.int32)
    for k in range(nparts):
        part[bounds[k]:bounds[k + 1]] = k
    return part


def patch_partition(G: int, P: int) -> np.ndarray:
    """Square patches of a G x G grid, node (r, c) -> column G r + c.

    Patch boundaries are floor(k G / P); patch (p, q) gets id P p + q.
    """
    band = np.searchsorted((np.arange(1, P + 1, dtype=np.int64) * G) // P,
                           np.arange(G), side="right").astype(np.int32)
    return (band[:, None] * P + band[None, :]).reshape(-1).astype(np.int32)


def _ragged_gather(ptr: np.ndarray, data: np.ndarray, sel: np.ndarray) -> np.ndarray:
    """Concatenate data[ptr[s]:ptr[s+1]] for s in sel (vectorised)."""
    if sel.size == 0:
        return np.empty(0, dtype=data.dtype)
    starts = ptr[sel].astype(np.int64)
    lens = (ptr[sel + 1] - ptr[sel]).astype(np.int64)
    tot = int(lens.sum())
    if tot == 0:
        return np.empty(0, dtype=data.dtype)
    offs = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return data[np.arange(tot, dtype=np.int64) + offs]


def bfs_partition(indptr, indices, m: int, n: int, sizes: np.ndarray) -> np.ndarray:
    """Grow parts of the given sizes by breadth-first search on the graph of A^T A.

    Two columns are neighbours when some row of A stores both.  Part k starts
    at the lowest-index unassigned column, then adds whole BFS levels (each
    level in ascending column order) until it reaches its size; the last level
    is truncated.  A search that dies out restarts at the lowest-index
    unassigned column, still filling part k.
    """
    assert int(sizes.sum()) == n
    indptr = np.asarray(indptr, dtype=np.int64)
    indices = np.asarray(indices, dtype=np.int64)
    # column -> rows (transpose pattern)
    order = np.argsort(indices, kind="stable")
    rows_of = np.repeat(np.arange(m, dtype=np.int64), np.diff(indptr))[order]
    cptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(indices, minlength=n), out=cptr[1:])
    part = np.full(n, -1, dtype=np.int32)
    seed_ptr = 0
    for k, target in enumerate(sizes.tolist()):
        count = 0
        frontier = np.empty(0, dtype=np.int64)
        while count < target:
            if frontier.size == 0:
                while part[seed_ptr] >= 0:
                    seed_ptr += 1
                frontier = np.array([seed_ptr], dtype=np.int64)
                part[seed_ptr] = k
                count += 1
                continue
            rows = np.unique(_ragged_gather(cptr, rows_of, frontier))
            cols = np.unique(_ragged_gather(indptr, indices, rows))
            cols = cols[part[cols] < 0]
            take = cols[: target - count]
            part[take] = k
            count += take.size
            frontier = take
    assert (part >= 0).all()
    return part


# ---------------------------------------------------------------------------
# generators
# ---------------------------------------------------------------------------

def worked_example() -> Problem:
    """The 5 x 4 matrix of the paper's worked example (Section 3), 0-based.

    Subdomains: Omega_I1 = {1, 3}, Omega_I2 = {2, 4} in the paper's 1-based
    numbering, i.e. part = [0, 1, 0, 1].
    """
    dense = np.array([[1, 0, 6, 0],
                      [2, 4, 0, 0],
                      [3, 0, 0, 0],
                      [0, 5, 0, 7],
                      [0, 0, 0, 8]], dtype=np.float64)
    rows, cols = np.nonzero(dense)
    indptr, indices, data = _csr_from_rows(rows, cols, dense[rows, cols], 5)
    return Problem("worked_example", 5, 4, indptr, indices, data,
                   np.array([1.0, -1.0, 2.0, 0.5, -0.25]),
                   np.array([0, 1, 0, 1], dtype=np.int32), 2, 0.6, 1e-12)


def random_banded(n: int, m_rows: int, nparts: int, seed: int, tau: float = 0.1,
                  tol: float = 1e-8, k: int = 4, half_width: int = 20,
                  reg: float = 0.1, name: str = "random_banded") -> Problem:
    """Rows i < m_rows: k distinct columns floor(i n / m_rows) + U{-w..w}.

    Columns are clipped to [0, n-1]; repeats within a row are redrawn; values
    N(0,1) are drawn after all columns, in CSR order.  Then the n rows
    reg * e_j are appended and b ~ N(0,1) of length m_rows + n is drawn.
    The partition is contiguous with nparts parts.
    """
    rng = np.random.default_rng(seed)
    centre = (np.arange(m_rows, dtype=np.int64) * n) // m_rows

    def draw(rows):
        off = rng.integers(-half_width, half_width + 1, size=rows.shape[0])
        return np.clip(centre[rows] + off, 0, n - 1)

    row_of_entry, cols = _distinct_rows(rng, np.full(m_rows, k, dtype=np.int64), draw)
    vals = rng.standard_normal(cols.shape[0])
    row_of_entry, cols, vals, m = _append_diag_rows(row_of_entry, cols, vals, m_rows, n, reg)
    indptr, indices, data = _csr_from_rows(row_of_entry, cols, vals, m)
    b = rng.standard_normal(m)
    return Problem(name, m, n, indptr, indices, data, b,
                   contiguous_partition(n, nparts), nparts, tau, tol)


def grid_gradient(G: int, P: int, seed: int, tau: float = 0.1, tol: float = 1e-8,
                  reg: float = 1e-3, name: str = "grid_gradient") -> Problem:
    """Forward differences on a G x G grid plus reg * e_j rows.

    Node (r, c) is column G r + c.  Rows: every horizontal edge (r, c)-(r, c+1)
    in r-major order, then every vertical edge (r, c)-(r+1, c), each with -w at
    the tail and +w at the head, w = 10^U(-2,2); then the G^2 rows reg * e_j.
    b ~ N(0,1).  Partition: P x P square patches.
    """
    rng = np.random.default_rng(seed)
    n = G * G
    r, c = np.meshgrid(np.arange(G, dtype=np.int64), np.arange(G - 1, dtype=np.int64),
                       indexing="ij")
    h_tail = (G * r + c).reshape(-1)
    h_head = h_tail + 1
    r, c = np.meshgrid(np.arange(G - 1, dtype=np.int64), np.arange(G, dtype=np.int64),
                       indexing="ij")
    v_tail = (G * r + c).reshape(-1)
    v_head = v_tail + G
    tail = np.concatenate([h_tail, v_tail])
    head = np.concatenate([h_head, v_head])
    ne = tail.shape[0]
    w = 10.0 ** rng.uniform(-2.0, 2.0, size=ne)
    # tail < head always, so each row's columns are (tail, head) in order
    row_of_entry = np.repeat(np.arange(ne, dtype=np.int64), 2)
    cols = np.stack([tail, head], axis=1).reshape(-1)
    vals = np.stack([-w, w], axis=1).reshape(-1)
    row_of_entry, cols, vals, m = _append_diag_rows(row_of_entry, cols, vals, ne, n, reg)
    indptr, indices, data = _csr_from_rows(row_of_entry, cols, vals, m)
    b = rng.standard_normal(m)
    return Problem(name, m, n, indptr, indices, data, b,
                   patch_partition(G, P), P * P, tau, tol,
                   extra={"grid": G, "patches": P, "rng": rng})


def irregular_clustered(n: int, m_rows: int, nparts: int, seed: int, tau: float = 0.05,
                        tol: float = 1e-8, var: float = 2000.0, p_geom: float = 0.2,
                        kmax: int = 64, reg: float = 1e-4, size_lo: float = 500.0,
                        size_span: float = 2500.0, name: str = "irregular") -> Problem:
    """Irregular, badly scaled rows with a BFS partition of the A^T A graph.

    Row lengths k = min(1 + Geometric(p), kmax) (numpy's geometric has support
    >= 1, so k >= 2); a uniform cluster centre per row; columns are
    (centre + rint(N(0, var))) mod n with repeats redrawn; values N(0,1);
    column j is then scaled by 10^U(-3,3); n rows reg * e_j are appended and
    b ~ N(0,1).  Part sizes are size_lo + size_span * U, rescaled to sum to n
    (floored, the remainder added one by one to the first parts), and the
    parts are grown by ``bfs_partition``.
    """
    rng = np.random.default_rng(seed)
    klen = np.minimum(1 + rng.geometric(p_geom, size=m_rows), kmax).astype(np.int64)
    centre = rng.integers(0, n, size=m_rows)
    sd = math.sqrt(var)

    def draw(rows):
        off = np.rint(rng.normal(0.0, sd, size=rows.shape[0])).astype(np.int64)
        return (centre[rows] + off) % n

    row_of_entry, cols = _distinct_rows(rng, klen, draw)
    vals = rng.standard_normal(cols.shape[0])
    scale = 10.0 ** rng.uniform(-3.0, 3.0, size=n)
    vals = vals * scale[cols]
    row_of_entry, cols, vals, m = _append_diag_rows(row_of_entry, cols, vals, m_rows, n, reg)
    indptr, indices, data = _csr_from_rows(row_of_entry, cols, vals, m)
    b = rng.standard_normal(m)
    raw = size_lo + size_span * rng.uniform(size=nparts)
    sizes = np.floor(raw * n / raw.sum()).astype(np.int64)
    sizes[: n - int(sizes.sum())] += 1
    part = bfs_partition(indptr, indices, m, n, sizes)
    return Problem(name, m, n, indptr, indices, data, b, part, nparts, tau, tol)


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def banded_1000() -> Problem:
    """Tiny plain FP64 workload: 2000 random rows + 1000 rows 0.1 e_j, n = 1000,
    8 contiguous parts, tau = 0.1, tol 1e-8, seed 0."""
    return random_banded(1000, 2000, 8, seed=0, tau=0.1, tol=1e-8, name="banded_1000")


def grid_1000(G: int = 1000, P: int = 16) -> Problem:
    """Grid-gradient workload: 1000 x 1000 grid (n = 1e6, m = 2,998,000),
    16 x 16 = 256 square patches, tau = 0.1, seed 1."""
    return strip_rng(grid_gradient(G, P, seed=1, tau=0.1, tol=1e-8, name="grid_1000"))


def irregular_1m(n: int = 1_000_000, m_rows: int = 3_000_000, nparts: int = 512) -> Problem:
    """Ill-conditioned irregular workload: 3e6 random rows + 1e6 rows 1e-4 e_j,
    512 BFS parts, tau = 0.05, seed 2."""
    return irregular_clustered(n, m_rows, nparts, seed=2, tau=0.05, tol=1e-8, name="irregular_1m")


def banded_batch_64(count: int = 64, n_lo: float = 5e3, n_hi: float = 2e5) -> list[Problem]:
    """Batched workload: ``count`` independent random-banded instances.

    Instance j uses default_rng(3000 + j): n_j = round(exp U(ln n_lo, ln n_hi)),
    N_j = round(exp U(ln 8, ln 128)), then ``random_banded`` with 2 n_j random
    rows, seeded from the same generator stream.
    """
    probs = []
    for j in range(count):
        rng = np.random.default_rng(3000 + j)
        nj = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        Nj = int(round(math.exp(rng.uniform(math.log(8), math.log(128)))))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        probs.append(random_banded(nj, 2 * nj, Nj, seed=sub_seed, tau=0.1, tol=1e-8,
                                   name=f"banded_batch_64[{j}]"))
    return probs


def grid_500(G: int = 500, P: int = 16) -> Problem:
    """Differentiable workload: the grid generator at 500 x 500, tol 1e-10,
    seed 4; ``extra['x_star']`` ~ N(0,1) is drawn after b."""
    p = grid_gradient(G, P, seed=4, tau=0.1, tol=1e-10, name="grid_500")
    rng = p.extra.pop("rng")
    p.extra["x_star"] = rng.standard_normal(p.n)
    return p


def fd_entries(prob: Problem, count_b: int = 10, count_vals: int = 10,
               seed: int = 4001) -> tuple[np.ndarray, np.ndarray]:
    """Seeded entries for finite-difference checks: (indices into b, indices into vals)."""
    rng = np.random.default_rng(seed)
    ib = rng.choice(prob.m, size=count_b, replace=False)
    iv = rng.choice(prob.nnz, size=count_vals, replace=False)
    return ib.astype(np.int64), iv.astype(np.int64)


def small_config(kind: str, seed: int = 7) -> Problem:
    """Reduced-size versions of the workloads for parity tests the oracle can
    finish in seconds (several tiles per block, ragged tails)."""
    if kind == "banded":
        return random_banded(1000, 2000, 8, seed=seed, name="banded_small")
    if kind == "grid":
        p = grid_gradient(40, 4, seed=seed, name="grid_small")
        p.extra.pop("rng")
        return p
    if kind == "irregular":
        return irregular_clustered(6000, 18000, 6, seed=seed, size_lo=500, size_span=2500,
                                   var=400.0, name="irregular_small")
    raise ValueError(kind)


def strip_rng(p: Problem) -> Problem:
    p.extra.pop("rng", None)
    return p
