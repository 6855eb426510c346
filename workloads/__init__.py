"""Seeded synthetic least-squares workloads.

This package only draws inputs (a sparse matrix A in CSR form, a right-hand
side b, a column partition and the solver parameters).  It contains none of
the preconditioner's arithmetic, so both the CPU oracle and the GPU library
can be driven by the same data without sharing any solver code.
"""
from .generators import (  # noqa: F401
    Problem,
    worked_example,
    random_banded,
    grid_gradient,
    irregular_clustered,
    banded_1000,
    grid_1000,
    irregular_1m,
    banded_batch_64,
    grid_500,
    small_config,
    fd_entries,
)
