"""MI355X (gfx950) two-level Schwarz preconditioned Krylov solvers for sparse least squares.

The compute path is the HIP library ``liblsq2l.so`` (C ABI in
``include/lsq2l.h``); ``binding`` marshals PyTorch device tensors into it and
``autograd`` wraps solve/backward as a ``torch.autograd.Function``.
"""
from .binding import (  # noqa: F401
    Solver, solver_from_problem, load_library, default_options, release_cache, transpose,
    Lsq2lError, OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, CHOL_BREAKDOWN, PCG_BREAKDOWN,
    FP64, MIXED, ADDITIVE, ONE_LEVEL, BALANCED, RAS, DEFLATED, PCG, LSQR, GMRES, EXPORTS,
    ORDER_AUTO, ORDER_SPLIT, ORDER_GLOBAL, FACTOR_CHOLESKY, FACTOR_QR,
)
from .autograd import LeastSquaresSolve, lstsq  # noqa: F401,E402
