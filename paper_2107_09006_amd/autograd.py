"""``torch.autograd.Function`` around the library's solve and adjoint.

``LeastSquaresSolve.apply(vals, b, solver)`` returns x = argmin ||A x - b||
for A with the sparsity pattern held by ``solver`` and the values ``vals``;
its backward runs the library's adjoint (a second preconditioned solve with
the same setup) and returns dL/dvals and dL/db.  The preconditioner is built
from the values the solver was set up with; passing different values
re-runs the setup, since the preconditioner must match the operator.
"""
from __future__ import annotations

import torch

from .binding import Solver


class LeastSquaresSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals: torch.Tensor, b: torch.Tensor, solver: Solver):
        if not torch.equal(vals.detach(), solver.vals):
            raise ValueError("vals differ from the values the solver was set up with; "
                             "build a new Solver for new values")
        x, info, _ = solver.solve(b.detach().contiguous())
        ctx.solver = solver
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        dLdb, dLdv, _ = ctx.solver.backward(gx.detach().contiguous().to(torch.float64),
                                            want_b=ctx.needs_input_grad[1],
                                            want_vals=ctx.needs_input_grad[0])
        return dLdv, dLdb, None


def lstsq(vals: torch.Tensor, b: torch.Tensor, solver: Solver) -> torch.Tensor:
    """Differentiable x = argmin ||A(vals) x - b||_2 (two-level Schwarz PCG)."""
    return LeastSquaresSolve.apply(vals, b, solver)
