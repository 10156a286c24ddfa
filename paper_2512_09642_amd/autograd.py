"""Differentiable s-step CG solve.

Forward: x = A(k)^{-1} b with the library's s-step solver.  Backward, given
dL/dx: the adjoint system A^T lam = dL/dx is solved by the same s-step
iteration (A is symmetric), then dL/db = lam and dL/dk = -lam^T (dA/dk) x,
which the library scatters onto the operator's coefficients
(``sstep_grad_operator``: -lam_i x_j on a CSR pattern, -(lam_p - lam_q)(x_p - x_q)
on an interior face, -lam_p x_p on a boundary face).
"""
from __future__ import annotations

import torch

from .solver import Operator, Solver


def _load(solver: Solver, coeffs: torch.Tensor) -> object:
    """Loads ``coeffs`` into ``solver`` and returns the token that marks them
    as the solver's current coefficients."""
    op = solver.op
    if op.kind == 0:
        new = Operator.csr(op.row_ptr, op.col_idx, coeffs.detach())
    else:
        kx, ky, kz = op.split_faces(coeffs.detach())
        new = Operator.stencil(*op.dims, kx, ky, kz)
    solver.update_coefficients(new)
    token = object()
    solver.coeff_token = token
    return token


class SStepSolve(torch.autograd.Function):
    """``x = SStepSolve.apply(coeffs, b, solver, tol)``.

    ``coeffs`` holds the operator's coefficient values: the CSR ``val`` array
    or the concatenated face coefficients ``[kx | ky | kz]`` (device float64).
    They are loaded into ``solver`` before the solve, and again before the
    adjoint solve if the shared solver has been given other coefficients in
    between (several forwards before their backwards).  Returns x; gradients
    flow to ``coeffs`` and ``b``.
    """

    @staticmethod
    def forward(ctx, coeffs: torch.Tensor, b: torch.Tensor, solver: Solver, tol: float = 1e-8):
        token = _load(solver, coeffs)
        x, st = solver.solve(b.detach().contiguous(), None, tol)
        solver.last_forward_stats = st
        ctx.solver = solver
        ctx.tol = tol
        ctx.token = token
        # coeffs is saved so that backward solves the adjoint with the operator
        # of this forward (autograd raises if it is modified in place meanwhile)
        ctx.save_for_backward(x, coeffs)
        return x

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        x, coeffs = ctx.saved_tensors
        solver: Solver = ctx.solver
        if solver.coeff_token is not ctx.token:
            # another forward (or update_coefficients) has loaded other
            # coefficients into the shared solver since: reload this one's
            ctx.token = _load(solver, coeffs)
        lam, sta = solver.solve_adjoint(gx.detach().contiguous(), None, ctx.tol)
        solver.last_adjoint_stats = sta
        dcoef = solver.grad_operator(lam, x) if ctx.needs_input_grad[0] else None
        db = lam if ctx.needs_input_grad[1] else None
        return dcoef, db, None, None


def sstep_solve(coeffs: torch.Tensor, b: torch.Tensor, solver: Solver, tol: float = 1e-8) -> torch.Tensor:
    """Functional form of :class:`SStepSolve`."""
    return SStepSolve.apply(coeffs, b, solver, tol)
