"""Differentiable contact solve: torch.autograd.Function around fgmres_solve.

Forward: x = A(K)^-1 b with the block-AMG preconditioned FGMRES.
Backward (hand-written adjoint): A^T lam = dL/dx solved by FGMRES with the
transposed V-cycle on the same hierarchy; dL/db = lam and
dL/dK_ij = -lam_i x_j on K's stored entries (amg_grad_K).  Both solves and
the gradient sampling run in the HIP library.
"""
from __future__ import annotations

import torch

from .camg import AMGSolver


class ContactSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver: AMGSolver, K_val: torch.Tensor, b: torch.Tensor, rtol: float = 1e-10, m: int = 50):
        if K_val is not None:
            solver.update_fine_values(K_val=K_val.detach())
        x, info = solver.solve(b.detach(), rtol=rtol, m=m)
        if not info["converged"]:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.solver = solver
        ctx.rtol = rtol
        ctx.m = m
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        (x,) = ctx.saved_tensors
        solver = ctx.solver
        lam, info = solver.solve(gx.contiguous(), transpose=True, rtol=ctx.rtol, m=ctx.m)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        grad_K = solver.grad_K(lam, x) if ctx.needs_input_grad[1] else None
        grad_b = lam if ctx.needs_input_grad[2] else None
        return None, grad_K, grad_b, None, None


def contact_solve(solver: AMGSolver, K_val: torch.Tensor, b: torch.Tensor, rtol: float = 1e-10, m: int = 50):
    return ContactSolve.apply(solver, K_val, b, rtol, m)
