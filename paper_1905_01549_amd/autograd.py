"""Differentiable sparse solve: x = A(values)^{-1} b with gradients from an
adjoint solve instead of unrolled iterations.

For a loss L(x), with A symmetric (A^T = A), the backward pass solves
A lambda = dL/dx with the same CG variant and returns

    dL/db      = lambda
    dL/dA_e    = -lambda[row(e)] * x[col(e)]   for every stored entry e,

treating each stored entry as an independent parameter (both halves of a
symmetric pair receive their own term).  Both steps run in libprcg
(`prcg_adjoint`: the CG solve and the sparse outer-product kernel).
"""
from __future__ import annotations

import torch

from .prcg import Matrix


class SolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, b, matrix: Matrix, variant: str = "pr", tol: float = 1e-10, maxit: int = 10000):
        matrix.set_values(values)
        x, info = matrix.solve(b, variant, tol, maxit)
        if info.status != "ok":
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.save_for_backward(values, x)
        ctx.matrix, ctx.variant, ctx.tol, ctx.maxit = matrix, variant, tol, maxit
        ctx.last_info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        values, x = ctx.saved_tensors
        m = ctx.matrix
        m.set_values(values)  # the handle may have been reused since the forward pass
        gb, gv, info = m.adjoint(x, gx.contiguous(), ctx.variant, ctx.tol, ctx.maxit,
                                 want_b=ctx.needs_input_grad[1], want_values=ctx.needs_input_grad[0])
        if info.status != "ok":
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        return gv, gb, None, None, None, None


def solve(values: torch.Tensor, b: torch.Tensor, matrix: Matrix, variant: str = "pr", tol: float = 1e-10,
          maxit: int = 10000) -> torch.Tensor:
    """x = A^{-1} b for A with `matrix`'s sparsity pattern and the given values."""
    return SolveFn.apply(values, b, matrix, variant, tol, maxit)
