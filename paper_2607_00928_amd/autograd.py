"""Differentiable least-squares inverse NUDFT.

``lsq_solve(f, points, nx, ny)`` returns c = argmin ||A(points) c - f||_2 as a
complex128 (nx, ny) tensor and supports backward to f and to the point
coordinates.  Forward and backward both run in the library (nudft2_solve with
normal-equation refinement, nudft2_lsq_backward); this module only passes
tensors.  The plan (with its HSS factors) is kept from the forward pass and
reused by the backward pass instead of storing intermediate iterates.
"""
from __future__ import annotations

import torch

from . import Plan

__all__ = ["lsq_solve"]


class _LsqSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, points, nx, ny, precision, eps, ir_tol, ir_maxit):
        plan = Plan(points.detach(), nx, ny, precision=precision, eps=eps, ir_tol=ir_tol,
                    ir_maxit=ir_maxit, refine=1)
        plan.factor()
        fd = f.detach().contiguous()
        c = plan.solve(fd)
        ctx.plan = plan
        ctx.points_device = points.device
        ctx.save_for_backward(fd, c)
        return c

    @staticmethod
    def backward(ctx, grad_c):
        fd, c = ctx.saved_tensors
        plan = ctx.plan
        need_pts = ctx.needs_input_grad[1]
        g = grad_c.detach().to(torch.complex128).contiguous()
        gf, gp = plan.lsq_backward(fd, c, g, points_grad=need_pts)
        ctx.plan = None
        plan.close()
        gpts = gp.to(ctx.points_device) if gp is not None else None
        return (gf if ctx.needs_input_grad[0] else None), gpts, None, None, None, None, None, None


def lsq_solve(f: torch.Tensor, points: torch.Tensor, nx: int, ny: int, *, precision="fp32",
              eps=1e-2, ir_tol=1e-13, ir_maxit=60) -> torch.Tensor:
    """c(f, points) = argmin_c ||A(points) c - f||_2, differentiable in f and
    points.  f: complex128 CUDA tensor (M,); points: float64 tensor (M, 2)."""
    return _LsqSolve.apply(f, points, int(nx), int(ny), precision, float(eps), float(ir_tol),
                           int(ir_maxit))
