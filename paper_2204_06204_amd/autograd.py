"""Differentiable displacement solve with a hand-written adjoint.

The sensitivity of Sec. 3 is the adjoint formula for the self-adjoint
compliance (grad l = -1/2 u^T dK/dv u).  For a general objective L(u) the
chain rule needs one adjoint solve K lambda = dL/du (K is symmetric), then
    dL/drho_e = -ds_e lambda_e^T KE u_e,   dL/dx = C^T (dL/drho),
with C the density filter.  Both solves and the bilinear element pass run in
libfbto.so; element strains are recomputed from the nodal vectors, nothing
per element is stored between forward and backward.

Precision: float64 designs use the mixed solve (FP32 Jacobi-PCG inner
iterations, FP64 residual refinement) to `rtol`; float32 designs use FP32
Jacobi-PCG to `rtol`.
"""
from __future__ import annotations

import torch

from .grid import Grid


def _solve(grid: Grid, rho: torch.Tensor, rhs: torch.Tensor, rtol: float, max_steps: int) -> torch.Tensor:
    u = torch.zeros_like(rhs)
    if rhs.dtype == torch.float64:
        grid.solve_refined(rho, rhs.contiguous(), u, rtol, max_refine=100, inner_steps=max_steps,
                           inner_dtype=torch.float32, inner_rtol=1e-3)
    else:
        grid.inner_solve(rho, rhs.contiguous(), u, max_steps, rtol=rtol)
    return u


class DisplacementSolve(torch.autograd.Function):
    """u = K(C(x))^{-1} f, differentiable in the design x."""

    @staticmethod
    def forward(ctx, x, grid: Grid, f, rtol: float = 1e-10, max_steps: int = 200000):
        rho = grid.filter(x.contiguous())
        u = _solve(grid, rho, f, rtol, max_steps)
        ctx.grid, ctx.rtol, ctx.max_steps = grid, rtol, max_steps
        ctx.save_for_backward(rho, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        rho, u = ctx.saved_tensors
        grid = ctx.grid
        lam = _solve(grid, rho, grad_u.contiguous(), ctx.rtol, ctx.max_steps)   # adjoint solve
        drho = grid.sensitivity(rho, u, lam=lam)                             # -ds lam^T KE u
        dx = grid.filter(drho, transpose=True)
        return dx, None, None, None, None


class Compliance(torch.autograd.Function):
    """c = f^T K(C(x))^{-1} f (summed over load cases).  Self-adjoint: the
    backward pass reuses u as the adjoint, no second solve."""

    @staticmethod
    def forward(ctx, x, grid: Grid, f, rtol: float = 1e-10, max_steps: int = 200000):
        rho = grid.filter(x.contiguous())
        u = _solve(grid, rho, f, rtol, max_steps)
        obj = torch.zeros(1, dtype=torch.float64, device=x.device)
        grid.sensitivity(rho, u, f=f, obj=obj, dobj=torch.empty_like(rho))
        ctx.grid = grid
        ctx.save_for_backward(rho, u)
        return obj[0].to(x.dtype)

    @staticmethod
    def backward(ctx, grad_c):
        rho, u = ctx.saved_tensors
        grid = ctx.grid
        drho = grid.sensitivity(rho, u)                                      # -ds u^T KE u
        dx = grid.filter(drho, transpose=True)
        return dx * grad_c.to(dx.dtype), None, None, None, None


def displacement(x, grid: Grid, f, rtol: float = 1e-10, max_steps: int = 200000):
    return DisplacementSolve.apply(x, grid, f, rtol, max_steps)


def compliance(x, grid: Grid, f, rtol: float = 1e-10, max_steps: int = 200000):
    return Compliance.apply(x, grid, f, rtol, max_steps)


def target_displacement(x, grid: Grid, f, target: torch.Tensor, rtol: float = 1e-10,
                        max_steps: int = 200000):
    """L = target . u  (e.g. -u_z at an output node of a compliant mechanism);
    its gradient takes the true adjoint solve K lambda = target."""
    u = displacement(x, grid, f, rtol, max_steps)
    return torch.dot(target, u)
