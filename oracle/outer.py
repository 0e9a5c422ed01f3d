"""One outer (design) iteration of the first-order bilevel method (oracle).

Alg. 1 alternates one low-level refinement of u with one projected
gradient step on the design using the inexact displacement.  Order used
here (the text of Sec. 4 uses the inexact result *after* the low-level
step for the sensitivity):
  1. rho = C(x)                      density filter (Remark, Sec. 3)
  2. s, ds, diag(K) from rho          modified SIMP (Sec. 3)
  3. u <- m Jacobi-PCG steps from u   low-level refinement (Alg. 1 / 3);
     or, for Alg. 3 (CPFBTO), one step with the Krylov preconditioner of
     Eq. LSP (low_level=("krylov", D, beta))
  4. c = f^T u,  g_rho = -ds w        approximate sensitivity (Alg. 1)
  5. g_x = C^T g_rho
  6. g_x <- g_x - mean(g_x)           mean-projected gradient (Sec. 4.2)
  7. y = x - alpha_k * g_x / 2,  alpha_k = alpha0 k^(-3/4)   (Sec. 5)
     (the paper's objective is l = c/2, so its gradient is g_x / 2)
  8. x <- Proj_X(y)                   Sec. 4.2, Eq. piecewiseLinearEQ
  9. metrics ||x_new - x||_inf, ||r||_inf (recursive residual), c (Sec. 5)
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .density_filter import cone_filter_matrix, filter_forward, filter_transpose
from .element import element_stiffness
from .grid import Grid
from .operator import apply_K, assemble_K, jacobi_diag, simp_dscale, simp_scale
from .projection import project_volume_ref
from .sensitivity import element_energy
from .solve import krylov_step_ref, pcg_ref, solve_direct


def step_size(alpha0: float, k: int) -> float:
    """alpha_k = alpha0 * k^(-3/4) (Sec. 5; the decay exponent satisfies the
    step-size assumptions of Thm. 1)."""
    return alpha0 * float(k) ** (-0.75)


@dataclasses.dataclass
class OuterRecord:
    k: int
    compliance: float
    dx_inf: float
    r_inf: float
    lam: float
    volume: float


class OuterContext:
    """Grid, element matrix and filter matrix of a problem, built once."""

    def __init__(self, nx, ny, nz, filter_radius, fixed_mask, springs=(), young=1.0,
                 poisson=0.3, penal=3.0, rho_min=1e-3, use_csr=None):
        self.grid = Grid(nx, ny, nz)
        self.KE = element_stiffness(young, poisson)
        self.H, self.Hs = cone_filter_matrix(self.grid, filter_radius)
        self.fixed = np.asarray(fixed_mask, dtype=np.uint8)
        self.springs = springs
        self.penal, self.rho_min = penal, rho_min
        self.use_csr = (self.grid.E <= 70000) if use_csr is None else use_csr

    def operator(self, s):
        if self.use_csr:
            K = assemble_K(self.grid, s, self.fixed, self.springs, self.KE)
            return lambda v: K @ v
        return lambda v: apply_K(self.grid, s, v, self.fixed, self.springs, self.KE)


def outer_step_ref(ctx: OuterContext, x, u, f, k, alpha0, inner_steps, lo, hi, vmax,
                   mean_project=True, low_level=None):
    """Returns (x_new, u_new, OuterRecord, g_x).  low_level=None runs
    `inner_steps` Jacobi-PCG steps; ("krylov", D, beta) runs Alg. 3's one
    preconditioned step u <- u - beta M^-1 (K u - f) (r_inf is then the true
    residual after the step); ("exact",) solves K u = f directly (sparse LU),
    the projected-gradient-descent baseline."""
    g = ctx.grid
    rho = filter_forward(ctx.H, ctx.Hs, x)
    s = simp_scale(rho, ctx.penal, ctx.rho_min)
    ds = simp_dscale(rho, ctx.penal, ctx.rho_min)
    D = jacobi_diag(g, s, ctx.fixed, ctx.springs, ctx.KE)
    A = ctx.operator(s)
    F = np.atleast_2d(f)
    U = np.array(np.atleast_2d(u), dtype=np.float64, copy=True)
    r_inf = 0.0
    if low_level is not None and low_level[0] == "exact":
        Kx = assemble_K(g, s, ctx.fixed, ctx.springs, ctx.KE)
    for r in range(F.shape[0]):
        if low_level is None:
            U[r], res = pcg_ref(A, D, F[r], U[r], inner_steps)
        elif low_level[0] == "exact":
            U[r] = solve_direct(Kx, F[r])
            res = F[r] - Kx @ U[r]
        else:
            _, deg, beta = low_level
            U[r], res = krylov_step_ref(A, F[r], U[r], deg, beta)
        r_inf = max(r_inf, float(np.abs(res).max()))
    c = float(sum(F[r] @ U[r] for r in range(F.shape[0])))
    g_rho = -ds * element_energy(g, U, ctx.fixed, ctx.KE)
    g_x = filter_transpose(ctx.H, ctx.Hs, g_rho)
    if mean_project:
        g_x = g_x - g_x.mean()
    y = x - step_size(alpha0, k) * 0.5 * g_x
    x_new, lam = project_volume_ref(y, lo, hi, vmax, return_lambda=True)
    rec = OuterRecord(k=k, compliance=c, dx_inf=float(np.abs(x_new - x).max()),
                      r_inf=r_inf, lam=float(lam), volume=float(x_new.sum()))
    return x_new, (U if np.ndim(u) == 2 else U[0]), rec, g_x


def run_outer_ref(ctx: OuterContext, x_init, f, iters, alpha0, inner_steps, lo, hi, vmax,
                  mean_project=True, u0=None, low_level=None):
    """x_0 = Proj_X(x_init), u_0 = 0 (or u0); then `iters` outer steps."""
    x = project_volume_ref(np.asarray(x_init, dtype=np.float64), lo, hi, vmax)
    F = np.atleast_2d(f)
    u = np.zeros_like(F) if u0 is None else np.array(u0, dtype=np.float64)
    recs, xs = [], [x.copy()]
    for k in range(1, iters + 1):
        x, u, rec, _ = outer_step_ref(ctx, x, u, F, k, alpha0, inner_steps, lo, hi, vmax,
                                      mean_project, low_level)
        recs.append(rec)
        xs.append(x.copy())
    return x, u, recs, xs


def default_alpha0(ctx: OuterContext, x_init, f, inner_steps, lo, hi, vmax,
                   max_move=0.2, mean_project=True, low_level=None):
    """Step-size reading: alpha0 such that the first step moves no density
    by more than `max_move`:  alpha0 = max_move / max|g_P(x_1) / 2|
    (low_level as in outer_step_ref)."""
    x = project_volume_ref(np.asarray(x_init, dtype=np.float64), lo, hi, vmax)
    F = np.atleast_2d(f)
    _, _, _, g_x = outer_step_ref(ctx, x, np.zeros_like(F), F, 1, 0.0, inner_steps, lo, hi,
                                  vmax, mean_project, low_level)
    return max_move / float(np.abs(0.5 * g_x).max())


def true_objective(ctx: OuterContext, x, f):
    """The objective at a design with the low-level problem solved exactly
    (Sec. 3, Eq. opt; Sec. 5 tracks it as l(v_k)):
        l(x) = 1/2 sum_r f_r^T K(rho(x))^-1 f_r   (half the compliance),
    and its gradient with respect to the design, through the filter:
        grad l = 1/2 C^T(-ds_e u_e^T KE u_e)  with u_r = K^-1 f_r.
    Returns (l, grad_l, U) from direct sparse solves."""
    g = ctx.grid
    rho = filter_forward(ctx.H, ctx.Hs, x)
    s = simp_scale(rho, ctx.penal, ctx.rho_min)
    ds = simp_dscale(rho, ctx.penal, ctx.rho_min)
    K = assemble_K(g, s, ctx.fixed, ctx.springs, ctx.KE)
    F = np.atleast_2d(f)
    U = np.stack([solve_direct(K, F[r]) for r in range(F.shape[0])])
    l = 0.5 * float(sum(F[r] @ U[r] for r in range(F.shape[0])))
    grad = 0.5 * filter_transpose(ctx.H, ctx.Hs, -ds * element_energy(g, U, ctx.fixed, ctx.KE))
    return l, grad, U


def relative_projection_error(x, grad, alpha, lo, hi, vmax):
    """Delta^v = || Proj_X(x - alpha grad) - x ||^2 / alpha^2, the high-level
    optimality measure of Sec. 4 (defined after Thm. 1): zero exactly when x
    satisfies the first-order conditions on X."""
    z = project_volume_ref(np.asarray(x, dtype=np.float64) - alpha * np.asarray(grad), lo, hi, vmax)
    return float(((z - x) ** 2).sum()) / (alpha * alpha)
