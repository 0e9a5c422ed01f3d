"""Sensitivities (oracle, FP64).

Sec. 3 gives the exact gradient of the compliance objective,
grad l = -1/2 u^T (dK/dv) u, and Alg. 1 uses the same expression with the
inexact displacement u_k.  For K = P (sum_e s_e P_e^T KE P_e) P + ...,
dK/drho_e = ds_e P P_e^T KE P_e P, so for c = f^T u (= 2 l):
    dc/drho_e = -ds_e w_e,   w_e = (P u)_e^T KE (P u)_e.
A linear functional L = t^T u (e.g. a target displacement) needs the adjoint
lambda = K^{-1} t (K symmetric):  dL/drho_e = -ds_e lambda_e^T KE u_e.
With several load cases the objective and gradient are summed.
"""
from __future__ import annotations

import numpy as np

from .element import element_stiffness
from .grid import Grid
from .operator import simp_dscale


def _masked(u, fixed_mask):
    u = np.asarray(u, dtype=np.float64)
    if fixed_mask is None:
        return u
    return np.where(np.asarray(fixed_mask) == 0, u, 0.0)


def element_bilinear(grid: Grid, lam, u, fixed_mask=None, KE=None, chunk=1 << 16):
    """b_e = lambda_e^T KE u_e for every element (u, lambda: [ndof] or
    [nrhs][ndof]; summed over right-hand sides)."""
    KE = element_stiffness() if KE is None else KE
    U = np.atleast_2d(_masked(u, fixed_mask))
    L = np.atleast_2d(_masked(lam, fixed_mask))
    out = np.zeros(grid.E)
    for e0 in range(0, grid.E, chunk):
        e = np.arange(e0, min(grid.E, e0 + chunk))
        edof = grid.elem_dofs(e)
        for r in range(U.shape[0]):
            ue, le = U[r][edof], L[r][edof]
            out[e] += np.einsum("ei,ij,ej->e", le, KE, ue)
    return out


def element_bilinear_at(grid: Grid, lam, u, elems, fixed_mask=None, KE=None):
    """b_e = lambda_e^T KE u_e at the given elements only (for sampled checks
    on grids too large for the full pass)."""
    KE = element_stiffness() if KE is None else KE
    U = np.atleast_2d(_masked(u, fixed_mask))
    L = np.atleast_2d(_masked(lam, fixed_mask))
    edof = grid.elem_dofs(np.asarray(elems))
    out = np.zeros(len(elems))
    for r in range(U.shape[0]):
        out += np.einsum("ei,ij,ej->e", L[r][edof], KE, U[r][edof])
    return out


def element_energy(grid: Grid, u, fixed_mask=None, KE=None):
    """w_e = u_e^T KE u_e."""
    return element_bilinear(grid, u, u, fixed_mask, KE)


def compliance_gradient(grid: Grid, rho_phys, u, fixed_mask=None, penal=3.0,
                        rho_min=1e-3, KE=None):
    """dc/drho_phys for c = sum_r f_r^T u_r."""
    return -simp_dscale(rho_phys, penal, rho_min) * element_energy(grid, u, fixed_mask, KE)


def adjoint_gradient(grid: Grid, rho_phys, u, lam, fixed_mask=None, penal=3.0,
                     rho_min=1e-3, KE=None):
    """dL/drho_phys for L = t^T u with adjoint lam = K^{-1} t."""
    return -simp_dscale(rho_phys, penal, rho_min) * element_bilinear(grid, lam, u, fixed_mask, KE)
