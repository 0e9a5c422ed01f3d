"""Density-weighted stiffness operator K(rho) (oracle, FP64).

K(v) = sum_e A_e(v) K_e with the modified-SIMP activation
A_e = rho_min + (1 - rho_min) rho_e^p: the paper's power law v^eta
(Sec. 3, stiffness laws) kept strictly positive so that the spectrum bound
(Eq. KVBound) holds; any smooth positive activation is admitted by the
Remark on activations in Sec. 3.

Supports: a fixed DOF gets an identity row and column (its value is
prescribed to 0 by the load vector and the initial guess); springs add k to
the diagonal of free DOFs.  In matrix form
    K_bc = P (sum_e s_e P_e^T KE P_e + S) P + (I - P),   P = diag(free).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .element import element_stiffness
from .grid import Grid


def simp_scale(rho, penal=3.0, rho_min=1e-3):
    """s_e = rho_min + (1 - rho_min) rho_e^p."""
    rho = np.asarray(rho, dtype=np.float64)
    return rho_min + (1.0 - rho_min) * rho ** penal


def simp_dscale(rho, penal=3.0, rho_min=1e-3):
    """ds_e / d rho_e = p (1 - rho_min) rho_e^(p - 1)."""
    rho = np.asarray(rho, dtype=np.float64)
    return penal * (1.0 - rho_min) * rho ** (penal - 1.0)


def _springs(springs):
    if springs is None or len(springs) == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    if isinstance(springs, tuple) and len(springs) == 2 and isinstance(springs[0], np.ndarray):
        return springs
    dof = np.array([s[0] for s in springs], dtype=np.int64)
    k = np.array([s[1] for s in springs], dtype=np.float64)
    return dof, k


def assemble_K(grid: Grid, s, fixed_mask=None, springs=None, KE=None) -> sp.csr_matrix:
    """Assembled sparse K_bc (CSR), summing element matrices by COO duplicates."""
    KE = element_stiffness() if KE is None else KE
    s = np.asarray(s, dtype=np.float64)
    edof = grid.elem_dofs()
    nloc = edof.shape[1]  # 24 (hex8) or 8 (Q4)
    rows = np.repeat(edof, nloc, axis=1).ravel()
    cols = np.tile(edof, (1, nloc)).ravel()
    vals = (s[:, None, None] * KE[None, :, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(grid.ndof, grid.ndof)).tocsr()
    dof, k = _springs(springs)
    if dof.size:
        K = K + sp.csr_matrix((k, (dof, dof)), shape=K.shape)
    if fixed_mask is not None:
        free = (np.asarray(fixed_mask) == 0).astype(np.float64)
        P = sp.diags(free)
        K = (P @ K @ P + sp.diags(1.0 - free)).tocsr()
    K.sum_duplicates()
    return K


def apply_K(grid: Grid, s, u, fixed_mask=None, springs=None, KE=None, chunk=1 << 16):
    """y = K_bc u by the element loop  y += P_e^T (s_e KE P_e u)  (no matrix
    stored).  u may be [ndof] or [nrhs][ndof]."""
    KE = element_stiffness() if KE is None else KE
    s = np.asarray(s, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    squeeze = u.ndim == 1
    U = u[None, :] if squeeze else u
    free = None
    if fixed_mask is not None:
        free = np.asarray(fixed_mask) == 0
        U = np.where(free[None, :], U, 0.0)
    Y = np.zeros_like(U)
    for e0 in range(0, grid.E, chunk):
        e = np.arange(e0, min(grid.E, e0 + chunk))
        edof = grid.elem_dofs(e)
        for r in range(U.shape[0]):
            ue = U[r][edof]                              # [chunk, 24]
            ye = s[e][:, None] * (ue @ KE.T)
            Y[r] += np.bincount(edof.ravel(), weights=ye.ravel(), minlength=grid.ndof)
    dof, k = _springs(springs)
    if dof.size:
        Y[:, dof] += k[None, :] * U[:, dof]
    if free is not None:
        uo = u[None, :] if squeeze else u
        Y = np.where(free[None, :], Y, uo)
    return Y[0] if squeeze else Y


def apply_K_rows(grid: Grid, s, u, nodes, fixed_mask=None, springs=None, KE=None):
    """Rows of K_bc u at the given nodes, each summed from its incident
    elements one by one (for sampled checks on grids too large to assemble).
    Returns [len(nodes), d] (single right-hand side; d = 3, or 2 on a
    plane grid)."""
    KE = element_stiffness() if KE is None else KE
    d_n = getattr(grid, "dim", 3)
    s = np.asarray(s, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    free = None if fixed_mask is None else (np.asarray(fixed_mask) == 0)
    dof, k = _springs(springs)
    spring = dict(zip(dof.tolist(), k.tolist()))
    out = np.zeros((len(nodes), d_n))
    for r, n in enumerate(nodes):
        acc = np.zeros(d_n)
        for e, a in grid.node_elems(int(n)):
            edof = grid.elem_dofs([e])[0]
            ue = u[edof] if free is None else np.where(free[edof], u[edof], 0.0)
            acc += s[e] * (KE[d_n * a:d_n * a + d_n, :] @ ue)
        for c in range(d_n):
            d = d_n * int(n) + c
            if d in spring and (free is None or free[d]):
                acc[c] += spring[d] * u[d]
            if free is not None and not free[d]:
                acc[c] = u[d]
        out[r] = acc
    return out


def jacobi_diag(grid: Grid, s, fixed_mask=None, springs=None, KE=None):
    """diag(K_bc), summed element by element from diag(KE)."""
    KE = element_stiffness() if KE is None else KE
    s = np.asarray(s, dtype=np.float64)
    edof = grid.elem_dofs()
    d = np.bincount(edof.ravel(), weights=(s[:, None] * np.diag(KE)[None, :]).ravel(),
                    minlength=grid.ndof)
    dof, k = _springs(springs)
    if dof.size:
        d[dof] += k
    if fixed_mask is not None:
        d = np.where(np.asarray(fixed_mask) == 0, d, 1.0)
    return d
