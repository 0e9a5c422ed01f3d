"""Linear density filter (oracle, FP64).

The Remark on modifiers in Sec. 3 admits a smooth convolution C inside the
activation, K(v) = sum_e A_e(C(v)) K_e.  The experiments (Sec. 5) use a 7x7
separable Gaussian; the workloads here use the linear "cone" filter
    rho_e = sum_j H_ej x_j / Hs_e,  H_ej = max(0, r - |c_e - c_j|),
    Hs_e = sum_j H_ej,
over element centres, truncated at the grid boundary (no padding).  Its
transpose maps a gradient w.r.t. rho to one w.r.t. x:
    g_x = H^T (g_rho / Hs).
H is built here by plain neighbour enumeration as a sparse matrix.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

from .grid import Grid


def stencil_offsets(radius: float):
    """Integer offsets d with |d| < r (the cone weight r - |d| is positive)."""
    R = int(math.ceil(radius)) - 1
    out = []
    for dz, dy, dx in itertools.product(range(-R, R + 1), repeat=3):
        dist = math.sqrt(dx * dx + dy * dy + dz * dz)
        if radius - dist > 0.0:
            out.append((dx, dy, dz, radius - dist))
    return out


def cone_filter_matrix(grid: Grid, radius: float):
    """(H, Hs): sparse H [E, E] and row sums Hs [E]."""
    ex, ey, ez = grid.elem_coords()
    rows, cols, vals = [], [], []
    e = np.arange(grid.E)
    for dx, dy, dz, w in stencil_offsets(radius):
        jx, jy, jz = ex + dx, ey + dy, ez + dz
        ok = (jx >= 0) & (jx < grid.nx) & (jy >= 0) & (jy < grid.ny) & (jz >= 0) & (jz < grid.nz)
        rows.append(e[ok])
        cols.append((jx + grid.nx * (jy + grid.ny * jz))[ok])
        vals.append(np.full(int(ok.sum()), w))
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(grid.E, grid.E))
    Hs = np.asarray(H.sum(axis=1)).ravel()
    return H, Hs


def filter_forward(H, Hs, x):
    """rho = (H x) / Hs."""
    return (H @ np.asarray(x, dtype=np.float64)) / Hs


def filter_transpose(H, Hs, g):
    """g_x = H^T (g / Hs)."""
    return H.T @ (np.asarray(g, dtype=np.float64) / Hs)


def _neighbours(grid: Grid, elems, dx, dy, dz):
    """Index of element e + (dx, dy, dz) for each e in elems, and whether it
    lies inside the grid."""
    ex, ey, ez = grid.elem_coords(np.asarray(elems))
    jx, jy, jz = ex + dx, ey + dy, ez + dz
    ok = (jx >= 0) & (jx < grid.nx) & (jy >= 0) & (jy < grid.ny) & (jz >= 0) & (jz < grid.nz)
    j = np.where(ok, jx + grid.nx * (jy + grid.ny * jz), 0)
    return j, ok


def filter_weight_sums_at(grid: Grid, radius: float, elems):
    """Hs_e for the given elements, summed over the stencil one offset at a
    time (for sampled checks on grids too large for the matrix)."""
    hs = np.zeros(len(elems))
    for dx, dy, dz, w in stencil_offsets(radius):
        _, ok = _neighbours(grid, elems, dx, dy, dz)
        hs += np.where(ok, w, 0.0)
    return hs


def filter_forward_at(grid: Grid, radius: float, x, elems):
    """rho_e = sum_j H_ej x_j / Hs_e at the given elements."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros(len(elems))
    for dx, dy, dz, w in stencil_offsets(radius):
        j, ok = _neighbours(grid, elems, dx, dy, dz)
        acc += np.where(ok, w * x[j], 0.0)
    return acc / filter_weight_sums_at(grid, radius, elems)


def filter_transpose_at(grid: Grid, radius: float, g, elems):
    """g_x[j] = sum_e H_ej g_e / Hs_e at the given elements j (H is
    symmetric: the cone weight depends on the distance only)."""
    g = np.asarray(g, dtype=np.float64)
    acc = np.zeros(len(elems))
    for dx, dy, dz, w in stencil_offsets(radius):
        e, ok = _neighbours(grid, elems, dx, dy, dz)
        hs = filter_weight_sums_at(grid, radius, e)
        acc += np.where(ok, w * g[e] / hs, 0.0)
    return acc
