"""Pins of the plane (2D) oracle: the Q4 element, its assembled operator,
and the separable Gaussian filter (Sec. 5's filter), each checked against
something other than its own formula."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.operator import apply_K, apply_K_rows, assemble_K, jacobi_diag
from oracle.plane import (GAUSS_HALF, GAUSS_SIGMA, Grid2D, PlaneContext, gauss_weights_1d,
                          gaussian_filter_matrix, plane_stress_lame, q4_stiffness,
                          tip_deflection_timoshenko)
from oracle.density_filter import filter_forward, filter_transpose
from oracle.solve import krylov_step_ref, solve_direct


def _gauss_q4(E, nu):
    """2x2 Gauss quadrature of B^T D B on the unit square, plane stress D
    written from Hooke's law (independent of q4_stiffness)."""
    D = E / (1 - nu * nu) * np.array([[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]])
    pts = [0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)]
    K = np.zeros((8, 8))
    for x, y in itertools.product(pts, pts):
        B = np.zeros((3, 8))
        for a in range(4):
            ax, ay = a & 1, a >> 1
            # N_a = (ax ? x : 1 - x) (ay ? y : 1 - y)
            dNx = (1 if ax else -1) * (y if ay else 1 - y)
            dNy = (x if ax else 1 - x) * (1 if ay else -1)
            B[0, 2 * a] = dNx
            B[1, 2 * a + 1] = dNy
            B[2, 2 * a] = dNy
            B[2, 2 * a + 1] = dNx
        K += 0.25 * B.T @ D @ B
    return K


@pytest.mark.parametrize("nu", [0.3, 0.0, 0.45])
def test_q4_equals_gauss_quadrature(nu):
    assert np.max(np.abs(q4_stiffness(1.0, nu) - _gauss_q4(1.0, nu))) < 1e-15


def test_q4_symmetry_rigid_modes_rank():
    KE = q4_stiffness()
    assert np.array_equal(KE, KE.T)
    xy = [(a & 1, a >> 1) for a in range(4)]
    modes = [np.tile([1.0, 0.0], 4), np.tile([0.0, 1.0], 4),
             np.array([v for (x, y) in xy for v in (-y, x)], dtype=float)]
    for r in modes:
        assert np.max(np.abs(KE @ r)) < 1e-15
    ev = np.linalg.eigvalsh(KE)
    assert np.sum(ev > 1e-12) == 5 and np.all(ev > -1e-14)


def test_q4_uniform_strain_energy():
    """u = (exx x + g/2 y, eyy y + g/2 x): w_e = eps^T D eps (engineering
    shear g), area 1."""
    E, nu = 1.0, 0.3
    exx, eyy, g = 1e-3, -4e-4, 7e-4
    u = np.array([v for a in range(4) for (x, y) in [((a & 1), (a >> 1))]
                  for v in (exx * x + 0.5 * g * y, eyy * y + 0.5 * g * x)])
    eps = np.array([exx, eyy, g])
    D = E / (1 - nu * nu) * np.array([[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]])
    assert abs(u @ q4_stiffness(E, nu) @ u - eps @ D @ eps) < 1e-20
    lam, mu = plane_stress_lame(E, nu)
    assert abs(eps @ D @ eps - (lam * (exx + eyy) ** 2 + 2 * mu * (exx ** 2 + eyy ** 2) + mu * g * g)) < 1e-20


def test_plane_operator_rigid_modes_symmetry_and_element_loop():
    g = Grid2D(7, 5)
    rng = np.random.default_rng(0)
    s = rng.uniform(0.1, 1.0, g.E)
    KE = q4_stiffness()
    K = assemble_K(g, s, KE=KE)
    i, j = g.node_coords()
    for r in (np.stack([np.ones(g.N), np.zeros(g.N)], 1).ravel(),
              np.stack([np.zeros(g.N), np.ones(g.N)], 1).ravel(),
              np.stack([-j, i], 1).astype(float).ravel()):
        assert np.max(np.abs(K @ r)) < 1e-13
    assert abs(K - K.T).max() < 1e-16
    fixed = np.zeros(g.ndof, np.uint8)
    fixed[:2 * (g.nx + 1)] = 1
    u = rng.standard_normal(g.ndof)
    Kb = assemble_K(g, s, fixed, KE=KE)
    y_loop = apply_K(g, s, u, fixed, KE=KE)
    assert np.max(np.abs(Kb @ u - y_loop)) < 1e-13
    rows = apply_K_rows(g, s, u, [0, 9, 20, g.N - 1], fixed, KE=KE)
    for k, n in enumerate([0, 9, 20, g.N - 1]):
        assert np.max(np.abs(rows[k] - y_loop[2 * n:2 * n + 2])) < 1e-13
    assert np.max(np.abs(jacobi_diag(g, s, fixed, KE=KE) - Kb.diagonal())) < 1e-15


def test_plane_patch_test():
    """A linear displacement prescribed on the boundary of a uniform plate is
    reproduced exactly at every interior node."""
    g = Grid2D(6, 4)
    KE = q4_stiffness()
    s = np.ones(g.E)
    i, j = g.node_coords()
    exact = np.stack([1e-3 * i + 2e-4 * j, -5e-4 * j + 3e-4 * i], 1).ravel()
    bnd = (i == 0) | (i == g.nx) | (j == 0) | (j == g.ny)
    fixed = np.repeat(bnd, 2)
    K = assemble_K(g, s, KE=KE).tocsr()
    free = ~fixed
    rhs = -(K[free][:, fixed] @ exact[fixed])
    u = exact.copy()
    u[free] = spla.spsolve(K[free][:, free].tocsc(), rhs)
    assert np.max(np.abs(u - exact)) < 1e-15 * 1e3


def test_plane_cantilever_converges_to_timoshenko():
    """Solid cantilever L x h with a tip load spread over the end edge as a
    consistent (uniform) traction: the mean end deflection converges as h^2
    under refinement (Q4 with full integration is stiff in bending), and the
    Richardson-extrapolated value lies within 1% of Timoshenko's."""
    # same aspect ratio L/h = 8, element size halved twice (length units: elements)
    L_over_h = 8
    d = []
    for ny in (2, 4, 8):
        nx = L_over_h * ny
        g = Grid2D(nx, ny)
        KE = q4_stiffness()
        fixed = np.zeros(g.ndof, np.uint8)
        for j in range(ny + 1):
            fixed[2 * g.node(0, j):2 * g.node(0, j) + 2] = 1
        f = np.zeros(g.ndof)
        for j in range(ny + 1):
            f[2 * g.node(nx, j) + 1] = -(1.0 / ny) * (0.5 if j in (0, ny) else 1.0)
        u = solve_direct(assemble_K(g, np.ones(g.E), fixed, KE=KE), f)
        tip = -np.mean([u[2 * g.node(nx, j) + 1] for j in range(ny + 1)])
        d.append(tip / tip_deflection_timoshenko(nx, ny))
    e1, e2 = 1 - d[1], 1 - d[2]
    assert 0 < e2 < e1 and 3.0 < e1 / e2 < 5.0      # error falls about 4x per halving
    extrap = d[2] + (d[2] - d[1]) / 3.0
    assert abs(extrap - 1.0) < 0.01


def test_gaussian_filter_brute_force_and_separable():
    g = Grid2D(9, 6)
    H, Hs = gaussian_filter_matrix(g)
    w = gauss_weights_1d()
    ex, ey = g.elem_coords()
    x = np.random.default_rng(1).uniform(0.1, 1.0, g.E)
    # brute force over every pair of elements
    Hb = np.zeros((g.E, g.E))
    for e, j in itertools.product(range(g.E), range(g.E)):
        dx, dy = ex[j] - ex[e], ey[j] - ey[e]
        if abs(dx) <= GAUSS_HALF and abs(dy) <= GAUSS_HALF:
            Hb[e, j] = np.exp(-(dx * dx + dy * dy) / (2 * GAUSS_SIGMA ** 2))
    assert np.max(np.abs(H.toarray() - Hb)) < 1e-15
    # two normalised 1D passes (x, then y) give the same filter
    X = x.reshape(g.ny, g.nx)
    def pass1d(A, axis):
        out = np.zeros_like(A)
        n = A.shape[axis]
        for i in range(n):
            acc, ws = 0.0, 0.0
            for d in range(-GAUSS_HALF, GAUSS_HALF + 1):
                if 0 <= i + d < n:
                    acc = acc + w[d + GAUSS_HALF] * np.take(A, i + d, axis=axis)
                    ws += w[d + GAUSS_HALF]
            if axis == 1:
                out[:, i] = acc / ws
            else:
                out[i, :] = acc / ws
        return out
    sep = pass1d(pass1d(X, 1), 0).ravel()
    assert np.max(np.abs(filter_forward(H, Hs, x) - sep)) < 1e-15
    # constants kept, adjoint identity, full interior window
    assert np.max(np.abs(filter_forward(H, Hs, np.full(g.E, 0.3)) - 0.3)) < 1e-15
    gr = np.random.default_rng(2).standard_normal(g.E)
    assert abs(gr @ filter_forward(H, Hs, x) - x @ filter_transpose(H, Hs, gr)) < 1e-12
    big = Grid2D(9, 9)
    Hbig, _ = gaussian_filter_matrix(big)
    centre = 4 + 9 * 4
    assert Hbig[centre].nnz == 49
    assert abs(Hbig[centre].sum() - w.sum() ** 2) < 1e-14


def test_plane_krylov_step_solves_small_system():
    """Alg. 3's low-level step with D + 1 >= the number of free DOFs solves
    K u = f exactly (the Krylov space is the whole space)."""
    g = Grid2D(2, 1)
    fixed = np.zeros(g.ndof, np.uint8)
    for j in range(2):
        fixed[2 * g.node(0, j):2 * g.node(0, j) + 2] = 1
    f = np.zeros(g.ndof)
    f[2 * g.node(2, 1) + 1] = -1.0
    ctx = PlaneContext(2, 1, fixed)
    s = np.random.default_rng(3).uniform(0.2, 1.0, g.E)
    A = ctx.operator(s)
    K = assemble_K(g, s, fixed, KE=ctx.KE)
    u_ref = solve_direct(K, f)
    # the Krylov matrix of a distinct-eigenvalue system: degree = free DOFs - 1
    nfree = int((fixed == 0).sum())
    u, r = krylov_step_ref(A, f, np.zeros(g.ndof), nfree - 1)
    assert np.max(np.abs(u - u_ref)) < 1e-7 * np.max(np.abs(u_ref))
