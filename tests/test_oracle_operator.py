"""Pins for the oracle's operator K(rho) (CPU only): assembled CSR against
the element loop, rigid-body null space for any density field, symmetry,
energy identity, the patch test, and a cantilever beam against Timoshenko
beam theory."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle.grid import Grid


def _rigid_fields(g: Grid):
    i, j, k = g.node_coords()
    X = np.stack([i, j, k], axis=1).astype(float)
    out = []
    for c in range(3):
        v = np.zeros((g.N, 3)); v[:, c] = 1.0
        out.append(v.ravel())
    for w in np.eye(3):
        out.append(np.cross(w, X - X.mean(0)).ravel())
    return out


def test_csr_equals_element_loop_with_bcs_and_springs():
    g = Grid(5, 4, 3)
    rng = np.random.default_rng(0)
    s = oracle.simp_scale(rng.uniform(0.0, 1.0, g.E))
    mask = synth.random_mask(g.ndof, 0.1, seed=4)
    springs = ((7, 0.3), (int(np.flatnonzero(mask == 0)[-1]), 0.1))
    K = oracle.assemble_K(g, s, mask, springs)
    U = rng.standard_normal((3, g.ndof))
    Y = oracle.apply_K(g, s, U, mask, springs, chunk=17)
    for r in range(3):
        ref = K @ U[r]
        assert np.abs(Y[r] - ref).max() <= 1e-14 * np.abs(ref).max()
    assert abs(K - K.T).max() <= 1e-15 * abs(K).max()
    # fixed DOFs: identity rows
    fixed = np.flatnonzero(mask)
    assert np.array_equal(Y[0][fixed], U[0][fixed])
    # Jacobi diagonal
    assert np.abs(oracle.jacobi_diag(g, s, mask, springs) - K.diagonal()).max() < 1e-15
    # sampled rows
    nodes = [0, 17, g.N // 2, g.N - 1]
    rows = oracle.apply_K_rows(g, s, U[1], nodes, mask, springs)
    for r, n in enumerate(nodes):
        assert np.allclose(rows[r], Y[1][3 * n:3 * n + 3], rtol=0, atol=1e-14)


def test_rigid_modes_in_null_space_for_any_density():
    g = Grid(4, 3, 5)
    s = oracle.simp_scale(np.random.default_rng(1).uniform(0, 1, g.E))
    for v in _rigid_fields(g):
        y = oracle.apply_K(g, s, v)
        assert np.abs(y).max() < 1e-13


def test_energy_identity():
    g = Grid(3, 4, 2)
    rng = np.random.default_rng(2)
    s = oracle.simp_scale(rng.uniform(0, 1, g.E))
    u = rng.standard_normal(g.ndof)
    w = oracle.element_energy(g, u)
    assert abs(u @ oracle.apply_K(g, s, u) - s @ w) < 1e-12 * abs(s @ w)


def test_patch_test_interior_and_prescribed():
    """(i) an affine field has zero force at interior nodes of a homogeneous
    grid; (ii) prescribing it on the boundary and solving reproduces it in
    the interior to round-off."""
    g = Grid(5, 4, 4)
    s = np.ones(g.E)
    i, j, k = g.node_coords()
    X = np.stack([i, j, k], axis=1).astype(float)
    G = np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.4], [0.25, 0.05, 0.7]]) * 1e-3
    u = (X @ G.T).ravel()
    y = oracle.apply_K(g, s, u).reshape(-1, 3)
    interior = (i > 0) & (i < g.nx) & (j > 0) & (j < g.ny) & (k > 0) & (k < g.nz)
    assert np.abs(y[interior]).max() < 1e-17
    K = oracle.assemble_K(g, s)
    bnode = ~interior
    bdof = np.repeat(bnode, 3)
    I_ = np.flatnonzero(~bdof)
    B_ = np.flatnonzero(bdof)
    KII = K[I_][:, I_]
    KIB = K[I_][:, B_]
    uI = spla.spsolve(KII.tocsc(), -(KIB @ u[B_]))
    assert np.abs(uI - u[I_]).max() <= 1e-12 * np.abs(u).max()


def _beam_tip(nx, ny, nz, nu):
    g = Grid(nx, ny, nz)
    p = synth.cantilever(nx, ny, nz, volfrac=1.0, filter_radius=1.0, outer_iters=0,
                         inner_steps=0, x0=1.0)
    # consistent end-face traction, total force 1 in -z
    wj = np.ones(ny + 1); wj[[0, -1]] = 0.5
    wk = np.ones(nz + 1); wk[[0, -1]] = 0.5
    jj, kk = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    n = g.node(nx, jj.ravel(), kk.ravel())
    w = (wj[jj.ravel()] * wk[kk.ravel()]) / (ny * nz)
    f = np.zeros(g.ndof)
    f[3 * n + 2] = -w
    K = oracle.assemble_K(g, np.ones(g.E), p.fixed_mask, KE=oracle.element_stiffness(1.0, nu))
    u = oracle.solve_direct(K, f)
    return -float(w @ u[3 * n + 2])          # load-weighted mean deflection


@pytest.mark.slow
def test_cantilever_against_timoshenko():
    """Solid cantilever of slenderness L/h = 8 (nu = 0) meshed with m = 2, 4, 8
    elements through the thickness.  With unit elements the beam of mesh m
    has L = 8m, b = h = m, so m * deflection is mesh-independent in the
    limit: it converges as O(h^2) and the Richardson-extrapolated value
    matches Timoshenko's  PL^3/(3EI) + PL/(kappa G A)  (kappa = 5/6)."""
    nu = 0.0
    d = np.array([m * _beam_tip(8 * m, m, m, nu) for m in (2, 4, 8)])
    ratio = (d[1] - d[0]) / (d[2] - d[1])
    assert 3.0 < ratio < 5.0
    extrap = (4 * d[2] - d[1]) / 3
    L, b, h, E, G = 8.0, 1.0, 1.0, 1.0, 0.5
    timo = L ** 3 / (3 * E * b * h ** 3 / 12) + L / (5 / 6 * G * b * h)
    assert abs(extrap - timo) / timo < 5e-3


def test_simp_scale_power_law():
    """The modified SIMP law s = rho_min + (1 - rho_min) rho^p pinned by its
    end values (a void keeps the floor rho_min, solid material the full
    stiffness) and its scaling: s - rho_min is homogeneous of degree p."""
    rho = np.random.default_rng(3).uniform(0.01, 0.5, 50)
    for p, rmin in ((3.0, 1e-3), (1.0, 0.0), (2.5, 1e-2)):
        assert oracle.simp_scale(np.array([0.0]), p, rmin)[0] == rmin
        assert abs(oracle.simp_scale(np.array([1.0]), p, rmin)[0] - 1.0) <= 1e-15
        ratio = (oracle.simp_scale(2 * rho, p, rmin) - rmin) / (oracle.simp_scale(rho, p, rmin) - rmin)
        assert np.abs(ratio - 2.0 ** p).max() <= 1e-12
