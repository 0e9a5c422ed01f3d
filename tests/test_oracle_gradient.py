"""Pin the oracle's sensitivities against central finite differences of the
exact objective (direct FP64 solves), through the density filter, for the
compliance (self-adjoint) and a target-displacement objective with springs
(true adjoint)."""
import numpy as np
import pytest

import oracle
import synth
from oracle.grid import Grid


def _objective(g, p, H, Hs, x, which):
    rho = oracle.filter_forward(H, Hs, x)
    s = oracle.simp_scale(rho, p.penal, p.rho_min)
    K = oracle.assemble_K(g, s, p.fixed_mask, p.springs)
    u = oracle.solve_direct(K, p.loads[0])
    if which == "compliance":
        return float(p.loads[0] @ u), u, K, rho
    return float(p.target @ u), u, K, rho


def _adjoint_grad(g, p, H, Hs, x, which):
    val, u, K, rho = _objective(g, p, H, Hs, x, which)
    if which == "compliance":
        g_rho = oracle.compliance_gradient(g, rho, u, p.fixed_mask, p.penal, p.rho_min)
    else:
        lam = oracle.solve_direct(K, p.target)
        g_rho = oracle.adjoint_gradient(g, rho, u, lam, p.fixed_mask, p.penal, p.rho_min)
    return oracle.filter_transpose(H, Hs, g_rho)


def _fd_check(p, which, elems, h=1e-4, tol=1e-6):
    g = Grid(p.nx, p.ny, p.nz)
    H, Hs = oracle.cone_filter_matrix(g, p.filter_radius)
    x = p.x0.copy()
    grad = _adjoint_grad(g, p, H, Hs, x, which)
    gmax = np.abs(grad).max()
    for j in elems:
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (_objective(g, p, H, Hs, xp, which)[0] - _objective(g, p, H, Hs, xm, which)[0]) / (2 * h)
        if abs(grad[j]) >= 1e-3 * gmax:
            assert abs(fd - grad[j]) <= tol * abs(grad[j]), (j, fd, grad[j])
        else:
            assert abs(fd - grad[j]) <= tol * gmax


def test_compliance_gradient_fd_cfg1():
    p = synth.config("cfg1")
    p.x0 = synth.uniform_density(p.E, 9)          # non-uniform field
    _fd_check(p, "compliance", synth.fd_elements(p.E, 24, seed=2))


def test_compliance_gradient_fd_all_elements_small():
    p = synth.cantilever(4, 3, 2, volfrac=0.3, filter_radius=1.5, outer_iters=1,
                         inner_steps=1, seed=4)
    _fd_check(p, "compliance", range(p.E))


def test_target_displacement_adjoint_fd():
    p = synth.inverter(16, 8, 8, seed=3)
    _fd_check(p, "target", synth.fd_elements(p.E, 24, seed=2))


def test_sensitivity_sums_over_load_cases():
    g = Grid(3, 2, 2)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((3, g.ndof))
    total = oracle.element_energy(g, U)
    parts = sum(oracle.element_energy(g, U[r]) for r in range(3))
    assert np.allclose(total, parts, rtol=1e-14, atol=0)


def test_sampled_bilinear_equals_full_pass():
    """The per-element bilinear form used for sampled checks on large grids
    equals the full pass (two load cases, fixed DOFs masked)."""
    g = Grid(7, 5, 4)
    rng = np.random.default_rng(3)
    u = rng.normal(0.0, 1.0, (2, g.ndof))
    lam = rng.normal(0.0, 1.0, (2, g.ndof))
    mask = (rng.uniform(0.0, 1.0, g.ndof) < 0.1).astype(np.uint8)
    elems = rng.permutation(g.E)[:37]
    full = oracle.element_bilinear(g, lam, u, mask)
    assert np.allclose(oracle.element_bilinear_at(g, lam, u, elems, mask), full[elems], rtol=1e-14, atol=1e-13)
