"""Pins for the oracle's hex8 element stiffness (CPU only).

The paper never gives an element matrix (it is 2D and element-agnostic,
Sec. 3), so KE is pinned to independent constructions from elasticity:
Gauss quadrature of B^T D B in Voigt notation, the six rigid-body modes,
and the energy of uniform strain states.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle.element import material_lame


def voigt_D(young, poisson):
    lam, mu = material_lame(young, poisson)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3:, 3:] = np.eye(3) * mu
    return D


def gauss_KE(young=1.0, poisson=0.3):
    """B^T D B integrated with the 2x2x2 Gauss rule on the unit cube."""
    D = voigt_D(young, poisson)
    g = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    KE = np.zeros((24, 24))
    for x, y, z in itertools.product(g, g, g):
        B = np.zeros((6, 24))
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            fx = x if ax else 1 - x
            fy = y if ay else 1 - y
            fz = z if az else 1 - z
            dx = (1 if ax else -1) * fy * fz
            dy = fx * (1 if ay else -1) * fz
            dz = fx * fy * (1 if az else -1)
            c = 3 * a
            B[0, c] = dx
            B[1, c + 1] = dy
            B[2, c + 2] = dz
            B[3, c + 1], B[3, c + 2] = dz, dy          # gamma_yz
            B[4, c], B[4, c + 2] = dz, dx              # gamma_xz
            B[5, c], B[5, c + 1] = dy, dx              # gamma_xy
        KE += 0.125 * B.T @ D @ B
    return KE


def corner_coords():
    return np.array([(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)], dtype=float)


@pytest.mark.parametrize("nu", [0.0, 0.3, 0.45])
def test_closed_form_equals_gauss(nu):
    KE = oracle.element_stiffness(1.0, nu)
    assert np.abs(KE - gauss_KE(1.0, nu)).max() < 1e-15


def test_symmetry_rank_and_rigid_modes():
    KE = oracle.element_stiffness()
    assert np.array_equal(KE, KE.T)
    X = corner_coords() - 0.5
    modes = []
    for c in range(3):                      # translations
        v = np.zeros((8, 3)); v[:, c] = 1.0
        modes.append(v.ravel())
    for w in np.eye(3):                     # infinitesimal rotations w x X
        modes.append(np.cross(w, X).ravel())
    R = np.stack(modes, axis=1)
    assert np.abs(KE @ R).max() < 1e-15
    assert np.linalg.matrix_rank(KE, tol=1e-10) == 18


def test_diagonal_closed_form():
    lam, mu = material_lame(1.0, 0.3)
    assert np.allclose(np.diag(oracle.element_stiffness()), (lam + 4 * mu) / 9, rtol=0, atol=1e-16)
    assert abs(oracle.KE_DIAG - 0.2350427350427350) < 1e-15


def test_uniform_strain_energy():
    """u = eps x (affine) has element energy eps^T D eps times the volume 1,
    with engineering shear strains."""
    rng = np.random.default_rng(11)
    D = voigt_D(1.0, 0.3)
    KE = oracle.element_stiffness()
    X = corner_coords()
    for _ in range(5):
        G = rng.standard_normal((3, 3)) * 1e-3        # displacement gradient
        u = (X @ G.T).ravel()
        eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[1, 2] + G[2, 1],
                        G[0, 2] + G[2, 0], G[0, 1] + G[1, 0]])
        assert abs(u @ KE @ u - eps @ D @ eps) < 1e-18
    # the fixed example strain state
    eps = np.array([1e-3, 2e-3, -1e-3, 5e-4, -7e-4, 3e-4])
    G = np.array([[eps[0], eps[5] / 2, eps[4] / 2],
                  [eps[5] / 2, eps[1], eps[3] / 2],
                  [eps[4] / 2, eps[3] / 2, eps[2]]])
    u = (X @ G.T).ravel()
    assert abs(u @ KE @ u - 7.2423076923076923e-6) < 1e-18


def test_dilatation_eigenvalue():
    """Uniform dilatation is an eigenvector with eigenvalue (3 lambda + 2 mu)/2."""
    for nu in (0.0, 0.3, 0.45):
        lam, mu = material_lame(1.0, nu)
        v = (corner_coords() - 0.5).ravel()
        KE = oracle.element_stiffness(1.0, nu)
        assert np.allclose(KE @ v, (3 * lam + 2 * mu) / 2 * v, atol=1e-14)
