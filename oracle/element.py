"""Element stiffness of the trilinear hex8 unit-cube voxel (oracle, FP64).

The paper assembles K(v) from element integrals K_e = int_{Omega_e} k_e dx
(Sec. 3, Problem Formulation) on a regular grid (Sec. 4.3) but is written
in 2D and never names its element.  Here the element is the unit-cube
trilinear hex with exact integration, for isotropic linear elasticity
(Young's modulus E, Poisson ratio nu).  Parity unpinned as to the *choice*
of element (a reading); the matrix itself is pinned in
tests/test_oracle_element.py against Gauss quadrature, rigid-body modes and
the continuum energy of a uniform strain.

Local node a = ax + 2*ay + 4*az sits at corner (ax, ay, az) of the cube;
local DOF 3*a + c.
"""
from __future__ import annotations

import itertools

import numpy as np


def material_lame(young: float = 1.0, poisson: float = 0.3):
    """Lame constants (lambda, mu) of isotropic elasticity."""
    lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    mu = young / (2.0 * (1.0 + poisson))
    return lam, mu


def _one_d_integrals():
    """1D integrals of the linear basis phi_0 = 1 - t, phi_1 = t on [0, 1]:
    M[a, b] = int phi_a phi_b,  G[a, b] = int phi_a' phi_b',
    C[a, b] = int phi_a' phi_b."""
    M = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    s = np.array([-1.0, 1.0])          # phi_a' = s_a
    G = np.outer(s, s)
    C = np.outer(s, [0.5, 0.5])        # int phi_a' phi_b = s_a * 1/2
    return M, G, C


def element_stiffness(young: float = 1.0, poisson: float = 0.3) -> np.ndarray:
    """24 x 24 element stiffness KE, written out from the bilinear form
    a(u, v) = int lambda div u div v + 2 mu eps(u) : eps(v).

    With I_ij(a, b) = int d_i N_a d_j N_b  (N_a trilinear):
        KE[3a+i, 3b+j] = lambda I_ij(a,b) + mu I_ji(a,b) + mu delta_ij sum_l I_ll(a,b).
    I_ij factors over the three axes into the 1D integrals M, G, C.
    """
    lam, mu = material_lame(young, poisson)
    M, G, C = _one_d_integrals()
    corners = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]

    def I(i, j, a, b):
        ca, cb = corners[a], corners[b]
        val = 1.0
        for ax in range(3):
            if ax == i and ax == j:
                val *= G[ca[ax], cb[ax]]
            elif ax == i:
                val *= C[ca[ax], cb[ax]]          # d/dx_i on N_a
            elif ax == j:
                val *= C[cb[ax], ca[ax]]          # d/dx_j on N_b
            else:
                val *= M[ca[ax], cb[ax]]
        return val

    KE = np.zeros((24, 24))
    for a, b in itertools.product(range(8), range(8)):
        trace = sum(I(l, l, a, b) for l in range(3))
        for i, j in itertools.product(range(3), range(3)):
            KE[3 * a + i, 3 * b + j] = (lam * I(i, j, a, b) + mu * I(j, i, a, b)
                                        + (mu * trace if i == j else 0.0))
    return KE


def ke_diag_value(young: float = 1.0, poisson: float = 0.3) -> float:
    """Every diagonal entry of KE equals (lambda + 4 mu) / 9 (each I_ii(a,a)
    is 1 * 1/3 * 1/3)."""
    lam, mu = material_lame(young, poisson)
    return (lam + 4.0 * mu) / 9.0


KE_DIAG = ke_diag_value()
