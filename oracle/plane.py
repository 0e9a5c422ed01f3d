"""Two-dimensional variant of the hot path (oracle, FP64): the bilinear
quadrilateral (Q4) on a regular grid of unit squares, plane stress, and the
separable Gaussian density filter of the paper's experiments.

The paper is written in 2D on a regular grid (Sec. 4.3, Sec. 5) but names
neither its element nor its stress state.  Readings taken here:
  - element: the unit-square bilinear Q4 with exact (2x2) integration;
  - plane stress of unit thickness, isotropic (Young's modulus E, Poisson
    ratio nu); the paper sets E = 1 (Sec. 5, parameter sensitivity);
  - filter: the 7x7 separable Gaussian of Sec. 5 (filter paragraph), with
    1D weights g(d) = exp(-d^2 / (2 sigma^2)) for |d| <= 3 and the 2D weight
    H_ej = g(dx) g(dy) over element centres, truncated at the grid boundary
    and normalised by its row sum Hs_e, as the cone filter of the 3D path.
    The paper gives no sigma; sigma = 1.4 is the usual width of a 7-tap
    Gaussian (0.3 ((7 - 1) / 2 - 1) + 0.8).
Numbering: node n = i + (nx + 1) j, DOF 2 n + c, element e = ex + nx ey,
element-local node a = ax + 2 ay at corner (ax, ay) of the square.

Pins (tests/test_oracle_plane.py): KE against 2x2 Gauss quadrature of
B^T D B with the plane-stress D written independently, its three rigid
modes and rank 5, the energy of a uniform strain; the patch test on an
assembled grid; the filter against a brute-force 2D sum and its
factorisation into two 1D passes.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

GAUSS_HALF = 3          # 7 taps per axis
GAUSS_SIGMA = 1.4


def plane_stress_lame(young: float = 1.0, poisson: float = 0.3):
    """(lambda*, mu) of plane stress: the in-plane form of isotropic
    elasticity with the out-of-plane stress eliminated,
    lambda* = E nu / (1 - nu^2), mu = E / (2 (1 + nu))."""
    lam = young * poisson / (1.0 - poisson * poisson)
    mu = young / (2.0 * (1.0 + poisson))
    return lam, mu


def q4_stiffness(young: float = 1.0, poisson: float = 0.3) -> np.ndarray:
    """8 x 8 element stiffness of the unit-square Q4, plane stress, from the
    bilinear form int lambda* div u div v + 2 mu eps(u) : eps(v):
        KE[2a+i, 2b+j] = lambda* I_ij(a,b) + mu I_ji(a,b) + mu delta_ij sum_l I_ll(a,b),
    I_ij(a, b) = int d_i N_a d_j N_b, which factors over the two axes into the
    1D integrals of phi_0 = 1 - t, phi_1 = t:
        int phi_a phi_b = 1/3 (a = b) or 1/6,  int phi_a' phi_b' = s_a s_b,
        int phi_a' phi_b = s_a / 2,  s_0 = -1, s_1 = +1."""
    lam, mu = plane_stress_lame(young, poisson)
    M = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    s = np.array([-1.0, 1.0])
    G = np.outer(s, s)
    C = np.outer(s, [0.5, 0.5])
    corners = [(a & 1, (a >> 1) & 1) for a in range(4)]

    def I(i, j, a, b):
        ca, cb = corners[a], corners[b]
        val = 1.0
        for ax in range(2):
            if ax == i and ax == j:
                val *= G[ca[ax], cb[ax]]
            elif ax == i:
                val *= C[ca[ax], cb[ax]]
            elif ax == j:
                val *= C[cb[ax], ca[ax]]
            else:
                val *= M[ca[ax], cb[ax]]
        return val

    KE = np.zeros((8, 8))
    for a, b in itertools.product(range(4), range(4)):
        trace = I(0, 0, a, b) + I(1, 1, a, b)
        for i, j in itertools.product(range(2), range(2)):
            KE[2 * a + i, 2 * b + j] = (lam * I(i, j, a, b) + mu * I(j, i, a, b)
                                        + (mu * trace if i == j else 0.0))
    return KE


class Grid2D:
    """Structured grid of nx x ny unit squares (same interface as the 3D
    Grid where the operator, sensitivity and outer-step code use it)."""

    dim = 2

    def __init__(self, nx: int, ny: int):
        if min(nx, ny) < 1:
            raise ValueError("grid needs at least one element per axis")
        self.nx, self.ny = int(nx), int(ny)
        self.E = self.nx * self.ny
        self.N = (self.nx + 1) * (self.ny + 1)
        self.ndof = 2 * self.N

    def node(self, i, j):
        return i + (self.nx + 1) * j

    def elem_coords(self, e=None):
        e = np.arange(self.E) if e is None else np.asarray(e)
        return e % self.nx, e // self.nx

    def node_coords(self, n=None):
        n = np.arange(self.N) if n is None else np.asarray(n)
        return n % (self.nx + 1), n // (self.nx + 1)

    def elem_nodes(self, e=None) -> np.ndarray:
        ex, ey = self.elem_coords(e)
        cols = [self.node(ex + (a & 1), ey + (a >> 1)) for a in range(4)]
        return np.stack(cols, axis=1).astype(np.int64)

    def elem_dofs(self, e=None) -> np.ndarray:
        """[len(e), 8] global DOFs, local DOF 2a + c."""
        en = self.elem_nodes(e)
        return (2 * en[:, :, None] + np.arange(2)[None, None, :]).reshape(en.shape[0], 8)

    def node_elems(self, n: int):
        i, j = (int(v) for v in self.node_coords(n))
        out = []
        for ay in (0, 1):
            for ax in (0, 1):
                ex, ey = i - ax, j - ay
                if 0 <= ex < self.nx and 0 <= ey < self.ny:
                    out.append((ex + self.nx * ey, ax + 2 * ay))
        return out


def gauss_weights_1d(half: int = GAUSS_HALF, sigma: float = GAUSS_SIGMA) -> np.ndarray:
    """g(d) = exp(-d^2 / (2 sigma^2)) for d = -half .. half."""
    d = np.arange(-half, half + 1, dtype=np.float64)
    return np.exp(-d * d / (2.0 * sigma * sigma))


def gaussian_filter_matrix(grid: Grid2D, half: int = GAUSS_HALF, sigma: float = GAUSS_SIGMA):
    """(H, Hs): H_ej = g(dx) g(dy) for every pair of elements within the
    (2 half + 1)^2 window, by plain enumeration of the window; Hs = row sums."""
    g = gauss_weights_1d(half, sigma)
    ex, ey = grid.elem_coords()
    e = np.arange(grid.E)
    rows, cols, vals = [], [], []
    for dy in range(-half, half + 1):
        for dx in range(-half, half + 1):
            jx, jy = ex + dx, ey + dy
            ok = (jx >= 0) & (jx < grid.nx) & (jy >= 0) & (jy < grid.ny)
            rows.append(e[ok])
            cols.append((jx + grid.nx * jy)[ok])
            vals.append(np.full(int(ok.sum()), g[dx + half] * g[dy + half]))
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(grid.E, grid.E))
    Hs = np.asarray(H.sum(axis=1)).ravel()
    return H, Hs


class PlaneContext:
    """Grid, element matrix and filter matrix of a plane problem, with the
    attributes outer.outer_step_ref reads (the same as OuterContext's).
    The paper's stiffness law is v^eta with a lower bound on v (Sec. 3,
    Sec. 5: eta = 3, lower bound 0.1): rho_min = 0 with the box's lo = 0.1."""

    def __init__(self, nx, ny, fixed_mask, young=1.0, poisson=0.3, penal=3.0, rho_min=0.0,
                 half=GAUSS_HALF, sigma=GAUSS_SIGMA):
        self.grid = Grid2D(nx, ny)
        self.KE = q4_stiffness(young, poisson)
        self.H, self.Hs = gaussian_filter_matrix(self.grid, half, sigma)
        self.fixed = np.asarray(fixed_mask, dtype=np.uint8)
        self.springs = ()
        self.penal, self.rho_min = penal, rho_min

    def operator(self, s):
        from .operator import assemble_K
        K = assemble_K(self.grid, s, self.fixed, self.springs, self.KE)
        return lambda v: K @ v


def tip_deflection_timoshenko(length: float, height: float, young: float = 1.0,
                              poisson: float = 0.3, load: float = 1.0) -> float:
    """Tip deflection of a cantilever of unit thickness under an end load P
    (plane stress): P L^3 / (3 E I) + P L / (kappa G A), I = h^3 / 12,
    A = h, kappa = 5 / 6, G = E / (2 (1 + nu))."""
    I = height ** 3 / 12.0
    G = young / (2.0 * (1.0 + poisson))
    return load * length ** 3 / (3.0 * young * I) + load * length / (5.0 / 6.0 * G * height)
