"""Seeded synthetic problems and inputs.

Shared by the CPU oracle's tests, the GPU parity tests and the benchmark.
This module only *defines problems*: grid sizes, supports, loads, springs,
initial designs and seeded random vectors.  It holds none of the method's
arithmetic (no element stiffness, no operator, no solve, no filter, no
projection), so that the oracle and the HIP path share nothing else.

Numbering (used by both sides and by the C ABI):
  node  n = i + (nx+1) * (j + (ny+1) * k),   0 <= i <= nx, ...
  DOF   3*n + c,  c in {0: x, 1: y, 2: z}
  elem  e = ex + nx * (ey + ny * ez)
  multi-RHS vectors are stored as [nrhs][3N].
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Problem", "node_id", "n_nodes", "n_elems", "cantilever", "inverter",
    "bridge", "multiload_cantilever", "config", "CONFIG_NAMES",
    "uniform_density", "normal_vector", "random_mask", "fd_elements",
]


def n_nodes(nx: int, ny: int, nz: int) -> int:
    return (nx + 1) * (ny + 1) * (nz + 1)


def n_elems(nx: int, ny: int, nz: int) -> int:
    return nx * ny * nz


def node_id(i, j, k, nx: int, ny: int):
    """Global node number of grid point (i, j, k) (x fastest)."""
    return i + (nx + 1) * (j + (ny + 1) * k)


@dataclasses.dataclass
class Problem:
    """A voxel-grid SIMP problem instance (all arrays host-side numpy)."""

    name: str
    nx: int
    ny: int
    nz: int
    volfrac: float
    filter_radius: float
    outer_iters: int
    inner_steps: int
    fixed_mask: np.ndarray            # uint8 [3N], 1 = DOF fixed (u = 0)
    loads: np.ndarray                 # float64 [nrhs][3N]
    x0: np.ndarray                    # float64 [E], initial design
    springs: Tuple[Tuple[int, float], ...] = ()   # (dof, k) pairs
    target: Optional[np.ndarray] = None  # float64 [3N]: objective L = target . u
    young: float = 1.0
    poisson: float = 0.3
    penal: float = 3.0
    rho_min: float = 1e-3
    seed: int = 0
    note: str = ""

    @property
    def E(self) -> int:
        return n_elems(self.nx, self.ny, self.nz)

    @property
    def N(self) -> int:
        return n_nodes(self.nx, self.ny, self.nz)

    @property
    def ndof(self) -> int:
        return 3 * self.N

    @property
    def nrhs(self) -> int:
        return int(self.loads.shape[0])

    @property
    def vmax(self) -> float:
        """Total-material bound of the feasible set: sum(x) <= volfrac * E."""
        return float(self.volfrac * self.E)

    def spring_arrays(self):
        dof = np.array([s[0] for s in self.springs], dtype=np.int64)
        k = np.array([s[1] for s in self.springs], dtype=np.float64)
        return dof, k


# --------------------------------------------------------------------------
# seeded random inputs
# --------------------------------------------------------------------------

def uniform_density(E: int, seed: int = 0, lo: float = 0.2, hi: float = 0.4) -> np.ndarray:
    """i.i.d. U[lo, hi] densities in element order (x fastest), FP64."""
    return np.random.default_rng(seed).uniform(lo, hi, E)


def normal_vector(n: int, seed: int = 1, nrhs: int = 1) -> np.ndarray:
    """i.i.d. N(0, 1) vectors, shape [nrhs][n], FP64."""
    return np.random.default_rng(seed).standard_normal((nrhs, n))


def random_mask(ndof: int, frac: float, seed: int = 3) -> np.ndarray:
    """Random fixed-DOF mask (uint8) with about `frac` of DOFs fixed."""
    return (np.random.default_rng(seed).random(ndof) < frac).astype(np.uint8)


def fd_elements(E: int, count: int = 32, seed: int = 2) -> np.ndarray:
    """Elements picked for finite-difference checks."""
    return np.sort(np.random.default_rng(seed).choice(E, count, replace=False))


# --------------------------------------------------------------------------
# supports and loads
# --------------------------------------------------------------------------

def _clamp_face_x0(nx, ny, nz) -> np.ndarray:
    mask = np.zeros(3 * n_nodes(nx, ny, nz), dtype=np.uint8)
    j, k = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    n = node_id(0, j.ravel(), k.ravel(), nx, ny)
    for c in range(3):
        mask[3 * n + c] = 1
    return mask


def _point_load(nx, ny, nz, i, j, k, comp, value=-1.0) -> np.ndarray:
    f = np.zeros(3 * n_nodes(nx, ny, nz))
    f[3 * node_id(i, j, k, nx, ny) + comp] = value
    return f


def cantilever(nx, ny, nz, *, volfrac, filter_radius, outer_iters, inner_steps,
               load_node=None, x0=None, seed=0, name=None, note="") -> Problem:
    """x = 0 face clamped (all three DOFs); unit -z load at `load_node`
    (default: free end, mid-height in y, bottom z)."""
    if load_node is None:
        load_node = (nx, ny // 2, 0)
    mask = _clamp_face_x0(nx, ny, nz)
    f = _point_load(nx, ny, nz, *load_node, comp=2, value=-1.0)[None, :]
    E = n_elems(nx, ny, nz)
    if x0 is None:
        x0 = uniform_density(E, seed)
    elif np.isscalar(x0):
        x0 = np.full(E, float(x0))
    return Problem(name=name or f"cantilever_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                   volfrac=volfrac, filter_radius=filter_radius,
                   outer_iters=outer_iters, inner_steps=inner_steps,
                   fixed_mask=mask, loads=f, x0=np.asarray(x0, dtype=np.float64),
                   seed=seed, note=note)


def inverter(nx=128, ny=64, nz=64, *, seed=0, spring_k=0.1, volfrac=0.25,
             filter_radius=2.0, outer_iters=100, inner_steps=8) -> Problem:
    """Seesaw-type inverter: fulcrum strip of fixed nodes on the bottom face
    (56 <= i <= 72 at 128 elements, scaled otherwise), input push f_z = -1 at
    (nx-8, ny/2, nz-1), output node (8, ny/2, nz-1), springs k on the z DOF of
    input and output.  Objective L = -u_z(out), i.e. target = -e_{out,z}."""
    N = n_nodes(nx, ny, nz)
    mask = np.zeros(3 * N, dtype=np.uint8)
    lo_i, hi_i = (56 * nx) // 128, (72 * nx) // 128
    ii, jj = np.meshgrid(np.arange(lo_i, hi_i + 1), np.arange(ny + 1), indexing="ij")
    n = node_id(ii.ravel(), jj.ravel(), 0, nx, ny)
    for c in range(3):
        mask[3 * n + c] = 1
    n_in = node_id(nx - 8, ny // 2, nz - 1, nx, ny)
    n_out = node_id(8, ny // 2, nz - 1, nx, ny)
    f = np.zeros(3 * N)
    f[3 * n_in + 2] = -1.0
    target = np.zeros(3 * N)
    target[3 * n_out + 2] = -1.0
    springs = ((3 * n_in + 2, spring_k), (3 * n_out + 2, spring_k))
    E = n_elems(nx, ny, nz)
    return Problem(name=f"inverter_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                   volfrac=volfrac, filter_radius=filter_radius,
                   outer_iters=outer_iters, inner_steps=inner_steps,
                   fixed_mask=mask, loads=f[None, :], x0=uniform_density(E, seed),
                   springs=springs, target=target, seed=seed)


def bridge(nx=256, ny=128, nz=128, *, seed=0, volfrac=0.15, filter_radius=2.0,
           outer_iters=20, inner_steps=8) -> Problem:
    """Bridge: node lines (0, j, 0) and (nx, j, 0) fixed (all DOFs); uniform
    -z traction of total force 1 on the top face z = nz, lumped as the
    consistent bilinear nodal loads (interior t, edges t/2, corners t/4,
    t = 1/(nx*ny))."""
    N = n_nodes(nx, ny, nz)
    mask = np.zeros(3 * N, dtype=np.uint8)
    for i in (0, nx):
        n = node_id(i, np.arange(ny + 1), 0, nx, ny)
        for c in range(3):
            mask[3 * n + c] = 1
    t = 1.0 / (nx * ny)
    wi = np.ones(nx + 1); wi[0] = wi[-1] = 0.5
    wj = np.ones(ny + 1); wj[0] = wj[-1] = 0.5
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    f = np.zeros(3 * N)
    n = node_id(ii.ravel(), jj.ravel(), nz, nx, ny)
    f[3 * n + 2] = -t * (wi[ii.ravel()] * wj[jj.ravel()])
    E = n_elems(nx, ny, nz)
    return Problem(name=f"bridge_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                   volfrac=volfrac, filter_radius=filter_radius,
                   outer_iters=outer_iters, inner_steps=inner_steps,
                   fixed_mask=mask, loads=f[None, :], x0=uniform_density(E, seed),
                   seed=seed)


def multiload_cantilever(nx=384, ny=192, nz=192, *, seed=2, volfrac=0.1,
                         filter_radius=3.0, outer_iters=20, inner_steps=8) -> Problem:
    """Cantilever clamped at x = 0 with 4 load cases: unit loads at 4 seeded
    distinct nodes of the free-end face i = nx, directions +y, -y, +z, -z."""
    mask = _clamp_face_x0(nx, ny, nz)
    N = n_nodes(nx, ny, nz)
    face = np.random.default_rng(seed).choice((ny + 1) * (nz + 1), 4, replace=False)
    dirs = ((1, +1.0), (1, -1.0), (2, +1.0), (2, -1.0))
    f = np.zeros((4, 3 * N))
    for r, (idx, (comp, sgn)) in enumerate(zip(face, dirs)):
        j, k = int(idx) % (ny + 1), int(idx) // (ny + 1)
        f[r, 3 * node_id(nx, j, k, nx, ny) + comp] = sgn
    E = n_elems(nx, ny, nz)
    return Problem(name=f"multiload_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                   volfrac=volfrac, filter_radius=filter_radius,
                   outer_iters=outer_iters, inner_steps=inner_steps,
                   fixed_mask=mask, loads=f, x0=np.full(E, volfrac), seed=seed)


CONFIG_NAMES = ("cfg1", "cfg2", "cfg3", "cfg3_inverter", "cfg4", "cfg5")


def config(name: str) -> Problem:
    """The five workload configurations of the benchmark: grid, volume
    fraction, filter radius, inner steps, load and supports of each."""
    if name == "cfg1":
        return cantilever(16, 8, 8, volfrac=0.3, filter_radius=1.5, outer_iters=50,
                          inner_steps=5, load_node=(16, 4, 0), x0=0.3, name="cfg1",
                          note="16x8x8 = 1,024 elements, 1,377 nodes, 4,131 DOFs")
    if name == "cfg2":
        return cantilever(64, 32, 32, volfrac=0.25, filter_radius=2.0, outer_iters=100,
                          inner_steps=8, seed=0, name="cfg2")
    if name == "cfg3":
        return cantilever(128, 64, 64, volfrac=0.25, filter_radius=2.0, outer_iters=100,
                          inner_steps=8, seed=0, name="cfg3")
    if name == "cfg3_inverter":
        return inverter(128, 64, 64)
    if name == "cfg4":
        return bridge(256, 128, 128)
    if name == "cfg5":
        return multiload_cantilever(384, 192, 192)
    raise KeyError(name)


def small_cases() -> Sequence[Problem]:
    """Small grids that still span several GPU tiles and a ragged tail."""
    out = []
    for (nx, ny, nz), seed in (((24, 13, 11), 5), ((37, 9, 6), 6), ((3, 2, 2), 7)):
        p = cantilever(nx, ny, nz, volfrac=0.3, filter_radius=1.5, outer_iters=10,
                       inner_steps=5, seed=seed)
        out.append(p)
    return out


# --------------------------------------------------------------------------
# plane (2D) problems: the paper's own setting
# --------------------------------------------------------------------------
# Numbering on a plane grid: node n = i + (nx+1) * j, DOF 2*n + c
# (c in {0: x, 1: y}), element e = ex + nx * ey, vectors [nrhs][2N].

@dataclasses.dataclass
class PlaneProblem:
    """A plane-grid SIMP problem (Q4 elements, Gaussian filter)."""

    name: str
    nx: int
    ny: int
    volfrac: float
    fixed_mask: np.ndarray            # uint8 [2N]
    loads: np.ndarray                 # float64 [nrhs][2N]
    x0: np.ndarray                    # float64 [E]
    lo: float = 0.1                   # lower bound of the box (the paper's v_)
    degree: int = 20                  # Krylov degree D of Alg. 3
    beta: float = 1.0                 # step of the low-level update
    filter_half: int = 3              # 7 x 7 window
    filter_sigma: float = 1.4
    young: float = 1.0
    poisson: float = 0.3
    penal: float = 3.0
    rho_min: float = 0.0
    note: str = ""

    @property
    def E(self) -> int:
        return self.nx * self.ny

    @property
    def N(self) -> int:
        return (self.nx + 1) * (self.ny + 1)

    @property
    def ndof(self) -> int:
        return 2 * self.N

    @property
    def nrhs(self) -> int:
        return int(self.loads.shape[0])

    @property
    def vmax(self) -> float:
        return float(self.volfrac * self.E)


def plane_cantilever(nx: int, ny: int, volfrac: float, *, name=None, note="") -> PlaneProblem:
    """Plane cantilever: the x = 0 edge clamped (both DOFs), a unit -y load at
    the free end's middle node (nx, ny // 2); initial design uniform at the
    volume fraction."""
    N = (nx + 1) * (ny + 1)
    mask = np.zeros(2 * N, dtype=np.uint8)
    for j in range(ny + 1):
        mask[2 * (j * (nx + 1))] = mask[2 * (j * (nx + 1)) + 1] = 1
    f = np.zeros((1, 2 * N))
    f[0, 2 * (nx + (nx + 1) * (ny // 2)) + 1] = -1.0
    return PlaneProblem(name=name or f"plane_cantilever_{nx}x{ny}", nx=nx, ny=ny, volfrac=volfrac,
                        fixed_mask=mask, loads=f, x0=np.full(nx * ny, float(volfrac)), note=note)


# Grid shapes and volume fractions of the paper's benchmark table (resolution
# "a x b" read as a rows (y) by b columns (x)); the loads and supports of its
# benchmarks exist only in its figures, so a cantilever stands in for each.
PLANE_TABLE = (
    ("teaser", 256, 128, 0.4), ("a", 576, 192, 0.3), ("b", 576, 192, 0.3), ("c", 384, 192, 0.3),
    ("d", 240, 160, 0.4), ("e", 160, 160, 0.5), ("f", 384, 128, 0.5), ("g", 256, 128, 0.3),
)


def plane_config(name: str) -> PlaneProblem:
    """A plane cantilever at one of the table's shapes ("plane_a" ...), or the
    small parity case "plane_small" (48 x 16)."""
    if name == "plane_small":
        return plane_cantilever(48, 16, 0.4, name=name)
    for key, nx, ny, vf in PLANE_TABLE:
        if name == f"plane_{key}":
            return plane_cantilever(nx, ny, vf, name=name, note=f"{ny} x {nx}, volume fraction {vf}")
    raise KeyError(name)
