"""Structured voxel grid connectivity (oracle).

The paper notes that on a regular grid the element-to-node map is known in
closed form (Sec. 4.3).  Numbering: node i + (nx+1)(j + (ny+1)k), DOF 3n+c,
element ex + nx(ey + ny ez), element-local node a = ax + 2ay + 4az.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, nx: int, ny: int, nz: int):
        if min(nx, ny, nz) < 1:
            raise ValueError("grid needs at least one element per axis")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.E = nx * ny * nz
        self.N = (nx + 1) * (ny + 1) * (nz + 1)
        self.ndof = 3 * self.N

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def elem_coords(self, e=None):
        e = np.arange(self.E) if e is None else np.asarray(e)
        ex = e % self.nx
        ey = (e // self.nx) % self.ny
        ez = e // (self.nx * self.ny)
        return ex, ey, ez

    def node_coords(self, n=None):
        n = np.arange(self.N) if n is None else np.asarray(n)
        i = n % (self.nx + 1)
        j = (n // (self.nx + 1)) % (self.ny + 1)
        k = n // ((self.nx + 1) * (self.ny + 1))
        return i, j, k

    def elem_nodes(self, e=None) -> np.ndarray:
        """[len(e), 8] global node numbers of each element's local nodes."""
        ex, ey, ez = self.elem_coords(e)
        cols = []
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            cols.append(self.node(ex + ax, ey + ay, ez + az))
        return np.stack(cols, axis=1).astype(np.int64)

    def elem_dofs(self, e=None) -> np.ndarray:
        """[len(e), 24] global DOFs, local DOF 3a + c."""
        en = self.elem_nodes(e)
        return (3 * en[:, :, None] + np.arange(3)[None, None, :]).reshape(en.shape[0], 24)

    def node_elems(self, n: int):
        """Elements incident to node n, with the node's local index in each."""
        i, j, k = (int(v) for v in self.node_coords(n))
        out = []
        for az in (0, 1):
            for ay in (0, 1):
                for ax in (0, 1):
                    ex, ey, ez = i - ax, j - ay, k - az
                    if 0 <= ex < self.nx and 0 <= ey < self.ny and 0 <= ez < self.nz:
                        out.append((ex + self.nx * (ey + self.ny * ez), ax + 2 * ay + 4 * az))
        return out
