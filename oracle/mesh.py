"""Box mesh of Q2 hexahedra: node and element numbering, Dirichlet nodes.

Test infrastructure (oracle). The domain is [0,Lx]x[0,Ly]x[0,Lz] with
nx*ny*nz equal box elements. Nodes form the (2nx+1)(2ny+1)(2nz+1) tensor grid
(element vertices plus edge, face and cell mid-points), numbered
ix + Nx*(iy + Ny*iz), x fastest. Elements are numbered ex + nx*(ey + ny*ez).
Boundary conditions per outer face, in the order x-, x+, y-, y+, z-, z+:
0 = homogeneous Dirichlet (Sec. 3 poses the model problem with it),
1 = homogeneous Neumann.
"""
from __future__ import annotations

import numpy as np

DIRICHLET = 0
NEUMANN = 1


class BoxMesh:
    def __init__(self, ne, lengths=(1.0, 1.0, 1.0), bc=(DIRICHLET,) * 6):
        self.ne = tuple(int(v) for v in ne)
        self.lengths = tuple(float(v) for v in lengths)
        self.bc = tuple(int(v) for v in bc)
        self.h = tuple(L / n for L, n in zip(self.lengths, self.ne))
        self.nn = tuple(2 * n + 1 for n in self.ne)

    @property
    def n_nodes(self):
        return int(np.prod(self.nn))

    @property
    def n_elem(self):
        return int(np.prod(self.ne))

    def node_id(self, ix, iy, iz):
        Nx, Ny, _ = self.nn
        return np.asarray(ix) + Nx * (np.asarray(iy) + Ny * np.asarray(iz))

    def element_nodes(self):
        """(n_elem, 27) global node ids; local node a = ax + 3ay + 9az
        (computed once per mesh)."""
        if getattr(self, "_conn", None) is None:
            self._conn = self._element_nodes()
        return self._conn

    def _element_nodes(self):
        nx, ny, nz = self.ne
        ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
        a = np.arange(27)
        ax, ay, az = a % 3, (a // 3) % 3, a // 9
        return self.node_id(2 * ex[:, None] + ax, 2 * ey[:, None] + ay, 2 * ez[:, None] + az)

    def node_coords(self):
        Nx, Ny, Nz = self.nn
        hx, hy, hz = self.h
        iz, iy, ix = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
        return np.stack([ix.ravel() * hx / 2, iy.ravel() * hy / 2, iz.ravel() * hz / 2], axis=1)

    def node_grid_index(self):
        """(ix, iy, iz) per node."""
        Nx, Ny, Nz = self.nn
        g = np.arange(self.n_nodes)
        return g % Nx, (g // Nx) % Ny, g // (Nx * Ny)

    def dirichlet_mask(self):
        ix, iy, iz = self.node_grid_index()
        m = np.zeros(self.n_nodes, bool)
        for d, i in enumerate((ix, iy, iz)):
            if self.bc[2 * d] == DIRICHLET:
                m |= i == 0
            if self.bc[2 * d + 1] == DIRICHLET:
                m |= i == self.nn[d] - 1
        return m

    def unknowns(self):
        """Global ids of the nodes that carry an unknown (non-Dirichlet)."""
        return np.flatnonzero(~self.dirichlet_mask())
