"""Non-overlapping box partitions, subdomain closures and interface faces.

Test infrastructure (oracle). Sec. 3 decomposes the domain into
non-overlapping subdomains with interfaces between them; the paper's runs cut
one axis only (Sec. 6). Here a partition is a tensor product of cut lists,
one per axis, so every subdomain is a box of elements and two subdomains that
touch share either a whole face, an edge or a corner.

Subdomain s = px + Px*(py + Py*pz). Its local unknowns are the nodes of its
closed element box minus nodes on outer Dirichlet faces, numbered x fastest
over the kept index ranges lo[d]..hi[d] (global node indices).

Directed faces: face (s <- j) carries the Robin datum that subdomain s
receives from neighbour j. They are ordered by s, then axis (x, y, z), then
side (lower, upper). The nodes of a face are listed with the first tangential
axis fastest (for an x-face: y fastest, then z; y-face: x then z; z-face: x
then y), over s's kept ranges; the two directions of one interface list the
same global nodes in the same order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import BoxMesh, DIRICHLET


@dataclass
class Subdomain:
    s: int
    pidx: tuple
    e0: tuple
    e1: tuple
    lo: tuple
    hi: tuple
    neighbor: dict = field(default_factory=dict)  # (axis, side) -> j

    @property
    def shape(self):
        return tuple(h - l + 1 for l, h in zip(self.lo, self.hi))

    @property
    def n(self):
        return int(np.prod(self.shape))


@dataclass
class Face:
    index: int
    s: int
    j: int
    axis: int
    side: int  # side of s: 0 lower, 1 upper
    nodes: np.ndarray  # global node ids
    tshape: tuple  # (n_a, n_b), tangential axes in increasing order


class BoxPartition:
    def __init__(self, mesh: BoxMesh, cuts):
        self.mesh = mesh
        self.cuts = []
        for d in range(3):
            c = [int(v) for v in cuts[d]]
            if any(b <= a for a, b in zip(c, c[1:])) or any(v <= 0 or v >= mesh.ne[d] for v in c):
                raise ValueError("cuts must be strictly increasing inside (0, ne)")
            self.cuts.append(c)
        self.nparts = tuple(len(c) + 1 for c in self.cuts)
        bounds = [[0] + c + [mesh.ne[d]] for d, c in enumerate(self.cuts)]
        Px, Py, Pz = self.nparts
        self.subs = []
        for pz in range(Pz):
            for py in range(Py):
                for px in range(Px):
                    p = (px, py, pz)
                    e0 = tuple(bounds[d][p[d]] for d in range(3))
                    e1 = tuple(bounds[d][p[d] + 1] for d in range(3))
                    lo, hi = [], []
                    for d in range(3):
                        l, h = 2 * e0[d], 2 * e1[d]
                        if e0[d] == 0 and mesh.bc[2 * d] == DIRICHLET:
                            l += 1
                        if e1[d] == mesh.ne[d] and mesh.bc[2 * d + 1] == DIRICHLET:
                            h -= 1
                        lo.append(l)
                        hi.append(h)
                    s = px + Px * (py + Py * pz)
                    self.subs.append(Subdomain(s, p, e0, e1, tuple(lo), tuple(hi)))
        for sub in self.subs:
            for d in range(3):
                for side in (0, 1):
                    q = list(sub.pidx)
                    q[d] += -1 if side == 0 else 1
                    if 0 <= q[d] < self.nparts[d]:
                        sub.neighbor[(d, side)] = q[0] + Px * (q[1] + Py * q[2])
        self.faces = []
        for sub in self.subs:
            for d in range(3):
                for side in (0, 1):
                    if (d, side) in sub.neighbor:
                        nodes, tshape = self._face_nodes(sub, d, side)
                        self.faces.append(Face(len(self.faces), sub.s, sub.neighbor[(d, side)],
                                               d, side, nodes, tshape))
        self.face_index = {(f.s, f.j): f.index for f in self.faces}

    @property
    def n_sub(self):
        return len(self.subs)

    def local_nodes(self, sub: Subdomain):
        """Global ids of s's local unknowns in local order (x fastest)."""
        (lx, ly, lz), (hx, hy, hz) = sub.lo, sub.hi
        iz, iy, ix = np.meshgrid(np.arange(lz, hz + 1), np.arange(ly, hy + 1),
                                 np.arange(lx, hx + 1), indexing="ij")
        return self.mesh.node_id(ix.ravel(), iy.ravel(), iz.ravel())

    def _face_nodes(self, sub: Subdomain, d, side):
        plane = 2 * sub.e0[d] if side == 0 else 2 * sub.e1[d]
        ta, tb = [a for a in range(3) if a != d]
        ra = np.arange(sub.lo[ta], sub.hi[ta] + 1)
        rb = np.arange(sub.lo[tb], sub.hi[tb] + 1)
        B, A = np.meshgrid(rb, ra, indexing="ij")
        idx = [None, None, None]
        idx[d] = np.full(A.size, plane)
        idx[ta] = A.ravel()
        idx[tb] = B.ravel()
        return self.mesh.node_id(*idx), (ra.size, rb.size)

    def elements_of(self, sub: Subdomain):
        nx, ny, _ = self.mesh.ne
        ez, ey, ex = np.meshgrid(np.arange(sub.e0[2], sub.e1[2]), np.arange(sub.e0[1], sub.e1[1]),
                                 np.arange(sub.e0[0], sub.e1[0]), indexing="ij")
        return (ex + nx * (ey + ny * ez)).ravel()

    def multiplicity(self):
        """Number of subdomain copies of every global node."""
        m = np.zeros(self.mesh.n_nodes)
        for sub in self.subs:
            m[self.local_nodes(sub)] += 1
        return m
