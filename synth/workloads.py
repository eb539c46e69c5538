"""Named workloads: box mesh, box partition, Robin coefficient, load and tolerance.

A workload is a plain description; building matrices from it is the solver's
job (the oracle on the CPU, the HIP library on the GPU).

  c1  unit cube, 16^3 Q2 elements, all-Dirichlet, 2x2x1 equal subdomains,
      p = 8/h on every interface, 3 Gaussian blobs, tol 1e-8 (FP64 plain form)
  c2  unit cube, 64^3 elements, 4x4x4 equal subdomains, p = 8/h, layered
      crater-like anomaly with 10 blobs, tol 1e-8 (FP64 vs FP32-inner)
  c3  unit cube, 96x96x48 elements (hx = hy = 1/96, hz = 1/48), 15 random cuts
      in x and 15 in y (widths uniform on {2..9}, redrawn until they sum to
      96), z uncut -> 256 column subdomains of uneven size; p = 8/h_normal
  c4  unit cube, 48^3 elements, 3x3x3, top face z = 1 homogeneous Neumann,
      all other faces Dirichlet (the adjoint workload)
  c5  unit cube, 128^3 elements, 8x8x8 subdomains (the large batched solve)
  c5copy  unit cube, 32^3 elements, 2x2x2 subdomains: the small copy on which
      candidate transmission conditions are scored before the c5 solve
  slab32 / slab64 / slab128  the shape of the paper's Sec. 6 runs: a
      250 x 250 x 15 box (scaled to 1 x 1 x 0.06, 320 x 320 x 19 elements,
      16.0 M nodes) cut into 32, 64 or 128 slabs along x, crater-like field
      with the thin axis z vertical, tol 1e-6 (a slab's x-y node plane is
      larger than a workgroup marches, so the solver marches it along y).
      Robin coefficients: the
      second-order symmetric condition from the Fourier optimisation over the
      interface's frequency range (extra["kmin"], extra["kmax"])

The gravitational constant is the one the paper quotes in Sec. 2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .generators import blobs_density, crater_density, random_widths, widths_to_cuts

G_PAPER = 6.672e-11  # m^3 kg^-1 s^-2, Sec. 2

DIRICHLET = 0
NEUMANN = 1


@dataclass
class Workload:
    name: str
    ne: tuple
    lengths: tuple
    bc: tuple  # x-, x+, y-, y+, z-, z+
    cuts: tuple  # per axis: tuple of interior cut element indices
    p: float  # Robin coefficient used on every directed interface face
    tol: float
    seed: int
    G: float = G_PAPER
    density: str = "blobs"
    n_blobs: int = 3
    extra: dict = field(default_factory=dict)
    up: int = 2  # vertical axis of the crater-like field

    @property
    def h(self):
        return tuple(float(L) / n for L, n in zip(self.lengths, self.ne))

    @property
    def nparts(self):
        return tuple(len(c) + 1 for c in self.cuts)

    @property
    def n_sub(self):
        return int(np.prod(self.nparts))

    @property
    def n_elem(self):
        return int(np.prod(self.ne))

    @property
    def n_nodes(self):
        return int(np.prod([2 * n + 1 for n in self.ne]))

    def drho(self):
        """Per-element density anomaly (kg/m^3) for this workload's seed."""
        if self.density == "blobs":
            return blobs_density(self.ne, self.lengths, self.n_blobs, self.seed)
        if self.density == "crater":
            return crater_density(self.ne, self.lengths, self.seed, self.n_blobs, self.up)
        raise ValueError(self.density)


def equal_cuts(n_elem, parts):
    if n_elem % parts:
        raise ValueError("equal split needs parts | n_elem")
    w = n_elem // parts
    return tuple(int(w * k) for k in range(1, parts))


def workload(name: str, seed: int = 0, **over) -> Workload:
    dirichlet = (DIRICHLET,) * 6
    if name == "c1":
        ne = (16, 16, 16)
        wl = Workload(name, ne, (1.0, 1.0, 1.0), dirichlet,
                      (equal_cuts(16, 2), equal_cuts(16, 2), ()), 8.0 * 16, 1e-8, seed,
                      density="blobs", n_blobs=3)
    elif name == "c2":
        ne = (64, 64, 64)
        wl = Workload(name, ne, (1.0, 1.0, 1.0), dirichlet,
                      tuple(equal_cuts(64, 4) for _ in range(3)), 8.0 * 64, 1e-8, seed,
                      density="crater", n_blobs=10)
    elif name == "c3":
        ne = (96, 96, 48)
        rng = np.random.default_rng(seed)
        wx, _ = random_widths(rng, 96, 16, 2, 9)
        wy, _ = random_widths(rng, 96, 16, 2, 9)
        cuts = (tuple(int(c) for c in widths_to_cuts(wx)),
                tuple(int(c) for c in widths_to_cuts(wy)), ())
        wl = Workload(name, ne, (1.0, 1.0, 1.0), dirichlet, cuts, 8.0 * 96, 1e-8, seed,
                      density="crater", n_blobs=10)
    elif name == "c4":
        ne = (48, 48, 48)
        bc = (DIRICHLET,) * 5 + (NEUMANN,)
        wl = Workload(name, ne, (1.0, 1.0, 1.0), bc,
                      tuple(equal_cuts(48, 3) for _ in range(3)), 8.0 * 48, 1e-10, seed,
                      density="crater", n_blobs=10)
    elif name == "c5":
        ne = (128, 128, 128)
        wl = Workload(name, ne, (1.0, 1.0, 1.0), dirichlet,
                      tuple(equal_cuts(128, 8) for _ in range(3)), 8.0 * 128, 1e-8, seed,
                      density="crater", n_blobs=10)
    elif name == "c5copy":
        ne = (32, 32, 32)
        wl = Workload(name, ne, (1.0, 1.0, 1.0), dirichlet,
                      tuple(equal_cuts(32, 2) for _ in range(3)), 8.0 * 32, 1e-8, seed,
                      density="crater", n_blobs=10)
    elif name in ("slab32", "slab64", "slab128"):
        parts = int(name[4:])
        ne = (320, 320, 19)
        lengths = (1.0, 1.0, 0.06)
        widths = [320 // parts + (1 if k < 320 % parts else 0) for k in range(parts)]
        cuts = (tuple(int(v) for v in np.cumsum(widths)[:-1]), (), ())
        hy, hz = lengths[1] / ne[1], lengths[2] / ne[2]
        # tangential modes of an x-interface (Dirichlet edges): the lowest
        # sin(pi y / Ly) sin(pi z / Lz), the highest at the node spacing h/2
        kmin = float(np.pi * np.hypot(1.0 / lengths[1], 1.0 / lengths[2]))
        kmax = float(np.pi * np.hypot(2.0 / hy, 2.0 / hz))
        wl = Workload(name, ne, lengths, dirichlet, cuts, 8.0 * ne[0], 1e-6, seed, density="crater", n_blobs=10,
                      extra={"kmin": kmin, "kmax": kmax, "robin_kind": 2}, up=2)
    else:
        raise KeyError(name)
    for k, v in over.items():
        setattr(wl, k, v)
    return wl


def small(ne, nparts, p_times_h=8.0, bc=None, seed=0, tol=1e-10, density="blobs",
          lengths=(1.0, 1.0, 1.0), cuts=None):
    """A small test workload with equal (or given) cuts."""
    bc = bc if bc is not None else (DIRICHLET,) * 6
    if cuts is None:
        cuts = tuple(equal_cuts(n, k) for n, k in zip(ne, nparts))
    h = float(lengths[0]) / ne[0]
    return Workload("small", tuple(ne), tuple(lengths), tuple(bc), tuple(tuple(c) for c in cuts),
                    p_times_h / h, tol, seed, density=density, n_blobs=3)


WORKLOADS = ("c1", "c2", "c3", "c4", "c5", "c5copy", "slab32", "slab64", "slab128")
