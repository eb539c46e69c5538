"""Seeded density-anomaly fields and random partitions.

All fields are returned per element, as the value of the field at the element
centroid, flattened with the element index ex + nx*(ey + ny*ez) (x fastest).
The paper's measured Chicxulub data is not available; these crater-like
synthetic anomalies (Gaussian blobs, horizontal layers and a buried ring) stand
in for it (Sec. 6 describes the real case only qualitatively).

Random draws use numpy.random.default_rng(seed) and happen in a fixed,
documented order so that every consumer sees the same field for a seed.
"""
from __future__ import annotations

import numpy as np


def element_centroids(ne, lengths):
    """Centroids of the nx*ny*nz box elements, shape (n_elem, 3), x fastest."""
    nx, ny, nz = (int(n) for n in ne)
    hx, hy, hz = (float(L) / n for L, n in zip(lengths, ne))
    cx = (np.arange(nx) + 0.5) * hx
    cy = (np.arange(ny) + 0.5) * hy
    cz = (np.arange(nz) + 0.5) * hz
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def blob_params(rng, n_blobs, lengths=(1.0, 1.0, 1.0)):
    """Draw n_blobs Gaussian blobs.

    Per blob, in this order: centre (3 draws, uniform in [0.2, 0.8] times the
    box length per axis), width sigma (uniform [0.05, 0.15]), amplitude
    magnitude (uniform [100, 500] kg/m^3), then its sign (integers(0, 2):
    0 -> +1, 1 -> -1).
    """
    L = np.asarray(lengths, float)
    blobs = []
    for _ in range(n_blobs):
        c = rng.uniform(0.2, 0.8, size=3) * L
        sigma = rng.uniform(0.05, 0.15)
        amp = rng.uniform(100.0, 500.0)
        sign = 1.0 - 2.0 * rng.integers(0, 2)
        blobs.append((c, sigma, sign * amp))
    return blobs


def _eval_blobs(xyz, blobs):
    out = np.zeros(xyz.shape[0])
    for c, sigma, amp in blobs:
        d2 = np.sum((xyz - c) ** 2, axis=1)
        out += amp * np.exp(-d2 / (2.0 * sigma * sigma))
    return out


def blobs_density(ne, lengths=(1.0, 1.0, 1.0), n_blobs=3, seed=0):
    """Sum of n_blobs random Gaussian blobs, per element (kg/m^3)."""
    rng = np.random.default_rng(seed)
    blobs = blob_params(rng, n_blobs, lengths)
    return _eval_blobs(element_centroids(ne, lengths), blobs)


def crater_density(ne, lengths=(1.0, 1.0, 1.0), seed=0, n_blobs=10, up=2):
    """Layered medium with a buried crater-like ring and random blobs.

    * three horizontal layers of equal thickness along the vertical axis `up`
      (z by default), each +-50 kg/m^3 with its sign drawn first (3 draws of
      integers(0, 2), bottom layer first);
    * a cylindrical ring 0.15 <= r <= 0.3 around the vertical axis through the
      box centre (r in units of the horizontal lengths), occupying the top 0.2
      of the box height, of -300 kg/m^3;
    * n_blobs Gaussian blobs drawn after the layer signs (see blob_params),
      their centres drawn in the frame whose third axis is vertical.
    """
    rng = np.random.default_rng(seed)
    signs = 1.0 - 2.0 * rng.integers(0, 2, size=3)
    order = [a for a in range(3) if a != up] + [up]   # horizontal, horizontal, vertical
    lengths = tuple(float(lengths[a]) for a in order)
    blobs = blob_params(rng, n_blobs, lengths)
    xyz = element_centroids(ne, [lengths[order.index(a)] for a in range(3)])[:, order]
    Lx, Ly, Lz = (float(v) for v in lengths)
    layer = np.minimum((xyz[:, 2] / Lz * 3.0).astype(int), 2)
    out = 50.0 * signs[layer]
    r = np.hypot(xyz[:, 0] / Lx - 0.5, xyz[:, 1] / Ly - 0.5)
    ring = (r >= 0.15) & (r <= 0.3) & (xyz[:, 2] >= 0.8 * Lz)
    out = out + np.where(ring, -300.0, 0.0)
    return out + _eval_blobs(xyz, blobs)


def uniform_density(ne, seed=0, lo=-300.0, hi=300.0):
    """Independent uniform values per element (a rough field for tests)."""
    rng = np.random.default_rng(seed)
    n = int(np.prod([int(v) for v in ne]))
    return rng.uniform(lo, hi, size=n)


def random_widths(rng, total, parts, lo, hi, max_draws=100000):
    """Subdomain widths (in elements) drawn i.i.d. uniform on {lo..hi}, the
    whole vector redrawn until it sums to `total`. Returns (widths, draws)."""
    for draw in range(1, max_draws + 1):
        w = rng.integers(lo, hi + 1, size=parts)
        if int(w.sum()) == total:
            return w.astype(np.int64), draw
    raise RuntimeError("random_widths: no admissible draw")


def widths_to_cuts(widths):
    """Interior cut positions (element indices) from a width vector."""
    return np.cumsum(np.asarray(widths, np.int64))[:-1]


def robin_candidates(n, h, seed=0):
    """Seeded candidate transmission coefficients for the batched search:
    p log-uniform on [h^-3/2, 10/h], q uniform on [0, h] (a log-uniform law on
    [0, h] does not exist). Returns (p, q), arrays of n values."""
    rng = np.random.default_rng(seed)
    lo, hi = np.log(h ** -1.5), np.log(10.0 / h)
    p = np.exp(rng.uniform(lo, hi, size=n))
    q = rng.uniform(0.0, h, size=n)
    return p, q
