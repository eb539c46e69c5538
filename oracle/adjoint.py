"""Surface gravity misfit and its gradient with respect to the density.

Test infrastructure (oracle). The potential of Sec. 2 depends linearly on the
density anomaly: Phi = K^-1 f, f = 4 pi G B drho with B_ie = int_e phi_i.
For the misfit J = 1/2 sum_i (Phi(x_i) - d_i)^2 at observation points x_i,
Phi(x_i) = (P Phi)_i with P the Q2 interpolation at the points, so

    dJ/ddrho = 4 pi G B^T psi,   K psi = P^T (P Phi - d)   (K symmetric),

the global direct adjoint. Everything here uses the oracle's own element
routines and direct solvers.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe
from .assemble import load_from_density
from .direct import solve_direct
from .mesh import BoxMesh


def observation_operator(mesh: BoxMesh, pts):
    """Sparse P (n_pts x n_nodes): Q2 interpolation of nodal values at pts.
    A point on an element boundary is assigned to the element on its lower
    side (the higher one at the upper box face)."""
    pts = np.asarray(pts, float)
    rows, cols, vals = [], [], []
    conn = mesh.element_nodes()
    nx, ny, nz = mesh.ne
    for i, x in enumerate(pts):
        e, ref = [], []
        for d in range(3):
            t = x[d] / mesh.h[d]
            k = min(int(np.floor(t)), mesh.ne[d] - 1)
            e.append(k)
            ref.append(t - k)
        el = e[0] + nx * (e[1] + ny * e[2])
        Vx, _ = fe.lagrange_1d([ref[0]])
        Vy, _ = fe.lagrange_1d([ref[1]])
        Vz, _ = fe.lagrange_1d([ref[2]])
        for a in range(27):
            w = Vx[a % 3, 0] * Vy[(a // 3) % 3, 0] * Vz[a // 9, 0]
            if w != 0.0:
                rows.append(i)
                cols.append(conn[el, a])
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(pts), mesh.n_nodes))


def top_face_points(n, lengths=(1.0, 1.0, 1.0)):
    """n x n observation points ((i+1/2)/n, (j+1/2)/n) on the top face z = Lz,
    i fastest."""
    c = (np.arange(n) + 0.5) / n
    Y, X = np.meshgrid(c, c, indexing="ij")
    return np.stack([X.ravel() * lengths[0], Y.ravel() * lengths[1],
                     np.full(n * n, float(lengths[2]))], axis=1)


def forward(mesh: BoxMesh, drho, G, method="auto"):
    return solve_direct(mesh, load_from_density(mesh, drho, G), method)


def misfit(P, phi, d):
    r = P @ phi - d
    return 0.5 * float(r @ r)


def density_transpose(mesh: BoxMesh, psi, G):
    """(4 pi G B^T psi)_e = 4 pi G sum_a psi_a int_e phi_a, element by element."""
    _, _, le = fe.element_matrices(mesh.h)
    return (4.0 * np.pi * G) * (psi[mesh.element_nodes()] @ le)


def gradient_direct(mesh: BoxMesh, P, drho, d, G, method="auto"):
    """dJ/ddrho by the global direct adjoint. Returns (grad, phi, psi)."""
    phi = forward(mesh, drho, G, method)
    g = P.T @ (P @ phi - d)
    psi = solve_direct(mesh, np.asarray(g).ravel(), method)
    return density_transpose(mesh, psi, G), phi, psi
