"""Global stiffness, load and residual by element loops.

Test infrastructure (oracle). Weak form of the gravity equation of Sec. 2,
Delta(Phi) = -4 pi G drho, with homogeneous Dirichlet data (Sec. 3):
find u with  sum_e int_e grad u . grad v = 4 pi G sum_e int_e drho v  for all v.
The density anomaly is constant per element (its value at the element
centroid), so the load is f_i = 4 pi G sum_e drho_e int_e phi_i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe
from .mesh import BoxMesh


def assemble_stiffness(mesh: BoxMesh):
    """Sparse stiffness over all nodes (no boundary condition applied)."""
    Ke, _, _ = fe.element_matrices(mesh.h)
    conn = mesh.element_nodes()
    rows = np.repeat(conn, 27, axis=1).ravel()
    cols = np.tile(conn, (1, 27)).ravel()
    vals = np.tile(Ke.ravel(), mesh.n_elem)
    n = mesh.n_nodes
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def reduced_stiffness(mesh: BoxMesh):
    """Stiffness restricted to the unknown (non-Dirichlet) nodes."""
    K = assemble_stiffness(mesh)
    free = mesh.unknowns()
    return K[free][:, free].tocsr(), free


def apply_stiffness(mesh: BoxMesh, u_nodes):
    """K u over all nodes, element by element (no assembled matrix)."""
    Ke, _, _ = fe.element_matrices(mesh.h)
    conn = mesh.element_nodes()
    ue = u_nodes[conn]  # (n_elem, 27)
    ye = ue @ Ke.T
    return np.bincount(conn.ravel(), weights=ye.ravel(), minlength=mesh.n_nodes)


def load_from_density(mesh: BoxMesh, drho_elem, G):
    """f_i = 4 pi G sum_e drho_e int_e phi_i over all nodes."""
    _, _, le = fe.element_matrices(mesh.h)
    conn = mesh.element_nodes()
    w = (4.0 * np.pi * G) * np.asarray(drho_elem, float)[:, None] * le[None, :]
    return np.bincount(conn.ravel(), weights=w.ravel(), minlength=mesh.n_nodes)


def load_from_function(mesh: BoxMesh, fun, nq=3):
    """f_i = int fun(x) phi_i(x) dx by an nq^3 Gauss rule per element."""
    pts, w = fe.volume_rule(nq)
    phi, _ = fe.basis_3d(mesh.h, pts)
    vol = float(np.prod(mesh.h))
    conn = mesh.element_nodes()
    nx, ny, nz = mesh.ne
    hx, hy, hz = mesh.h
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    org = np.stack([ex.ravel() * hx, ey.ravel() * hy, ez.ravel() * hz], axis=1)
    X = org[:, None, :] + pts[None, :, :] * np.array(mesh.h)[None, None, :]
    fv = fun(X[..., 0], X[..., 1], X[..., 2])  # (n_elem, nq^3)
    contrib = (fv * (w * vol)[None, :]) @ phi.T  # (n_elem, 27)
    return np.bincount(conn.ravel(), weights=contrib.ravel(), minlength=mesh.n_nodes)


def residual_norm(mesh: BoxMesh, u_nodes, f_nodes):
    """||f - K u||_2 / ||f||_2 over the unknown nodes; u must vanish on
    Dirichlet nodes."""
    free = mesh.unknowns()
    r = f_nodes - apply_stiffness(mesh, u_nodes)
    return float(np.linalg.norm(r[free]) / np.linalg.norm(f_nodes[free]))


def interpolate(mesh: BoxMesh, u_nodes, pts_ref_fn=None, nq=4):
    """Values and gradients of the FE function at an nq^3 Gauss rule in every
    element: returns (X (n_elem, nq^3, 3), u, grad u, weights*vol)."""
    pts, w = fe.volume_rule(nq)
    phi, grad = fe.basis_3d(mesh.h, pts)
    conn = mesh.element_nodes()
    ue = u_nodes[conn]
    nx, ny, nz = mesh.ne
    hx, hy, hz = mesh.h
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    org = np.stack([ex.ravel() * hx, ey.ravel() * hy, ez.ravel() * hz], axis=1)
    X = org[:, None, :] + pts[None, :, :] * np.array(mesh.h)[None, None, :]
    uq = ue @ phi
    gq = np.einsum("ea,aqd->eqd", ue, grad)
    return X, uq, gq, w * float(np.prod(mesh.h))
