"""Robin-augmented subdomain problems, by element and face-element loops.

Test infrastructure (oracle). On subdomain s the Schwarz step of Sec. 3 solves
the Poisson problem with a Robin condition d_n u + p u = g on every interface
face (the zeroth-order transmission operator A = p of Sec. 3) and the outer
boundary conditions elsewhere. Its weak form gives

    A_s = K_s^N + sum over interface faces F of s of  p_F * M_F,

with K_s^N the stiffness assembled from s's own elements over s's closure
(natural/Neumann on interfaces) and M_F = int_F phi_i phi_j the face mass
matrix, both restricted to s's unknowns. The right-hand side is
f_s + sum_F R_F^T lambda_F with f_s the load of s's own elements and
lambda_F = M_F g_F the discrete Robin datum on F.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe
from .partition import BoxPartition, Subdomain, Face


def _local_map(part: BoxPartition, sub: Subdomain):
    loc = -np.ones(part.mesh.n_nodes, np.int64)
    loc[part.local_nodes(sub)] = np.arange(sub.n)
    return loc


def _scatter(elem_conn, loc, Me, n):
    rows = loc[np.repeat(elem_conn, 27, axis=1)].ravel()
    cols = loc[np.tile(elem_conn, (1, 27))].ravel()
    vals = np.tile(Me.ravel(), elem_conn.shape[0])
    keep = (rows >= 0) & (cols >= 0) & (vals != 0.0)
    return sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n))


def neumann_stiffness(part: BoxPartition, sub: Subdomain):
    """K_s^N: stiffness of s's own elements on s's unknowns."""
    Ke, _, _ = fe.element_matrices(part.mesh.h)
    conn = part.mesh.element_nodes()[part.elements_of(sub)]
    return _scatter(conn, _local_map(part, sub), Ke, sub.n)


def face_elements(part: BoxPartition, face: Face):
    """Elements of s that have a face on the interface `face`."""
    sub = part.subs[face.s]
    e = part.elements_of(sub)
    nx, ny, _ = part.mesh.ne
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    coord = (ex, ey, ez)[face.axis]
    target = sub.e0[face.axis] if face.side == 0 else sub.e1[face.axis] - 1
    return e[coord == target]


def face_mass_local(part: BoxPartition, face: Face):
    """M_F restricted to the face's own node list (face.nodes order)."""
    Mf = fe.face_mass_side(part.mesh.h, face.axis, face.side)
    conn = part.mesh.element_nodes()[face_elements(part, face)]
    loc = -np.ones(part.mesh.n_nodes, np.int64)
    loc[face.nodes] = np.arange(face.nodes.size)
    return _scatter(conn, loc, Mf, face.nodes.size)


def face_stiffness_local(part: BoxPartition, face: Face):
    """K_F = int_F grad_t phi_i . grad_t phi_j restricted to the face's node
    list (natural condition at the face's edges)."""
    Kf = fe.face_stiffness_side(part.mesh.h, face.axis, face.side)
    conn = part.mesh.element_nodes()[face_elements(part, face)]
    loc = -np.ones(part.mesh.n_nodes, np.int64)
    loc[face.nodes] = np.arange(face.nodes.size)
    return _scatter(conn, loc, Kf, face.nodes.size)


def face_operator_local(part: BoxPartition, face: Face, p, q=0.0):
    """The discrete transmission operator p M_F + q K_F of one face."""
    A = p * face_mass_local(part, face)
    if q != 0.0:
        A = A + q * face_stiffness_local(part, face)
    return A.tocsr()


def face_restriction(part: BoxPartition, face: Face):
    """Indices into s's local vector of the face nodes, in face order."""
    loc = _local_map(part, part.subs[face.s])
    idx = loc[face.nodes]
    assert np.all(idx >= 0)
    return idx


def robin_matrix(part: BoxPartition, sub: Subdomain, p_face, q_face=None):
    """A_s = K_s^N + sum_F R_F^T (p_F M_F + q_F K_F) R_F. p_face(face) and
    q_face(face) give the coefficients of the directed face (s <- j)."""
    A = neumann_stiffness(part, sub)
    for f in part.faces:
        if f.s != sub.s:
            continue
        R = face_restriction(part, f)
        P = sp.csr_matrix((np.ones(R.size), (R, np.arange(R.size))), shape=(sub.n, R.size))
        q = 0.0 if q_face is None else q_face(f)
        A = A + P @ face_operator_local(part, f, p_face(f), q) @ P.T
    return A.tocsr()


def density_load(part: BoxPartition, sub: Subdomain, drho_elem, G):
    """f_s: load of s's own elements, on s's unknowns."""
    _, _, le = fe.element_matrices(part.mesh.h)
    el = part.elements_of(sub)
    conn = part.mesh.element_nodes()[el]
    loc = _local_map(part, sub)
    w = (4.0 * np.pi * G) * np.asarray(drho_elem, float)[el][:, None] * le[None, :]
    idx = loc[conn].ravel()
    keep = idx >= 0
    return np.bincount(idx[keep], weights=w.ravel()[keep], minlength=sub.n)


def split_load(part: BoxPartition, f_nodes):
    """f_s = f / multiplicity on s's unknowns (a nodal load split evenly among
    the subdomain copies of each node); sum_s R_s^T f_s = f."""
    m = part.multiplicity()
    return [f_nodes[part.local_nodes(sub)] / m[part.local_nodes(sub)] for sub in part.subs]
