"""Q2 Lagrange finite elements on axis-aligned boxes, by Gauss quadrature.

Test infrastructure (oracle). The paper uses "high order" finite elements
(abstract, Sec. 6) without naming the element; the reading taken here is the
27-node Q2 Lagrange hexahedron with 1D nodes {0, 1/2, 1} on the reference
interval. Every matrix is computed by quadrature of the weak form of the
Poisson problem of Sec. 2 (integral of grad(phi_a) . grad(phi_b), of
phi_a * phi_b and of phi_a), never from a closed form, so that closed forms can
be used as independent checks.

Local node numbering inside an element: a = ax + 3*ay + 9*az (x fastest),
with (ax, ay, az) in {0, 1, 2}^3 the position on the 1D node set.
"""
from __future__ import annotations

import numpy as np

NODES_1D = np.array([0.0, 0.5, 1.0])


def gauss_01(n):
    """n-point Gauss-Legendre rule mapped to [0, 1] (points, weights)."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_1d(t):
    """Values V[a, i] and derivatives D[a, i] (d/dt) of the three Q2 Lagrange
    polynomials of the nodes {0, 1/2, 1} at reference points t[i]."""
    t = np.atleast_1d(np.asarray(t, float))
    V = np.empty((3, t.size))
    D = np.empty((3, t.size))
    for a in range(3):
        others = [b for b in range(3) if b != a]
        denom = 1.0
        for b in others:
            denom *= NODES_1D[a] - NODES_1D[b]
        val = np.ones_like(t)
        for b in others:
            val = val * (t - NODES_1D[b])
        V[a] = val / denom
        der = np.zeros_like(t)
        for b in others:  # product rule over the two linear factors
            rest = np.ones_like(t)
            for c in others:
                if c != b:
                    rest = rest * (t - NODES_1D[c])
            der = der + rest
        D[a] = der / denom
    return V, D


def element_matrices_1d(h, nq=3):
    """1D element stiffness, mass and load on an interval of length h:
    K[a,b] = int L_a' L_b', M[a,b] = int L_a L_b, l[a] = int L_a."""
    t, w = gauss_01(nq)
    V, D = lagrange_1d(t)
    K = (D * w) @ D.T / h
    M = (V * w) @ V.T * h
    l = V @ w * h
    return K, M, l


def _local_index():
    idx = np.arange(27)
    return idx % 3, (idx // 3) % 3, idx // 9


def basis_3d(h, pts_ref):
    """Values phi[a, q] and physical gradients grad[a, q, d] of the 27 Q2 basis
    functions of a box element of size h at reference points pts_ref[q] in
    [0,1]^3."""
    hx, hy, hz = (float(v) for v in h)
    pts_ref = np.asarray(pts_ref, float)
    Vx, Dx = lagrange_1d(pts_ref[:, 0])
    Vy, Dy = lagrange_1d(pts_ref[:, 1])
    Vz, Dz = lagrange_1d(pts_ref[:, 2])
    ax, ay, az = _local_index()
    phi = Vx[ax] * Vy[ay] * Vz[az]
    grad = np.stack([Dx[ax] / hx * Vy[ay] * Vz[az],
                     Vx[ax] * Dy[ay] / hy * Vz[az],
                     Vx[ax] * Vy[ay] * Dz[az] / hz], axis=-1)
    return phi, grad


def volume_rule(nq):
    """Tensor Gauss rule on [0,1]^3: points (nq^3, 3), x fastest, and weights."""
    t, w = gauss_01(nq)
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    WZ, WY, WX = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return pts, (WX * WY * WZ).ravel()


def element_matrices(h, nq=3):
    """27x27 element stiffness K_e, mass M_e and load vector l_e = int phi_a
    of a box element of size h = (hx, hy, hz), by an nq^3 Gauss rule (nq = 3
    integrates every Q2 product exactly)."""
    pts, w = volume_rule(nq)
    vol = float(np.prod(h))
    phi, grad = basis_3d(h, pts)
    wq = w * vol
    K = np.einsum("aqd,bqd,q->ab", grad, grad, wq)
    M = np.einsum("aq,bq,q->ab", phi, phi, wq)
    l = phi @ wq
    return K, M, l


def face_mass_side(h, axis, side, nq=3):
    """int_F phi_a phi_b over the element face with normal `axis` located at
    reference coordinate `side` (0 or 1), by an nq x nq Gauss rule."""
    t, w = gauss_01(nq)
    T1, T0 = np.meshgrid(t, t, indexing="ij")
    W1, W0 = np.meshgrid(w, w, indexing="ij")
    tang = [d for d in range(3) if d != axis]
    pts = np.zeros((nq * nq, 3))
    pts[:, axis] = float(side)
    pts[:, tang[0]] = T0.ravel()
    pts[:, tang[1]] = T1.ravel()
    area = float(h[tang[0]]) * float(h[tang[1]])
    phi, _ = basis_3d(h, pts)
    wq = (W0 * W1).ravel() * area
    return np.einsum("aq,bq,q->ab", phi, phi, wq)


def face_stiffness_side(h, axis, side, nq=3):
    """int_F grad_t phi_a . grad_t phi_b over the element face with normal
    `axis` at reference coordinate `side`: the tangential (surface) stiffness
    of the second-order transmission operator (Sec. 3, read as p + q k^2)."""
    t, w = gauss_01(nq)
    T1, T0 = np.meshgrid(t, t, indexing="ij")
    W1, W0 = np.meshgrid(w, w, indexing="ij")
    tang = [d for d in range(3) if d != axis]
    pts = np.zeros((nq * nq, 3))
    pts[:, axis] = float(side)
    pts[:, tang[0]] = T0.ravel()
    pts[:, tang[1]] = T1.ravel()
    area = float(h[tang[0]]) * float(h[tang[1]])
    _, grad = basis_3d(h, pts)
    gt = grad[:, :, tang]  # tangential components only
    wq = (W0 * W1).ravel() * area
    return np.einsum("aqd,bqd,q->ab", gt, gt, wq)
