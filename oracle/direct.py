"""Direct solvers: sparse LU, and fast diagonalisation for box problems.

Test infrastructure (oracle). Sparse LU (SuperLU through SciPy) is the plain
method for small problems. For large constant-coefficient box problems the
matrix is a Kronecker sum of 1D factors,

    A = (Kx + Ex) (x) My (x) Mz + Mx (x) (Ky + Ey) (x) Mz + Mx (x) My (x) (Kz + Ez),

(an identity of tensor-product elements that the tests check against the
3D-quadrature assembly), and is inverted exactly with the generalised
eigenpairs (K_d + E_d) V_d = M_d V_d Lambda_d, V_d^T M_d V_d = I:

    A^{-1} = (Vz (x) Vy (x) Vx) diag(1 / (lx_a + ly_b + lz_c)) (Vz (x) Vy (x) Vx)^T.

The 1D factors are assembled here from the oracle's own 1D element matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe
from .assemble import reduced_stiffness
from .mesh import BoxMesh, DIRICHLET


def lu_factor(A):
    return spla.splu(sp.csc_matrix(A))


def solve_lu(A, b):
    return lu_factor(A).solve(np.asarray(b, float))


def assemble_1d(n_elem, h, keep_lo, keep_hi, end_lo=0.0, end_hi=0.0):
    """1D stiffness and mass over n_elem Q2 elements of size h (2n_elem+1
    nodes), restricted to node indices keep_lo..keep_hi, with end_lo/end_hi
    added to the stiffness diagonal at the first/last node of the interval
    (a Robin coefficient at an interface end)."""
    k1, m1, _ = fe.element_matrices_1d(h)
    n = 2 * n_elem + 1
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    for e in range(n_elem):
        i = slice(2 * e, 2 * e + 3)
        K[i, i] += k1
        M[i, i] += m1
    K[0, 0] += end_lo
    K[n - 1, n - 1] += end_hi
    sel = slice(keep_lo, keep_hi + 1)
    return K[sel, sel], M[sel, sel]


class FDM:
    """Exact inverse of a Kronecker-sum operator from its three 1D factors."""

    def __init__(self, factors):
        self.V = []
        self.lam = []
        for K, M in factors:  # x, y, z
            lam, V = sla.eigh(K, M)
            self.V.append(V)
            self.lam.append(lam)
        lx, ly, lz = self.lam
        self.denom = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
        self.shape = tuple(V.shape[0] for V in self.V)

    def solve(self, b):
        nx, ny, nz = self.shape
        Vx, Vy, Vz = self.V
        B = np.asarray(b, float).reshape(nz, ny, nx)
        T = np.einsum("zyx,xa->zya", B, Vx)
        T = np.einsum("zya,yb->zba", T, Vy)
        T = np.einsum("zba,zc->cba", T, Vz)
        T = T / self.denom
        T = np.einsum("cba,zc->zba", T, Vz)
        T = np.einsum("zba,yb->zya", T, Vy)
        T = np.einsum("zya,xa->zyx", T, Vx)
        return T.ravel()


def global_fdm(mesh: BoxMesh):
    """FDM for the global Dirichlet-reduced stiffness of a box mesh."""
    fac = []
    for d in range(3):
        lo = 1 if mesh.bc[2 * d] == DIRICHLET else 0
        hi = 2 * mesh.ne[d] - (1 if mesh.bc[2 * d + 1] == DIRICHLET else 0)
        fac.append(assemble_1d(mesh.ne[d], mesh.h[d], lo, hi))
    return FDM(fac)


def solve_direct(mesh: BoxMesh, f_nodes, method="auto"):
    """Global Galerkin solution u = K^{-1} f on the unknowns; returns nodal
    values over all nodes (0 on Dirichlet nodes)."""
    free = mesh.unknowns()
    if method == "auto":
        method = "lu" if free.size <= 60000 else "fdm"
    u = np.zeros(mesh.n_nodes)
    if method == "lu":
        K, free = reduced_stiffness(mesh)
        u[free] = solve_lu(K, f_nodes[free])
    elif method == "fdm":
        u[free] = global_fdm(mesh).solve(f_nodes[free])
    else:
        raise ValueError(method)
    return u
