"""The non-overlapping Robin-Schwarz iteration with exact subdomain solves.

Test infrastructure (oracle). Sec. 3 states the method for two subdomains
(Jacobi order: iterate n+1 on one side uses iterate n of the other side).
Reading for many subdomains: one Robin datum per directed interface face.
With g_{s<-j} the Robin datum d_n u_s + p_sj u_s that s receives from j and
lambda = M_F g its discrete (face-mass weighted) form:

  1. lambda^0 = 0 on every directed face, u^0 = 0.
  2. for every s, solve exactly  A_s u_s = f_s + sum_j R_sj^T lambda_{s<-j}.
  3. for every directed face,
         lambda_{j<-s} <- -lambda_{s<-j} + (A_sj + A_js) R_sj u_s,
     A = p M_F (zeroth order) or p M_F + q K_F (second order, K_F the
     tangential face stiffness),
     the discrete form of d_{n_j} u + p_js u = -(d_{n_s} u_s + p_sj u_s)
     + (p_sj + p_js) u_s on the shared face (n_j = -n_s), where s's normal
     flux is read off its own Robin condition.
  4. u~ = average of the subdomain copies of every node; stop when
     ||f - K u~||_2 / ||f||_2 <= tol over the unknowns (the stopping
     threshold of Sec. 6, with the global residual as the reading of it).

At a fixed point lambda_{s<-j} + lambda_{j<-s} = (p_sj + p_js) M_F u_s =
(p_sj + p_js) M_F u_j, so the copies agree and summing the subdomain problems
gives the global Galerkin system K u = f.
"""
from __future__ import annotations

import numpy as np

from . import subdomain as sd
from .assemble import residual_norm
from .direct import FDM, assemble_1d, lu_factor
from .partition import BoxPartition


class SchwarzOracle:
    def __init__(self, part: BoxPartition, p_face, solver="auto", q_face=0.0):
        """p_face, q_face: float (same value on every directed face) or a
        callable face -> value; q > 0 selects the second-order transmission
        operator p M_F + q K_F (then only 'lu' applies). solver: 'lu', 'fdm' or
        'auto' (LU up to 20000 unknowns)."""
        self.part = part
        self.mesh = part.mesh
        as_arr = lambda v: (np.array([float(v(f)) for f in part.faces]) if callable(v)
                            else np.full(len(part.faces), float(v)))
        self.p = as_arr(p_face)
        self.q = as_arr(q_face)
        if np.any(self.p <= 0) or np.any(self.q < 0):
            raise ValueError("Robin coefficients must satisfy p > 0, q >= 0")
        if np.any(self.q > 0) and solver == "fdm":
            raise ValueError("second-order conditions are not a Kronecker sum: use LU")
        if np.any(self.q > 0):
            solver = "lu"
        self.opp = np.array([part.face_index[(f.j, f.s)] for f in part.faces], np.int64)
        self.R = [sd.face_restriction(part, f) for f in part.faces]
        self.M = [sd.face_mass_local(part, f).tocsr() for f in part.faces]
        self.KF = [sd.face_stiffness_local(part, f).tocsr() if np.any(self.q > 0) else None for f in part.faces]
        self.nodes = [part.local_nodes(s) for s in part.subs]
        self.mult = part.multiplicity()
        self.faces_of = [[f.index for f in part.faces if f.s == s.s] for s in part.subs]
        self.solvers = []
        cache = {}
        for sub in part.subs:
            kind = solver
            if kind == "auto":
                kind = "lu" if sub.n <= 20000 else "fdm"
            if kind == "lu":
                A = sd.robin_matrix(part, sub, lambda f: self.p[f.index], lambda f: self.q[f.index])
                self.solvers.append(lu_factor(A).solve)
            elif kind == "fdm":
                key, fac = self._fdm_factors(sub)
                if key not in cache:
                    cache[key] = FDM(fac)
                self.solvers.append(cache[key].solve)
            else:
                raise ValueError(solver)

    def _fdm_factors(self, sub):
        fac, key = [], []
        for d in range(3):
            ends = []
            for side in (0, 1):
                j = sub.neighbor.get((d, side))
                ends.append(0.0 if j is None else self.p[self.part.face_index[(sub.s, j)]])
            ne = sub.e1[d] - sub.e0[d]
            klo, khi = sub.lo[d] - 2 * sub.e0[d], sub.hi[d] - 2 * sub.e0[d]
            fac.append(assemble_1d(ne, self.mesh.h[d], klo, khi, ends[0], ends[1]))
            key.append((ne, self.mesh.h[d], klo, khi, ends[0], ends[1]))
        return tuple(key), fac

    def local_rhs(self, f_sub, lam):
        out = []
        for s, fs in enumerate(f_sub):
            b = np.array(fs, float, copy=True)
            for fi in self.faces_of[s]:
                np.add.at(b, self.R[fi], lam[fi])
            out.append(b)
        return out

    def subdomain_solves(self, f_sub, lam):
        return [self.solvers[s](b) for s, b in enumerate(self.local_rhs(f_sub, lam))]

    def exchange(self, u, lam):
        """Returns the new Robin data from the subdomain solutions u."""
        new = [None] * len(lam)
        for g, face in enumerate(self.part.faces):
            f = self.opp[g]  # face (s <- j) with s = face.j: the sender
            us = u[face.j][self.R[f]]
            new[g] = -lam[f] + (self.p[g] + self.p[f]) * (self.M[g] @ us)
            if self.q[g] + self.q[f] > 0:
                new[g] = new[g] + (self.q[g] + self.q[f]) * (self.KF[g] @ us)
        return new

    def glue(self, u):
        U = np.zeros(self.mesh.n_nodes)
        for s, us in enumerate(u):
            U[self.nodes[s]] += us
        nz = self.mult > 0
        U[nz] /= self.mult[nz]
        return U

    def zero_data(self):
        return [np.zeros(f.nodes.size) for f in self.part.faces]

    def solve(self, f_sub, f_nodes, tol, max_outer=10000, check_every=1, lam=None,
              history=False):
        """Run the iteration until the global relative residual <= tol.
        Returns (u_nodes, outer_iterations, residual, history list)."""
        lam = self.zero_data() if lam is None else lam
        hist = []
        res = np.inf
        U = np.zeros(self.mesh.n_nodes)
        n = 0
        for n in range(1, max_outer + 1):
            u = self.subdomain_solves(f_sub, lam)
            lam = self.exchange(u, lam)
            if n % check_every == 0 or n == max_outer:
                U = self.glue(u)
                res = residual_norm(self.mesh, U, f_nodes)
                if history:
                    hist.append((n, res))
                if res <= tol:
                    break
        return U, n, res, hist
