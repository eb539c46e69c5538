"""Test helpers: build the oracle's view and the library's view of one workload
and move per-subdomain vectors between the two layouts (test infrastructure)."""
from __future__ import annotations

import numpy as np

from oracle import assemble as A
from oracle import mesh as M
from oracle import partition as P
from oracle import subdomain as SD


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


class Case:
    def __init__(self, ne, lengths=(1.0, 1.0, 1.0), bc=(0,) * 6, cuts=((), (), ()), p=8.0, G=6.672e-11):
        self.ne, self.lengths, self.bc, self.cuts, self.p, self.G = tuple(ne), tuple(lengths), tuple(bc), cuts, p, G
        self.mesh = M.BoxMesh(ne, lengths, bc)
        self.part = P.BoxPartition(self.mesh, cuts)

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.ne, wl.lengths, wl.bc, wl.cuts, wl.p, wl.G)

    def problem(self, **kw):
        from paper_2112_03851_amd.sos import Problem
        kw.setdefault("p", self.p)
        return Problem(self.ne, self.lengths, self.bc, cuts=self.cuts, **kw)

    def check_layout(self, prob):
        lay = prob.layout()
        assert len(lay["dims"]) == self.part.n_sub
        for s, sub in enumerate(self.part.subs):
            perm = lay["perm"][s]
            assert sorted(perm.tolist()) == [0, 1, 2], perm
            assert tuple(lay["dims"][s]) == tuple(sub.shape[g] for g in perm), (s, lay["dims"][s], sub.shape, perm)
            assert tuple(lay["lo"][s]) == sub.lo
        f = prob.faces()
        assert len(f) == len(self.part.faces)
        for a, b in zip(f, self.part.faces):
            assert tuple(a) == (b.s, b.j, b.axis, b.side)
        return lay

    @staticmethod
    def _axes(perm):
        """numpy axes that take an (nz, ny, nx) array (x fastest) to the local
        order (local axis 0 fastest): local axis a is global axis perm[a]."""
        return [2 - int(perm[2]), 2 - int(perm[1]), 2 - int(perm[0])]

    def to_local(self, lay, parts, dtype=np.float64):
        out = np.zeros(int(lay["offsets"][-1]), dtype)
        for s, v in enumerate(parts):
            sub = self.part.subs[s]
            nx, ny, nz = sub.shape
            v = np.transpose(np.asarray(v).reshape(nz, ny, nx), self._axes(lay["perm"][s])).ravel()
            o = int(lay["offsets"][s])
            out[o:o + v.size] = v
        return out

    def from_local(self, lay, vec):
        out = []
        for s, sub in enumerate(self.part.subs):
            perm = lay["perm"][s]
            o = int(lay["offsets"][s])
            loc = np.asarray(vec[o:o + sub.n]).reshape(*[sub.shape[g] for g in perm[::-1]])
            out.append(np.transpose(loc, np.argsort(self._axes(perm))).ravel())
        return out

    def lam_to_faces(self, lay, lam):
        fo = lay["face_off"]
        return [np.asarray(lam[int(fo[f]):int(fo[f + 1])]) for f in range(len(self.part.faces))]

    def faces_to_lam(self, lay, lam_faces):
        out = np.zeros(int(lay["face_off"][-1]))
        for f, v in enumerate(lam_faces):
            out[int(lay["face_off"][f]):int(lay["face_off"][f + 1])] = v
        return out

    def density_loads(self, drho):
        f = A.load_from_density(self.mesh, drho, self.G)
        fs = [SD.density_load(self.part, s, drho, self.G) for s in self.part.subs]
        return f, fs
