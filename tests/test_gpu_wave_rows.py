"""The fused CG kernel with wave-owned rows (each wave of a block owns whole
x-rows of the plane, one workgroup barrier per plane) against the oracle
(needs an MI355X).

The operator and the CG recurrences are the same as in the other block
mapping; only the thread that computes a node changes, so one outer
iteration must reproduce the oracle's exact subdomain solves, and whole
solves must reach the solution of the other mapping.
"""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import assemble as A
from oracle import schwarz as S
from synth.generators import uniform_density
from synth import workload

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _torch():
    import torch
    return torch


# Unknowns of a subdomain exclude Dirichlet nodes; with Neumann x and y faces
# the 32x16x6 mesh cut at x = 16 has 33x33-node planes.
PLANE33 = dict(ne=(32, 16, 6), bc=(1, 1, 1, 1, 0, 0), cuts=((16,), (), (3,)), p=200.0)
# (case, block, team): planes of one wave (at most 7x7 nodes), of exactly 11
# waves of 3 rows (33x33 nodes, two columns per thread), 7 waves of 5 rows
# (three columns) and 5 waves of 7 rows (four columns); ragged cuts, Neumann
# faces
CASES = {
    "small_team1": (dict(ne=(6, 5, 6), bc=(0, 0, 1, 0, 0, 0), cuts=((3,), (2,), (2, 4)), p=11.0), 64, 1),
    "small_team2": (dict(ne=(6, 5, 6), bc=(0, 0, 1, 0, 0, 0), cuts=((3,), (2,), (2, 4)), p=11.0), 64, 2),
    "plane33_cols2": (PLANE33, 704, 1),
    "plane33_cols3_team2": (PLANE33, 448, 2),
    "plane33_cols4": (PLANE33, 320, 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_one_outer_iteration_with_wave_rows_matches_oracle(name):
    """u^1 = A_s^-1 (f_s + sum R^T lambda^0) and lambda^1 from a random state,
    FP64 fused kernel with wave-owned rows, against the oracle's LU solves."""
    torch = _torch()
    kw, block, team = CASES[name]
    case = Case(**kw)
    prob = case.problem(precision="fp64", mode="batched", inner_tol=1e-30, inner_abs=1e-14, max_inner=4000,
                        block=block, team=team, wave_rows=1)
    lay = case.check_layout(prob)
    drho = uniform_density(case.ne, seed=3)
    f, fs = case.density_loads(drho)
    rng = np.random.default_rng(5)
    u0 = [1e-9 * rng.standard_normal(s.n) for s in case.part.subs]
    lam0 = [1e-10 * rng.standard_normal(fc.nodes.size) for fc in case.part.faces]
    prob.set_density(torch.tensor(drho, device="cuda"))
    prob.set_state(torch.tensor(case.to_local(lay, u0), device="cuda"),
                   torch.tensor(case.faces_to_lam(lay, lam0), device="cuda"))
    prob.iterate(1)
    u1, lam1 = prob.get_state()
    u1 = case.from_local(lay, u1.cpu().numpy())
    lam1 = case.lam_to_faces(lay, lam1.cpu().numpy())
    orc = S.SchwarzOracle(case.part, case.p, "lu")
    ur = orc.subdomain_solves(fs, lam0)
    lr = orc.exchange(ur, lam0)
    eu = max(np.abs(u1[s] - ur[s]).max() / np.abs(ur[s]).max() for s in range(case.part.n_sub))
    el = max(np.abs(lam1[fc] - lr[fc]).max() / np.abs(lr[fc]).max() for fc in range(len(lr)))
    print("max rel error: u", eu, "lambda", el, flush=True)
    for s in range(case.part.n_sub):
        assert np.abs(u1[s] - ur[s]).max() <= 1e-10 * np.abs(ur[s]).max(), (name, s)
    for fc in range(len(lr)):
        assert np.abs(lam1[fc] - lr[fc]).max() <= 1e-10 * np.abs(lr[fc]).max(), (name, fc)


@pytest.mark.parametrize("team", [1, 4])
def test_wave_rows_solve_matches_other_mapping(team):
    """Whole FP32-inner solves of the 16^3 workload (16x16-node planes, one
    column per thread, 4 rows per wave, two idle waves): same iteration count
    within 2 %, the oracle's residual below the tolerance and the same
    solution."""
    torch = _torch()
    wl = workload("c1", seed=0)
    case = Case.from_workload(wl)
    drho = torch.tensor(wl.drho(), device="cuda")
    f, _ = case.density_loads(wl.drho())
    ref = case.problem(precision="fp32", mode="batched", team=team, block=320)
    p1, s1 = ref.solve(drho, wl.tol)
    rows = case.problem(precision="fp32", mode="batched", team=team, block=384, wave_rows=1)
    p2, s2 = rows.solve(drho, wl.tol)
    assert s2["wave_rows"] == 1 and s1["wave_rows"] == 0 and s2["team"] == team and s2["converged"]
    res = A.residual_norm(case.mesh, p2.cpu().numpy(), f)
    assert res <= wl.tol * 1.001
    assert abs(s2["outer_iters"] - s1["outer_iters"]) <= 0.02 * s1["outer_iters"]
    assert (p1 - p2).abs().max().item() <= 1e-6 * p1.abs().max().item()


def test_wave_rows_that_cannot_cover_the_plane_are_rejected():
    """10 waves of 3 rows cannot cover a 33-row plane: EINVAL at setup."""
    from paper_2112_03851_amd.sos import SosError
    case = Case(**PLANE33)
    assert all(s.shape[:2] == (33, 33) for s in case.part.subs)
    with pytest.raises(SosError):
        case.problem(precision="fp32", mode="batched", block=640, wave_rows=1)
