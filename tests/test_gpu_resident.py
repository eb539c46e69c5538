"""The FP32 fused CG kernel with the direction p and the correction x (or x
alone) resident in LDS (needs an MI355X).

Each node's p and x are read and written only by the thread that owns the
node, in the same order and precision as through global memory, so a solve
with resident p and x must reproduce the other form bit for bit; the oracle
then checks the result itself.
"""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import assemble as A
from oracle import schwarz as S
from synth.generators import uniform_density
from synth import workload

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

PLANE33 = dict(ne=(32, 16, 6), bc=(1, 1, 1, 1, 0, 0), cuts=((16,), (), (3,)), p=200.0)
# 33x33x31-node subdomains: p and x need 270 KB with the march planes, x alone 152 KB
TALL33 = dict(ne=(32, 16, 16), bc=(1, 1, 1, 1, 0, 0), cuts=((16,), (), ()), p=200.0)


def _torch():
    import torch
    return torch


# (case, block, team, wave_rows, residency level when allowed: 1 p and x, 2 x)
SOLVES = {
    "c1_team1": ("c1", 256, 1, 0, 1),
    "c1_team4": ("c1", 256, 4, 0, 1),
    "c1_team2_wave_rows": ("c1", 384, 2, 1, 1),
    "plane33_team2": (PLANE33, 576, 2, 0, 1),
    "plane33_cols3_wave_rows": (PLANE33, 448, 1, 1, 1),
    "tall33_x_alone": (TALL33, 576, 1, 0, 2),
    "tall33_team2": (TALL33, 576, 2, 0, 1),
}


def _case(spec):
    if spec == "c1":
        wl = workload("c1", seed=0)
        return Case.from_workload(wl), wl.drho(), wl.tol
    case = Case(**spec)
    return case, uniform_density(case.ne, seed=7), 1e-8


@pytest.mark.parametrize("name", sorted(SOLVES))
def test_resident_solve_is_bitwise_the_global_one(name):
    torch = _torch()
    spec, block, team, rows, level = SOLVES[name]
    case, drho, tol = _case(spec)
    f, _ = case.density_loads(drho)
    d = torch.tensor(drho, device="cuda")
    out = {}
    for res in (0, 1):
        prob = case.problem(precision="fp32", mode="batched", block=block, team=team, wave_rows=rows, resident=res)
        phi, st = prob.solve(d, tol)
        assert st["resident"] == (level if res else 0) and st["team"] == team and st["converged"], (name, res, st)
        out[res] = (phi.cpu().numpy(), st)
        prob.close()
    (p0, s0), (p1, s1) = out[0], out[1]
    assert s0["outer_iters"] == s1["outer_iters"] and s0["inner_iters"] == s1["inner_iters"], name
    diff = np.abs(p0 - p1).max() / np.abs(p0).max()
    print(name, "max relative difference", diff, flush=True)
    assert diff == 0.0, name
    assert A.residual_norm(case.mesh, p1, f) <= tol * 1.001


def test_resident_one_outer_iteration_matches_oracle():
    """One outer iteration from a random state with a tight inner tolerance:
    the FP32 inner solves with resident p and x reach the oracle's exact
    subdomain solves to FP32 accuracy."""
    torch = _torch()
    case = Case(**PLANE33)
    prob = case.problem(precision="fp32", mode="batched", inner_tol=1e-6, inner_abs=0.0, max_inner=4000,
                        block=576, team=2, resident=1)
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
    u1, _ = prob.get_state()
    u1 = case.from_local(lay, u1.cpu().numpy())
    orc = S.SchwarzOracle(case.part, case.p, "lu")
    ur = orc.subdomain_solves(fs, lam0)
    for s in range(case.part.n_sub):
        assert np.abs(u1[s] - ur[s]).max() <= 1e-4 * np.abs(ur[s]).max(), s


def test_resident_falls_back_where_p_and_x_do_not_fit():
    """33x33x39-node subdomains in one block need 186 KB for x alone with the
    march planes: the kernel keeps p and x in global memory and still solves."""
    torch = _torch()
    case = Case(ne=(32, 16, 20), bc=(1, 1, 1, 1, 0, 0), cuts=((16,), (), ()), p=200.0)
    assert all(s.shape == (33, 33, 39) for s in case.part.subs)
    drho = uniform_density(case.ne, seed=1)
    f, _ = case.density_loads(drho)
    prob = case.problem(precision="fp32", mode="batched", block=576, team=1, resident=1)
    phi, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-8)
    assert st["resident"] == 0 and st["converged"]
    assert A.residual_norm(case.mesh, phi.cpu().numpy(), f) <= 1e-8 * 1.001
