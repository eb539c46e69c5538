"""Subdomains marched along x or y instead of z (needs an MI355X): the local
layout follows each subdomain's axis order, and every step that maps local
nodes to global ones (loads, copies, Robin data, exchange, assembly) goes
through it. Against the oracle: the operator apply, one outer iteration with
cross points and Neumann faces, the fixed point, and the paper's x-slabs of a
thin vertical box, whose x-y node planes are too large to march along z."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import assemble as A
from oracle import direct as D
from oracle import schwarz as S
from oracle import subdomain as SD
from paper_2112_03851_amd.sos import optimize_robin
from synth.generators import crater_density, uniform_density

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CASES = {
    "mixed_bc_ragged": dict(ne=(7, 6, 5), lengths=(1.0, 0.8, 1.3), bc=(0, 1, 0, 0, 1, 0),
                            cuts=((2, 3), (4,), (1,)), p=5.5),
    "thin_columns": dict(ne=(12, 10, 20), cuts=((2, 5, 9), (3, 7), ()), p=96.0),
}


@pytest.mark.parametrize("march", [1, 2])
@pytest.mark.parametrize("q", [0.0, 0.013])
@pytest.mark.parametrize("name", sorted(CASES))
def test_apply_with_forced_march_axis(name, q, march):
    import torch
    case = Case(**CASES[name])
    print("case", name, "q", q, "march", march, flush=True)
    prob = case.problem(q=q, march=march)
    lay = case.check_layout(prob)
    assert all(int(p[2]) == march - 1 for p in lay["perm"])
    rng = np.random.default_rng(13)
    xs = [rng.standard_normal(s.n) for s in case.part.subs]
    x = torch.tensor(case.to_local(lay, xs), device="cuda")
    y64 = case.from_local(lay, prob.apply_local(x).cpu().numpy())
    y32 = case.from_local(lay, prob.apply_local(x.float()).double().cpu().numpy())
    for s, sub in enumerate(case.part.subs):
        As = SD.robin_matrix(case.part, sub, lambda f: case.p, lambda f: q)
        ref = As @ xs[s]
        scale = np.abs(As).max() * np.abs(xs[s]).max()
        assert np.abs(y64[s] - ref).max() <= 1e-14 * scale * 8, (name, s)
        assert np.abs(y32[s] - ref).max() <= 2e-6 * scale * 8, (name, s)
    prob.close()


@pytest.mark.parametrize("mode", ["stepwise", "batched"])
@pytest.mark.parametrize("march", [1, 2])
@pytest.mark.parametrize("q", [0.0, 0.02])
def test_one_outer_iteration_with_forced_march_axis(q, march, mode):
    import torch
    case = Case((6, 5, 6), bc=(0, 0, 1, 0, 0, 0), cuts=((3,), (2,), (2, 4)), p=11.0)
    prob = case.problem(precision="fp64", mode=mode, inner_tol=1e-30, inner_abs=1e-14, max_inner=4000, q=q,
                        march=march)
    lay = case.check_layout(prob)
    drho = uniform_density(case.ne, seed=2)
    f, fs = case.density_loads(drho)
    rng = np.random.default_rng(4)
    u0 = [1e-9 * rng.standard_normal(s.n) for s in case.part.subs]
    lam0 = [1e-10 * rng.standard_normal(fc.nodes.size) for fc in case.part.faces]
    prob.set_density(torch.tensor(drho, device="cuda"))
    prob.set_state(torch.tensor(case.to_local(lay, u0), device="cuda"),
                   torch.tensor(case.faces_to_lam(lay, lam0), device="cuda"))
    prob.iterate(1)
    u1, lam1 = prob.get_state()
    u1 = case.from_local(lay, u1.cpu().numpy())
    lam1 = case.lam_to_faces(lay, lam1.cpu().numpy())
    orc = S.SchwarzOracle(case.part, case.p, "lu", q_face=q)
    ur = orc.subdomain_solves(fs, lam0)
    lr = orc.exchange(ur, lam0)
    eu = max(np.abs(u1[s] - ur[s]).max() / np.abs(ur[s]).max() for s in range(case.part.n_sub))
    el = max(np.abs(lam1[fc] - lr[fc]).max() / np.abs(lr[fc]).max() for fc in range(len(lr)))
    print("march", march, mode, "q", q, "max rel error: u", eu, "lambda", el, flush=True)
    assert eu <= 1e-10 and el <= 1e-10
    prob.close()


@pytest.mark.parametrize("march", [1, 2])
def test_fixed_point_with_forced_march_axis(march):
    import torch
    case = Case((9, 7, 6), lengths=(1.0, 0.9, 0.7), cuts=((2, 6), (3,), (1, 4)), p=20.0)
    drho = uniform_density(case.ne, seed=3)
    f, _ = case.density_loads(drho)
    ud = D.solve_direct(case.mesh, f, "lu")
    prob = case.problem(precision="fp32", mode="batched", max_outer=20000, inner_tol=1e-3, inner_abs=0.0,
                        march=march)
    phi, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-11)
    err = np.abs(phi.cpu().numpy() - ud).max() / np.abs(ud).max()
    print("march", march, "outer", st["outer_iters"], "err", err, flush=True)
    assert st["converged"] and err <= 1e-10
    prob.close()


def test_x_slabs_of_a_thin_vertical_box_march_along_y():
    """The paper's orientation: x-slabs of a box that is thin in z. A slab's
    x-y node plane (9 x 599) exceeds 4096 nodes, so it marches along y (its
    x-z plane has 45 nodes). With the Fourier-optimised second-order
    condition the FP64 solve needs the oracle's outer iteration count and
    reaches the direct solution."""
    import torch
    ne, lengths = (16, 300, 3), (1.0, 1.0, 0.06)
    case = Case(ne, lengths, cuts=((4, 8, 12), (), ()), p=1.0)
    kmin = np.pi * np.hypot(1 / lengths[1], 1 / lengths[2])
    kmax = np.pi * np.hypot(2 * ne[1] / lengths[1], 2 * ne[2] / lengths[2])
    pq, rho, _ = optimize_robin(2, kmin, kmax)
    p, q = pq[0], pq[1]
    drho = crater_density(ne, lengths, seed=2, up=2)
    f, fs = case.density_loads(drho)
    ud = D.solve_direct(case.mesh, f, "fdm")
    prob = case.problem(p=p, q=q, precision="fp64", mode="stepwise", inner_abs=1e-13, max_inner=4000)
    lay = case.check_layout(prob)
    print("slab axes", lay["perm"].tolist(), "dims", lay["dims"].tolist(), flush=True)
    assert all(p_.tolist() == [0, 2, 1] for p_ in lay["perm"])
    phi, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-10)
    prob.close()
    phi = phi.cpu().numpy()
    orc = S.SchwarzOracle(case.part, p, "lu", q_face=q)
    _, n_or, _, _ = orc.solve(fs, f, 1e-10, 5000)
    err = np.abs(phi - ud).max() / np.abs(ud).max()
    print("slabs along y: gpu outer", st["outer_iters"], "oracle", n_or, "err", err, flush=True)
    assert st["converged"] and abs(st["outer_iters"] - n_or) <= 1 and err <= 1e-8
    # the batched FP32-inner form in the same orientation
    prob = case.problem(p=p, q=q, precision="fp32", mode="batched", check_every=5)
    phi, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-8)
    prob.close()
    res = A.residual_norm(case.mesh, phi.cpu().numpy(), f)
    assert st["converged"] and res <= 1e-8 * 1.001
