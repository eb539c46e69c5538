"""Thin x-slabs as in the paper's Sec. 6 runs (needs an MI355X): with the
second-order condition from the Fourier optimisation (CMA-ES) the GPU Schwarz
solve reaches the global direct solution, needs the oracle's outer iteration
count, and fewer iterations than p = 8/h."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import direct as D
from oracle import schwarz as S
from paper_2112_03851_amd.sos import optimize_robin
from synth.generators import crater_density

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_slabs_with_optimised_second_order_condition():
    import torch
    ne, lengths = (24, 3, 20), (1.0, 0.1, 1.0)
    cuts = (tuple(range(3, 24, 3)), (), ())
    case = Case(ne, lengths, cuts=cuts, p=1.0)
    hy, hz = lengths[1] / ne[1], lengths[2] / ne[2]
    kmin = np.pi * np.hypot(1 / lengths[1], 1 / lengths[2])
    kmax = np.pi * np.hypot(2 / hy, 2 / hz)
    pq, rho, _ = optimize_robin(2, kmin, kmax)
    p, q = pq[0], pq[1]
    print("slabs", len(cuts[0]) + 1, "p", p, "q", q, "rho_max", rho, flush=True)
    drho = crater_density(ne, lengths, seed=1, up=1)
    f, fs = case.density_loads(drho)
    ud = D.solve_direct(case.mesh, f)
    orc = S.SchwarzOracle(case.part, p, "lu", q_face=q)
    _, n_or, res_or, _ = orc.solve(fs, f, 1e-10, 5000)
    prob = case.problem(p=p, q=q, precision="fp64", mode="stepwise", inner_abs=1e-13, max_inner=2000)
    phi, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-10)
    phi = phi.cpu().numpy()
    err = np.abs(phi - ud).max() / np.abs(ud).max()
    print("optimised: gpu outer", st["outer_iters"], "oracle", n_or, "err", err, flush=True)
    assert st["converged"] and err <= 1e-8
    assert abs(st["outer_iters"] - n_or) <= 1
    prob.close()
    p0 = 8.0 * ne[0] / lengths[0]
    prob0 = case.problem(p=p0, precision="fp64", mode="stepwise", inner_abs=1e-13, max_inner=2000)
    phi0, st0 = prob0.solve(torch.tensor(drho, device="cuda"), 1e-10)
    print("p = 8/h: gpu outer", st0["outer_iters"], flush=True)
    assert st0["converged"] and st0["outer_iters"] > st["outer_iters"]
    prob0.close()
