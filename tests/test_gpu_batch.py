"""Several copies of one problem with different transmission conditions in one
context (needs an MI355X): per-copy residual histories, rates and the best
copy against the oracle's Schwarz iteration run copy by copy, and a batched
solve that returns every copy's solution."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import direct as D
from oracle import schwarz as S
from synth import workload
from synth.generators import robin_candidates, uniform_density

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CASE = dict(ne=(8, 8, 8), cuts=((4,), (4,), (4,)), p=1.0)
P_H = np.array([1.0, 4.0, 8.0, 2.0, 0.5])       # p h per copy
Q_H = np.array([0.0, 0.01, 0.0, 0.05, 0.02])     # q / h per copy


def _torch():
    import torch
    return torch


def test_batch_rates_match_oracle_copy_by_copy():
    torch = _torch()
    case = Case(**CASE)
    h = 1.0 / case.ne[0]
    p, q = P_H / h, Q_H * h
    print("case", CASE, "copies", len(p), flush=True)
    prob = case.problem(precision="fp64", mode="stepwise", inner_abs=1e-14, max_inner=2000, check_every=1,
                        copies=len(p), p=p, q=q)
    drho = uniform_density(case.ne, seed=3)
    rates, r1, r2, best, st = prob.batch_rates(torch.tensor(drho, device="cuda"), 10, 20)
    assert st["outer_iters"] == 20
    f, fs = case.density_loads(drho)
    ref = []
    for c in range(len(p)):
        orc = S.SchwarzOracle(case.part, p[c], "lu", q_face=q[c])
        _, n, _, hist = orc.solve(fs, f, 0.0, max_outer=20, history=True)
        hd = dict(hist)
        ref.append((hd[20] / hd[10]) ** 0.1)
        print("copy", c, "gpu", r1[c], r2[c], "oracle", hd[10], hd[20], flush=True)
        assert abs(r1[c] - hd[10]) <= 1e-8 * hd[10]
        assert abs(r2[c] - hd[20]) <= 1e-8 * hd[20]
        assert abs(rates[c] - ref[c]) <= 1e-8
    assert best == int(np.argmin(ref))
    prob.close()


def test_batched_solve_returns_every_copy_solution():
    torch = _torch()
    case = Case(**CASE)
    h = 1.0 / case.ne[0]
    p, q = P_H[:3] / h, Q_H[:3] * h
    drho = uniform_density(case.ne, seed=5)
    f, _ = case.density_loads(drho)
    ud = D.solve_direct(case.mesh, f)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-8)):
        prob = case.problem(precision=prec, mode="batched", inner_tol=1e-2 if prec == "fp32" else 1e-6,
                            inner_abs=0.0, copies=3, p=p, q=q)
        phi, st = prob.solve(torch.tensor(drho, device="cuda"), tol)
        assert st["converged"]
        res = prob.batch_residuals()
        assert np.all(res <= tol) and abs(res.max() - st["rel_residual"]) <= 1e-12 * tol
        phi = phi.cpu().numpy().reshape(3, -1)
        for c in range(3):
            err = np.abs(phi[c] - ud).max() / np.abs(ud).max()
            print(prec, "copy", c, "err vs direct", err, flush=True)
            assert err <= 100 * tol
        prob.close()


def test_candidate_scoring_at_full_size_equals_single_copies():
    """128 candidates on the 32^3 copy (1,024 subdomains in each launch): the
    best copy's residuals equal those of the same condition solved alone."""
    torch = _torch()
    wl = workload("c5copy", seed=0)
    h = 1.0 / wl.ne[0]
    p, q = robin_candidates(128, h, seed=0)
    drho = torch.tensor(wl.drho(), device="cuda")
    case = Case.from_workload(wl)
    prob = case.problem(precision="fp32", mode="batched", inner_tol=0.1, check_every=10, copies=128, p=p, q=q)
    rates, r1, r2, best, st = prob.batch_rates(drho, 10, 20)
    print("best", best, "p", p[best], "q", q[best], "rate", rates[best], "range", np.nanmin(rates), np.nanmax(rates),
          flush=True)
    assert np.all(np.isfinite(rates)) and np.all(rates > 0) and np.all(rates < 1.5)
    assert best == int(np.argmin(rates))
    prob.close()
    for c in (best, 0):
        one = case.problem(precision="fp32", mode="batched", inner_tol=0.1, check_every=10, p=p[c], q=q[c])
        ra, a1, a2, b1, _ = one.batch_rates(drho, 10, 20)
        assert b1 == 0
        assert abs(a1[0] - r1[c]) <= 1e-3 * r1[c] and abs(a2[0] - r2[c]) <= 1e-3 * r2[c], (c, a1, a2, r1[c], r2[c])
        one.close()


@pytest.mark.parametrize("inner_tol,rtol_res,rtol_rate", [(1e-5, 1e-3, 1e-4), (0.1, 0.3, 0.02)])
def test_fp32_batch_rates_match_oracle_copy_by_copy(inner_tol, rtol_res, rtol_rate):
    """The FP32-inner batched scoring (the candidate search's path) against the
    oracle's exact Schwarz iteration copy by copy: 8 seeded second-order
    candidates on a 16^3 mesh with 2x2x2 subdomains. The inexact inner solves
    (relative tolerance eta) perturb each outer step by about eta, so after 10
    and 20 outer iterations the residuals differ from the exact iteration's
    by a few eta (eta = 0.1: up to 24 % measured, bound 3 eta) and the rates,
    a tenth power of their ratio, by a fraction of eta (1.1 % measured, bound
    eta / 5); with the production eta = 0.1 the chosen copy is still the
    oracle's best or within 1 % of its rate."""
    torch = _torch()
    case = Case((16, 16, 16), cuts=((8,), (8,), (8,)), p=1.0)
    h = 1.0 / case.ne[0]
    p, q = robin_candidates(8, h, seed=4)
    print("copies 8, inner_tol", inner_tol, "p", p, "q", q, flush=True)
    prob = case.problem(precision="fp32", mode="batched", inner_tol=inner_tol, inner_abs=0.0, check_every=10,
                        copies=len(p), p=p, q=q)
    drho = uniform_density(case.ne, seed=6)
    rates, r1, r2, best, st = prob.batch_rates(torch.tensor(drho, device="cuda"), 10, 20)
    prob.close()
    f, fs = case.density_loads(drho)
    ref = []
    for c in range(len(p)):
        orc = S.SchwarzOracle(case.part, p[c], "lu", q_face=q[c])
        _, n, _, hist = orc.solve(fs, f, 0.0, max_outer=20, history=True)
        hd = dict(hist)
        ref.append((hd[20] / hd[10]) ** 0.1)
        print("copy", c, "gpu", r1[c], r2[c], rates[c], "oracle", hd[10], hd[20], ref[c], flush=True)
        assert abs(r1[c] - hd[10]) <= rtol_res * hd[10]
        assert abs(r2[c] - hd[20]) <= rtol_res * hd[20]
        assert abs(rates[c] - ref[c]) <= rtol_rate * ref[c]
    ref = np.array(ref)
    assert ref[best] <= ref.min() * 1.01
