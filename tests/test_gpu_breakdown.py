"""Failure detection of the inner solves (needs an MI355X): a non-finite load,
a team barrier that never completes and an outer iteration limit end the
solve with their exact error codes, and every kernel still exits normally.
The residual history and the per-check log record each convergence check."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import assemble as A
from paper_2112_03851_amd import sos
from synth import workload

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _torch():
    import torch
    return torch


@pytest.mark.parametrize("prec,mode", [("fp32", "batched"), ("fp64", "stepwise"), ("fp64", "batched")])
def test_nan_in_density_reports_breakdown(prec, mode):
    torch = _torch()
    wl = workload("c1", seed=0)
    case = Case.from_workload(wl)
    drho = wl.drho()
    drho[len(drho) // 3] = np.nan
    prob = case.problem(precision=prec, mode=mode, check_every=4)
    print("case c1 NaN", prec, mode, flush=True)
    with pytest.raises(sos.SosError) as ei:
        prob.solve(torch.tensor(drho, device="cuda"), wl.tol)
    assert ei.value.code == sos.SOS_EBREAKDOWN
    assert "non-finite" in str(ei.value)
    # the context stays usable: a finite load solves
    phi, st = prob.solve(torch.tensor(wl.drho(), device="cuda"), wl.tol)
    assert st["converged"] and st["code"] == sos.SOS_OK
    prob.close()


def test_team_barrier_that_never_completes_reports_breakdown():
    """Every member waits for a tag no member writes, bounded by 20,000 ticks
    (0.2 ms): each barrier gives up, the solve stops with SOS_EBREAKDOWN at
    the first check and the context solves normally afterwards."""
    torch = _torch()
    wl = workload("c1", seed=0)
    case = Case.from_workload(wl)
    drho = torch.tensor(wl.drho(), device="cuda")
    prob = case.problem(precision="fp32", mode="batched", team=2, block=256, check_every=4)
    prob.debug_barrier(spin_ticks=20000, tag_skew=1)
    print("case c1 team 2, barrier forced to give up", flush=True)
    with pytest.raises(sos.SosError) as ei:
        prob.solve(drho, wl.tol)
    assert ei.value.code == sos.SOS_EBREAKDOWN
    assert "team barrier" in str(ei.value)
    hist = prob.history()
    assert len(hist) == 1 and hist[0][0] == 4
    prob.debug_barrier(0, 0)
    phi, st = prob.solve(drho, wl.tol)
    f, _ = case.density_loads(wl.drho())
    assert st["converged"] and st["team"] == 2
    assert A.residual_norm(case.mesh, phi.cpu().numpy(), f) <= wl.tol * 1.001
    prob.close()


def test_outer_limit_reports_enoconv_with_phi_written():
    torch = _torch()
    wl = workload("c1", seed=0)
    case = Case.from_workload(wl)
    prob = case.problem(precision="fp32", mode="batched", max_outer=1)
    phi, st = prob.solve(torch.tensor(wl.drho(), device="cuda"), wl.tol)
    assert st["code"] == sos.SOS_ENOCONV and not st["converged"] and st["outer_iters"] == 1
    assert torch.isfinite(phi).all() and phi.abs().max() > 0
    prob.close()


def test_residual_history_and_log(capfd):
    import os
    torch = _torch()
    wl = workload("c1", seed=0)
    case = Case.from_workload(wl)
    prob = case.problem(precision="fp32", mode="batched", check_every=5)
    os.environ["SOS_LOG"] = "1"
    try:
        phi, st = prob.solve(torch.tensor(wl.drho(), device="cuda"), wl.tol)
    finally:
        del os.environ["SOS_LOG"]
    hist = prob.history()
    assert st["converged"] and len(hist) == st["checks"]
    assert [h[0] for h in hist] == [5 * (i + 1) for i in range(len(hist))]
    assert hist[-1][1] == st["rel_residual"] and hist[-1][0] == st["outer_iters"]
    assert hist[-1][1] <= wl.tol < hist[-2][1]
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("sos: outer")]
    assert len(lines) == len(hist)
    assert float(lines[-1].split()[-1]) == pytest.approx(st["rel_residual"], rel=1e-6)
    prob.close()
