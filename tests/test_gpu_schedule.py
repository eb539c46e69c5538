"""Order of the fused kernel's blocks (needs an MI355X). With one block per
subdomain the subdomains do not interact inside a launch, so taking them in
decreasing order of their previous inner solve's work changes no result bit:
checked on uneven subdomains and on a batch of more subdomains than the
ordering kernel sorts in one chunk (1024). The per-subdomain inner iteration
counts add up to the solve's total."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import assemble as A
from oracle import direct as D
from synth.generators import uniform_density

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

# uneven columns: widths 3..8 elements in x and y, 16 planes of elements in z
UNEVEN = dict(ne=(24, 20, 16), cuts=((3, 8, 15), (4, 11), ()), p=160.0)


def _solve(case, drho, tol, schedule, **kw):
    import torch
    prob = case.problem(precision="fp32", mode="batched", block=256, team=1, schedule=schedule, **kw)
    phi, st = prob.solve(torch.tensor(drho, device="cuda"), tol)
    iters = prob.inner_iters()
    prob.close()
    return phi, st, iters


def test_schedule_by_work_changes_no_bit_on_uneven_subdomains():
    import torch
    case = Case(**UNEVEN)
    drho = uniform_density(case.ne, seed=8)
    f, _ = case.density_loads(drho)
    ud = D.solve_direct(case.mesh, f, "lu")
    kw = dict(check_every=5, max_outer=20000, inner_tol=1e-3, inner_abs=0.0)
    (p1, s1, i1), (p0, s0, i0) = (_solve(case, drho, 1e-11, s, **kw) for s in (1, 0))
    print("outer", s1["outer_iters"], s0["outer_iters"], "inner", s1["inner_iters"], s0["inner_iters"],
          "last inner counts", i1, flush=True)
    assert s1["converged"] and s1["team"] == 1
    assert torch.equal(p1, p0)
    assert s1["outer_iters"] == s0["outer_iters"] and s1["inner_iters"] == s0["inner_iters"] and i1 == i0
    assert len(set(i1)) > 1  # the order is not the fixed one
    phi = p1.cpu().numpy()
    err = np.abs(phi - ud).max() / np.abs(ud).max()
    res = A.residual_norm(case.mesh, phi, f)
    print("residual", res, "err vs direct", err, flush=True)
    assert res <= 1e-11 * 1.001 and err <= 1e-10


def test_schedule_by_work_over_several_sort_chunks():
    import torch
    case = Case(ne=(8, 8, 8), cuts=((2, 4, 6), (2, 4, 6), (2, 4, 6)))
    h = 1.0 / 8
    copies = 20  # 20 x 64 = 1280 subdomains
    p = np.geomspace(1.0 / h, 40.0 / h, copies)
    q = np.zeros(copies)
    drho = uniform_density(case.ne, seed=4)
    kw = dict(check_every=5, max_outer=20000, inner_tol=1e-2, inner_abs=0.0, copies=copies, p=p, q=q)
    (p1, s1, i1), (p0, s0, i0) = (_solve(case, drho, 1e-8, s, **kw) for s in (1, 0))
    print("outer", s1["outer_iters"], "inner", s1["inner_iters"], "distinct last counts", sorted(set(i1)), flush=True)
    assert s1["converged"] and len(i1) == 64 * copies
    assert torch.equal(p1, p0)
    assert s1["outer_iters"] == s0["outer_iters"] and s1["inner_iters"] == s0["inner_iters"] and i1 == i0
    f, _ = case.density_loads(drho)
    ud = D.solve_direct(case.mesh, f, "lu")
    phi = p1.cpu().numpy().reshape(copies, -1)
    for c in range(copies):
        err = np.abs(phi[c] - ud).max() / np.abs(ud).max()
        assert err <= 100 * 1e-8, (c, err)


def test_inner_iteration_counts_add_up_to_the_outer_iteration_total():
    import torch
    case = Case(**UNEVEN)
    drho = uniform_density(case.ne, seed=2)
    for schedule in (1, 0):
        prob = case.problem(precision="fp32", mode="batched", block=256, team=1, schedule=schedule, check_every=1,
                            max_outer=1, inner_tol=1e-3, inner_abs=0.0, max_inner=500)
        _, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-14)
        it = np.array(prob.inner_iters())
        prob.close()
        print("schedule", schedule, "counts", it.tolist(), "total", st["inner_iters"], flush=True)
        assert st["outer_iters"] == 1 and not st["converged"]
        assert len(it) == case.part.n_sub and np.all(it >= 1) and np.all(it <= 500)
        assert it.sum() == st["inner_iters"]
