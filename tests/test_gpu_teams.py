"""Team sizes per subdomain in the batched fused kernel (needs an MI355X):
uneven subdomains with different team sizes reach the oracle's direct
solution, graph replay and eager launches agree bit for bit, and the
autotuner gives every subdomain of a size bucket the same team size."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import assemble as A
from oracle import direct as D
from synth.generators import uniform_density

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

# uneven columns: widths 3..8 elements in x and y, 16 planes of elements in z
UNEVEN = dict(ne=(24, 20, 16), cuts=((3, 8, 15), (4, 11), ()), p=160.0)


def _buckets(dims):
    """The documented size buckets: one if node counts differ by at most
    1.5x, else three of equal width in log size, 0 the largest."""
    n = np.prod(np.asarray(dims, np.int64), axis=1)
    lo, hi = n.min(), n.max()
    if hi <= lo * 3 // 2:
        return np.zeros(len(n), int)
    k = np.minimum(2, (3 * np.log(n / lo) / np.log(hi / lo)).astype(int))
    return 2 - k


def test_mixed_team_sizes_match_direct_and_graph_matches_eager():
    import torch
    case = Case(**UNEVEN)
    drho = uniform_density(case.ne, seed=8)
    f, _ = case.density_loads(drho)
    ud = D.solve_direct(case.mesh, f, "lu")
    sizes = np.array([s.n for s in case.part.subs])
    # larger subdomains get larger teams: 1, 2, 4 by size tercile
    order = np.argsort(np.argsort(sizes))
    teams = np.where(order >= 2 * len(sizes) // 3, 4, np.where(order >= len(sizes) // 3, 2, 1))
    print("sizes", sizes.tolist(), "teams", teams.tolist(), flush=True)
    out = []
    for use_graph in (1, 0):
        prob = case.problem(precision="fp32", mode="batched", block=256, team=1, check_every=5, use_graph=use_graph,
                            max_outer=20000, inner_tol=1e-3, inner_abs=0.0)
        prob.set_teams(teams)
        assert np.array_equal(prob.teams(), teams)
        phi, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-11)
        assert st["converged"] and st["team"] == 4
        out.append((phi, st))
        prob.close()
    (p1, s1), (p2, s2) = out
    assert torch.equal(p1, p2) and s1["outer_iters"] == s2["outer_iters"] and s1["inner_iters"] == s2["inner_iters"]
    phi = p1.cpu().numpy()
    err = np.abs(phi - ud).max() / np.abs(ud).max()
    res = A.residual_norm(case.mesh, phi, f)
    print("mixed teams: outer", s1["outer_iters"], "residual", res, "err vs direct", err, flush=True)
    assert res <= 1e-11 * 1.001 and err <= 1e-10


def test_autotuner_picks_one_team_size_per_size_bucket():
    import torch
    case = Case(**UNEVEN)
    drho = uniform_density(case.ne, seed=9)
    f, _ = case.density_loads(drho)
    prob = case.problem(precision="fp32", mode="batched", check_every=10)
    phi, st = prob.solve(torch.tensor(drho, device="cuda"), 1e-8)
    teams = prob.teams()
    buckets = _buckets(prob.layout()["dims"])
    print("buckets", buckets.tolist(), "teams", teams.tolist(), "block", st["block"], flush=True)
    assert len(set(buckets.tolist())) == 3
    for b in range(3):
        assert len(set(teams[buckets == b].tolist())) == 1
    assert st["converged"] and st["team"] == teams.max()
    assert A.residual_norm(case.mesh, phi.cpu().numpy(), f) <= 1e-8 * 1.001
    prob.close()


def test_set_teams_rejects_teams_beyond_a_subdomains_planes():
    from paper_2112_03851_amd import sos
    case = Case((8, 8, 3), cuts=((4,), (4,), ()), p=64.0)
    prob = case.problem(precision="fp32", mode="batched", block=256, team=1)
    with pytest.raises(sos.SosError) as ei:
        prob.set_teams([8, 1, 1, 1])
    assert ei.value.code == sos.SOS_EINVAL and "z-planes" in str(ei.value)
    with pytest.raises(sos.SosError):
        prob.set_teams([0, 1, 1, 1])
    prob.close()


def test_fixed_block_or_team_is_kept_over_a_cached_tuning(tmp_path, monkeypatch):
    import torch
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("SOS_TUNE_CACHE", str(cache))
    case = Case(**UNEVEN)
    drho = torch.tensor(uniform_density(case.ne, seed=9), device="cuda")
    prob = case.problem(precision="fp32", mode="batched", check_every=10)
    _, st = prob.solve(drho, 1e-8)
    prob.close()
    auto = st["block"]
    assert st["converged"] and len(cache.read_text().splitlines()) == 1
    # a fixed block shape (teams tuned) and a fixed team size (shape tuned)
    # are kept although the cache holds a full search of the same geometry
    fixed = 320 if auto != 320 else 384
    prob = case.problem(precision="fp32", mode="batched", check_every=10, block=fixed)
    _, st = prob.solve(drho, 1e-8)
    prob.close()
    print("cached block", auto, "fixed", fixed, "got", st["block"], flush=True)
    assert st["converged"] and st["block"] == fixed
    prob = case.problem(precision="fp32", mode="batched", check_every=10, team=2)
    _, st = prob.solve(drho, 1e-8)
    teams = prob.teams()
    prob.close()
    assert st["converged"] and np.all(teams == 2)
    assert len(cache.read_text().splitlines()) == 1


def test_team_grid_that_cannot_be_resident_is_refused_and_does_not_leak():
    """A team grid larger than the GPU holds at once (64 subdomains x 8
    members of 1024 threads) is refused at launch with SOS_EHIP before any
    block runs, and the refusal does not reach the next problem's calls."""
    import torch
    from paper_2112_03851_amd import sos
    cuts = tuple(range(4, 32, 4))
    case = Case((32, 32, 16), cuts=(cuts, cuts, ()), p=256.0)
    drho = uniform_density(case.ne, seed=3)
    f, _ = case.density_loads(drho)
    d = torch.tensor(drho, device="cuda")
    prob = case.problem(precision="fp32", mode="batched", block=1024, team=8, check_every=5, max_outer=10)
    with pytest.raises(sos.SosError) as ei:
        prob.solve(d, 1e-8)
    prob.close()
    print("refused:", str(ei.value)[:160], flush=True)
    assert ei.value.code == sos.SOS_EHIP and "cooperative" in str(ei.value)
    prob = case.problem(precision="fp32", mode="batched", block=256, team=1, check_every=5, max_outer=20000,
                        inner_tol=1e-3, inner_abs=0.0)
    phi, st = prob.solve(d, 1e-8)
    prob.close()
    assert st["converged"] and A.residual_norm(case.mesh, phi.cpu().numpy(), f) <= 1e-8 * 1.001
