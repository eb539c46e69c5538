"""The Robin exchange after a change of the Robin coefficients and on faces
wider than one pass of an exchange block, against the oracle (needs an
MI355X)."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import schwarz as S
from synth.generators import uniform_density

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _one_iteration(case, prob, q, seed):
    import torch
    lay = case.check_layout(prob)
    drho = uniform_density(case.ne, seed=seed)
    f, fs = case.density_loads(drho)
    rng = np.random.default_rng(seed + 1)
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
    print("max rel error: u", eu, "lambda", el, flush=True)
    for s in range(case.part.n_sub):
        assert np.abs(u1[s] - ur[s]).max() <= 1e-10 * np.abs(ur[s]).max(), s
    for fc in range(len(lr)):
        assert np.abs(lam1[fc] - lr[fc]).max() <= 1e-10 * np.abs(lr[fc]).max(), fc


def test_exchange_uses_coefficients_set_after_setup():
    """Set up with p = 11, q = 0, switch to p = 7, q = 0.02: the next outer
    iteration (solves and exchange) is the oracle's with the new ones."""
    case = Case((6, 5, 6), bc=(0, 0, 1, 0, 0, 0), cuts=((3,), (2,), (2, 4)), p=11.0)
    prob = case.problem(precision="fp64", mode="stepwise", inner_abs=1e-14, max_inner=2000)
    prob.set_robin(7.0, 0.02)
    case.p = 7.0
    _one_iteration(case, prob, 0.02, seed=11)


def test_exchange_on_a_face_wider_than_one_block_pass():
    """A z-face of 521 x 1 nodes: one row per exchange block and more face
    nodes than threads, so a block visits some nodes in a second pass."""
    case = Case((260, 1, 2), bc=(1, 1, 0, 0, 0, 0), cuts=((), (), (1,)), p=40.0)
    assert [fc.nodes.size for fc in case.part.faces] == [521, 521]
    prob = case.problem(precision="fp64", mode="stepwise", inner_abs=1e-14, max_inner=4000)
    _one_iteration(case, prob, 0.0, seed=21)
