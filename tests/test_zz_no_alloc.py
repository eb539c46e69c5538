"""The allocation-free global residual (needs an MI355X): sos_residual_noalloc
against sos_residual on the same state, through the C-ABI, on two calls in a
row (the second on a smaller context), and its size limit."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from paper_2112_03851_amd import sos
from synth.generators import uniform_density

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _state(case, n_outer, seed):
    import torch
    prob = case.problem(precision="fp32", mode="batched", check_every=5)
    prob.set_density(torch.tensor(uniform_density(case.ne, seed=seed), device="cuda"))
    prob.iterate(n_outer)
    return prob


def test_noalloc_residual_matches_residual_twice_then_smaller():
    import torch
    big = Case((32, 32, 32), cuts=((16,), (16,), (16,)), p=256.0)
    small = Case((12, 10, 8), cuts=((5,), (4,), ()), p=80.0)
    for case, n_outer, seed in ((big, 20, 1), (small, 15, 2)):
        print("case", case.ne, "outer", n_outer, flush=True)
        prob = _state(case, n_outer, seed)
        phi0, r0 = prob.residual(want_phi=True)
        phi1, r1 = prob.residual_noalloc(want_phi=True)
        _, r2 = prob.residual_noalloc(want_phi=False)
        print("residual", r0, "noalloc", r1, r2, flush=True)
        assert np.isfinite(r0) and 0.0 < r0 < 1.0
        assert r1 == r0 and r2 == r0
        assert torch.equal(phi0, phi1)
        prob.close()


def test_noalloc_residual_rejects_contexts_beyond_its_scratch():
    case = Case((96, 96, 48), cuts=((24, 48, 72), (24, 48, 72), ()), p=768.0)
    prob = case.problem(precision="fp32", mode="batched")
    with pytest.raises(sos.SosError) as ei:
        prob.residual_noalloc()
    assert ei.value.code == sos.SOS_EINVAL and "scratch" in str(ei.value)
    prob.close()
