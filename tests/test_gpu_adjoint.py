"""Adjoint Schwarz solve and autograd (needs an MI355X): the gradient of a
surface gravity misfit with respect to the per-element density, against the
oracle's global direct adjoint and against central finite differences."""
import numpy as np
import pytest

from bridge import Case, gpu_available
from oracle import adjoint as AD
from synth import workload

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _gather_form(P):
    """Rows of the sparse observation operator as padded (index, weight) arrays."""
    P = P.tocsr()
    k = int(np.diff(P.indptr).max())
    idx = np.zeros((P.shape[0], k), np.int64)
    w = np.zeros((P.shape[0], k))
    for i in range(P.shape[0]):
        a, b = P.indptr[i], P.indptr[i + 1]
        idx[i, :b - a] = P.indices[a:b]
        w[i, :b - a] = P.data[a:b]
    return idx, w


def _misfit_grad_gpu(prob, drho, idx, w, d, tol):
    import torch
    from paper_2112_03851_amd.sos import SchwarzSolve
    x = torch.tensor(drho, device="cuda", requires_grad=True)
    phi = SchwarzSolve.apply(x, prob, tol)
    obs = (phi[torch.tensor(idx, device="cuda")] * torch.tensor(w, device="cuda")).sum(dim=1)
    J = 0.5 * ((obs - torch.tensor(d, device="cuda")) ** 2).sum()
    J.backward()
    return float(J.detach()), x.grad.cpu().numpy(), phi.detach().cpu().numpy()


def test_adjoint_gradient_small_matches_direct_adjoint_and_fd():
    case = Case((6, 6, 4), bc=(0, 0, 0, 0, 0, 1), cuts=((3,), (2, 4), (2,)), p=40.0)
    G = case.G
    from synth.generators import uniform_density
    P = AD.observation_operator(case.mesh, AD.top_face_points(7))
    d = P @ AD.forward(case.mesh, uniform_density(case.ne, seed=4), G, "lu")
    drho = uniform_density(case.ne, seed=5)
    idx, w = _gather_form(P)
    prob = case.problem(precision="fp64", mode="batched", inner_tol=1e-3, inner_abs=0.0, max_outer=50000)
    J, grad, phi = _misfit_grad_gpu(prob, drho, idx, w, d, 1e-12)
    ref, phi_ref, _ = AD.gradient_direct(case.mesh, P, drho, d, G, "lu")
    assert abs(J - AD.misfit(P, phi_ref, d)) <= 1e-8 * J
    assert np.abs(grad - ref).max() <= 1e-7 * np.abs(ref).max()
    rng = np.random.default_rng(1)
    eps = 0.1 * np.abs(drho).max()
    for e in rng.choice(case.mesh.n_elem, 10, replace=False):
        dp, dm = drho.copy(), drho.copy()
        dp[e] += eps
        dm[e] -= eps
        fd = (AD.misfit(P, AD.forward(case.mesh, dp, G, "lu"), d)
              - AD.misfit(P, AD.forward(case.mesh, dm, G, "lu"), d)) / (2 * eps)
        assert abs(fd - grad[e]) <= 1e-6 * np.abs(grad).max()


def test_adjoint_gradient_c4_48cube_27_subdomains():
    """48^3 elements, 3x3x3 subdomains, top face Neumann, 64x64 observation
    points on the top face, target from a seeded 'true' density: the gradient
    matches the global direct adjoint and central differences on 20 random
    elements to 1e-5 relative."""
    wl = workload("c4", seed=0)
    case = Case.from_workload(wl)
    P = AD.observation_operator(case.mesh, AD.top_face_points(64))
    true = workload("c4", seed=1).drho()
    d = P @ AD.forward(case.mesh, true, wl.G, "fdm")
    drho = wl.drho()
    idx, w = _gather_form(P)
    prob = case.problem(precision="fp64", mode="batched", inner_tol=1e-3, inner_abs=0.0, check_every=10,
                        max_outer=60000)
    J, grad, _ = _misfit_grad_gpu(prob, drho, idx, w, d, 1e-11)
    ref, _, _ = AD.gradient_direct(case.mesh, P, drho, d, wl.G, "fdm")
    rel = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    print("c4 adjoint: J", J, "rel err vs direct adjoint", rel, flush=True)
    assert rel <= 1e-5
    rng = np.random.default_rng(2)
    eps = 0.1 * np.abs(drho).max()
    scale = np.abs(ref).max()
    worst = 0.0
    for e in rng.choice(case.mesh.n_elem, 20, replace=False):
        dp, dm = drho.copy(), drho.copy()
        dp[e] += eps
        dm[e] -= eps
        fd = (AD.misfit(P, AD.forward(case.mesh, dp, wl.G, "fdm"), d)
              - AD.misfit(P, AD.forward(case.mesh, dm, wl.G, "fdm"), d)) / (2 * eps)
        worst = max(worst, abs(fd - grad[e]) / scale)
    print("c4 adjoint: worst FD difference / max|grad|", worst, flush=True)
    assert worst <= 1e-5
