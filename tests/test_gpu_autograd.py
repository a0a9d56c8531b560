"""torch.autograd path of the detector misfit (forward solve, exit currents, misfit;
backward adjoint solve and cross-section gradients through the C ABI) against the
oracle's discrete adjoint, and the chain rule through a torch parameterisation.

Bars: loss and gradients within 1e-6 of the oracle's, relative to their magnitude (the
target allows 1e-4); both sides converge SI to 1e-13.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from tests.common import gpu_problem, oracle_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def setup(n=8, seed_obs=3):
    wl = W.tomography(n=n, n_theta=8, n_z=4, smooth=1.0)
    faces = [(W.SIDE_L, 3, 1.0), (W.SIDE_B, 5, 0.5)]
    J_obs = np.random.default_rng(seed_obs).uniform(0.0, 0.05, (4, n))
    return wl, faces, J_obs


def test_autograd_matches_oracle_adjoint():
    import paper_2603_25233_amd as R
    wl, faces, J_obs = setup()
    op = oracle_problem(wl, bc_faces=faces)
    ref = oadj.loss_and_grad(op, J_obs)
    base = gpu_problem(wl, bc_faces=faces)
    sa = (base.sigma_t - base.sigma_s).clone().requires_grad_(True)
    ss = base.sigma_s.clone().requires_grad_(True)
    L, J = R.detector_misfit(sa, ss, base, J_obs, eps_si=1e-13)
    assert abs(L.item() - ref["loss"]) < 1e-10 * abs(ref["loss"])
    assert np.abs(J.cpu().numpy() - ref["J"]).max() < 1e-10 * np.abs(ref["J"]).max()
    L.backward()
    ga = sa.grad.cpu().numpy().reshape(-1)
    gs = ss.grad.cpu().numpy().reshape(-1)
    assert np.abs(ga - ref["grad_sigma_a"]).max() < 1e-6 * np.abs(ref["grad_sigma_a"]).max()
    assert np.abs(gs - ref["grad_sigma_s"]).max() < 1e-6 * np.abs(ref["grad_sigma_s"]).max()


def test_chain_rule_through_log_parameterisation():
    """sigma_a = exp(theta): autograd's dL/dtheta equals the oracle's dL/dsigma_a * sigma_a."""
    import paper_2603_25233_amd as R
    wl, faces, J_obs = setup(seed_obs=5)
    op = oracle_problem(wl, bc_faces=faces)
    ref = oadj.loss_and_grad(op, J_obs)
    base = gpu_problem(wl, bc_faces=faces)
    theta = torch.log(base.sigma_t - base.sigma_s).clone().requires_grad_(True)
    L, _ = R.detector_misfit(torch.exp(theta), base.sigma_s, base, J_obs, eps_si=1e-13)
    (2.0 * L).backward()
    want = 2.0 * ref["grad_sigma_a"] * (op.sigma_t - op.sigma_s)
    got = theta.grad.cpu().numpy().reshape(-1)
    assert np.abs(got - want).max() < 1e-6 * np.abs(want).max()


def test_batched_misfit_oracle_and_central_differences():
    """The optical-tomography functional over several source configurations (one
    isotropic point inflow per side, as the 16-source experiment at reduced size): loss
    and gradient against the oracle's discrete adjoint summed over sources, and the
    gradient against FP64 central differences (h = 1e-6) of the library's own forward
    solves on 64 seeded random cells, bar 1e-4 of the largest gradient entry."""
    import paper_2603_25233_amd as R
    n = 16
    wl = W.tomography(n=n, n_theta=8, n_z=4, smooth=2.0)
    faces = [(W.SIDE_L, 5, 1.0), (W.SIDE_R, 10, 1.0), (W.SIDE_B, 3, 1.0), (W.SIDE_T, 12, 1.0)]
    J_obs = np.random.default_rng(17).uniform(0.0, 0.02, (len(faces), 4, n))
    base = gpu_problem(wl)
    bcs = np.stack([R.inflow_moments(n, n, wl["domain"], [f]) for f in faces])
    ref_L = 0.0
    ref_ga = np.zeros(n * n)
    ref_gs = np.zeros(n * n)
    for s, f in enumerate(faces):
        r = oadj.loss_and_grad(oracle_problem(wl, bc_faces=[f]), J_obs[s])
        ref_L += r["loss"]
        ref_ga += r["grad_sigma_a"]
        ref_gs += r["grad_sigma_s"]
    sa = (base.sigma_t - base.sigma_s).clone().requires_grad_(True)
    ss = base.sigma_s.clone().requires_grad_(True)
    kw = dict(eps_si=1e-13, eps_dsa=1e-13)
    L, J = R.detector_misfit_batch(sa, ss, base, bcs, J_obs, **kw)
    assert J.shape == (len(faces), 4, n)
    assert abs(L.item() - ref_L) < 1e-10 * abs(ref_L)
    L.backward()
    ga = sa.grad.cpu().numpy().reshape(-1)
    gs = ss.grad.cpu().numpy().reshape(-1)
    assert np.abs(ga - ref_ga).max() < 1e-6 * np.abs(ref_ga).max()
    assert np.abs(gs - ref_gs).max() < 1e-6 * np.abs(ref_gs).max()
    cells = np.random.default_rng(23).choice(n * n, 64, replace=False)
    h = 1e-6
    fd = []
    with torch.no_grad():
        for c in cells:
            vals = []
            for sgn in (1.0, -1.0):
                s2 = (base.sigma_t - base.sigma_s).clone().reshape(-1)
                s2[c] += sgn * h
                vals.append(R.detector_misfit_batch(s2.reshape(n, n), base.sigma_s, base, bcs,
                                                    J_obs, **kw)[0].item())
            fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    assert np.abs(fd - ga[cells]).max() < 1e-4 * np.abs(ga).max()
