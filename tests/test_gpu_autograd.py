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
