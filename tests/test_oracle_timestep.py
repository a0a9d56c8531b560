"""Pins of the oracle's backward Euler step (the implicit time marching of Sec. 3.7)."""
import numpy as np
import pytest

from oracle import dg, lowrank, quadrature, si, timestep
from workloads import random_stream


def problem(nx=6, ny=5, nt=8, nz=2, c=0.9, seed=3, G=True):
    m = dg.Mesh(nx, ny)
    d, w = quadrature.cl_quadrature(nt, nz)
    st = np.random.default_rng(seed).uniform(1.0, 4.0, m.ncell)
    src = dg.source_moments_box(m, 1.0, (0.2, 0.7, 0.3, 0.8)) if G else np.zeros(m.ndof)
    return si.Problem(m, d, w, st, c * st, src)


def test_step_equals_direct_solve_of_the_step_system():
    """SI-DSA of one step equals the direct solve of
    (D_j + Sigma_t + I/dt) psi_j - Sigma_s sum_i w_i psi_i = G + g_j + psi^m_j / dt,
    assembled here from the steady operators plus the identity / dt."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    prob = problem()
    dt = 0.3
    psi_prev = np.random.default_rng(1).uniform(0.0, 1.0, (prob.nd, prob.mesh.ndof))
    A = si.coupled_matrix(prob) + sp.identity(prob.nd * prob.mesh.ndof) / dt
    rhs = np.concatenate([prob.G + prob.g_bc(j) + psi_prev[j] / dt for j in range(prob.nd)])
    psi_ref = spla.spsolve(A.tocsc(), rhs).reshape(prob.nd, -1)
    out = timestep.fr_step(prob, dt, psi_prev, eps_si=1e-13)
    assert out["converged"]
    assert np.abs(out["phi"] - prob.w @ psi_ref).max() < 1e-10 * np.abs(psi_ref).max()
    assert np.abs(out["psi"] - psi_ref).max() < 1e-10 * np.abs(psi_ref).max()
    psi_bf, phi_bf = timestep.brute_force_step(prob, dt, psi_prev)
    assert np.abs(psi_bf - psi_ref).max() < 1e-12 * np.abs(psi_ref).max()


@pytest.mark.parametrize("dt", [1e-2, 1.0, 1e3])
def test_steady_state_is_a_fixed_point(dt):
    """psi^m = the steady solution gives psi^{m+1} = psi^m for every dt."""
    prob = problem()
    psi_ss, phi_ss = si.brute_force(prob)
    out = timestep.fr_step(prob, dt, psi_ss, eps_si=1e-13)
    assert np.abs(out["phi"] - phi_ss).max() < 1e-10 * np.abs(phi_ss).max()
    assert np.abs(out["psi"] - psi_ss).max() < 1e-10 * np.abs(psi_ss).max()


def test_large_step_reaches_the_steady_state_and_decay_without_source():
    prob = problem()
    psi0 = np.random.default_rng(2).uniform(0.0, 1.0, (prob.nd, prob.mesh.ndof))
    _, phi_ss = si.brute_force(prob)
    out = timestep.fr_step(prob, 1e9, psi0, eps_si=1e-13)
    assert np.abs(out["phi"] - phi_ss).max() < 1e-7 * np.abs(phi_ss).max()
    # no source, vacuum: the particle content sum_j w_j <psi_j> falls every step
    p0 = problem(G=False)
    psi = psi0
    mass = [float(p0.w @ psi[:, 0::4].sum(axis=1))]
    for _ in range(4):
        psi = timestep.fr_step(p0, 0.2, psi, eps_si=1e-13)["psi"]
        mass.append(float(p0.w @ psi[:, 0::4].sum(axis=1)))
    assert all(b < a for a, b in zip(mass, mass[1:])) and mass[-1] > 0


def test_low_rank_step_at_full_rank_equals_full_rank_step():
    """Every class sampled (q covers them, tiny inner thresholds): the low-rank step is the
    full-rank step, also with a previous psi from a low-rank step."""
    prob = problem(nx=6, ny=6, nt=8, nz=2)
    K = len(lowrank.direction_classes(prob.dirs)[1])
    kw = dict(p=2, q=K, eps_res=1e-14, eps_diff=1e-14, eps_svd=1e-15)
    lr1 = timestep.lr_step(prob, 0.5, None, 1e-12, rand=random_stream(2), **kw)
    fr1 = timestep.fr_step(prob, 0.5, None, 1e-12)
    assert np.abs(lr1["phi"] - fr1["phi"]).max() < 1e-9 * np.abs(fr1["phi"]).max()
    assert np.abs(lr1["psi"] - fr1["psi"]).max() < 1e-9 * np.abs(fr1["psi"]).max()
    lr2 = timestep.lr_step(prob, 0.5, lr1["psi"], 1e-12, rand=random_stream(3), **kw)
    fr2 = timestep.fr_step(prob, 0.5, fr1["psi"], 1e-12)
    assert np.abs(lr2["phi"] - fr2["phi"]).max() < 1e-9 * np.abs(fr2["phi"]).max()


def test_low_rank_step_keeps_the_low_rank_steady_state():
    """The steady low-rank solution's X S V^T fed back as psi^m is a fixed point of the
    low-rank step to the inner thresholds."""
    prob = problem(nx=8, ny=8, nt=8, nz=4, c=0.99)
    kw = dict(p=1, q=8, eps_res=1e-10, eps_diff=1e-10, eps_svd=1e-11)
    ss = lowrank.lr_si_dsa(prob, 1e-11, rand=random_stream(5), **kw)
    psi_ss = (ss["X"] @ np.diag(ss["S"]) @ ss["V"].T).T
    out = timestep.lr_step(prob, 0.1, psi_ss, 1e-11, rand=random_stream(6), **kw)
    assert np.abs(out["phi"] - ss["phi"]).max() < 1e-7 * np.abs(ss["phi"]).max()
