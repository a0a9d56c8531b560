"""Pins of the oracle's full-rank SI-DSA and MIP diffusion correction (Sec. 2.2, Alg. 1)."""
import numpy as np
import pytest

from oracle import dg, dsa, quadrature, si


def small_problem(nx=6, ny=5, sig_t=1.0, sig_s=0.9, seed=0, hetero=False, bc=None):
    m = dg.Mesh(nx, ny, 0.0, 1.0, 0.0, 0.8)
    d, w = quadrature.cl_quadrature(8, 4)
    rng = np.random.default_rng(seed)
    st = sig_t * (rng.uniform(0.5, 2.0, m.ncell) if hetero else np.ones(m.ncell))
    ss = (sig_s / sig_t) * st
    G = dg.source_moments_box(m, 1.0, (0.3, 0.62, 0.2, 0.5))
    return si.Problem(m, d, w, st, ss, G, bc)


def test_infinite_medium_closed_form():
    """Uniform medium, G = Q, isotropic inflow g = Q/sigma_a => psi_j = phi = Q/sigma_a."""
    m = dg.Mesh(6, 4, 0.0, 1.5, 0.0, 1.0)
    d, w = quadrature.cl_quadrature(8, 4)
    st, ss, Q = 2.0, 1.5, 0.7
    phi_inf = Q / (st - ss)
    G = np.zeros((m.ncell, 4)); G[:, 0] = Q * np.sqrt(m.hx * m.hy)
    bc = np.zeros((4, 6, 2)); bc[0:2, :, 0] = phi_inf * np.sqrt(m.hy); bc[2:4, :, 0] = phi_inf * np.sqrt(m.hx)
    prob = si.Problem(m, d, w, st * np.ones(m.ncell), ss * np.ones(m.ncell), G.reshape(-1), bc)
    out = si.fr_si_dsa(prob, 1e-14, max_outer=200)
    exp = np.zeros((m.ncell, 4)); exp[:, 0] = phi_inf * np.sqrt(m.hx * m.hy)
    assert out["converged"]
    assert np.abs(out["phi"] - exp.reshape(-1)).max() < 1e-12


def test_matches_brute_force_coupled_solve():
    """Converged SI-DSA = direct solve of the whole coupled system eq. (mat-vec-a)."""
    rng = np.random.default_rng(3)
    bc = rng.uniform(0, 1, size=(4, 6, 2))
    prob = small_problem(hetero=True, bc=bc, sig_s=0.95)
    out = si.fr_si_dsa(prob, 1e-14, max_outer=300)
    _, phi_bf = si.brute_force(prob)
    assert out["converged"]
    assert np.abs(out["phi"] - phi_bf).max() < 1e-12 * np.abs(phi_bf).max() * 100


def test_dsa_independence_and_effect():
    """With and without DSA the fixed point is the same; DSA cuts iterations when thick."""
    prob = small_problem(sig_t=30.0, sig_s=29.7)
    a = si.fr_si_dsa(prob, 1e-12, max_outer=3000)
    b = si.fr_si_dsa(prob, 1e-12, max_outer=3000, use_dsa=False)
    assert a["converged"] and b["converged"]
    assert a["iters"] * 5 < b["iters"]
    ref = np.abs(a["phi"]).max()
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-8 * ref


def test_particle_balance():
    """Test function 1 on the coupled system: int sigma_a phi + leakage = int G."""
    prob = small_problem(hetero=True, sig_s=0.8)
    out = si.fr_si_dsa(prob, 1e-14, max_outer=300)
    m = prob.mesh
    phi = out["phi"]
    src = prob.sig_s4 * phi + prob.G
    from oracle import sweep
    psi, _ = sweep.sweep(m, prob.dirs, np.arange(prob.nd), prob.sigma_t, src, prob.bnd)
    one = np.sqrt(m.hx * m.hy)
    fi = np.zeros((4, 6, 2)); fi[0:2, :, 0] = np.sqrt(m.hy); fi[2:4, :, 0] = np.sqrt(m.hx)
    fint = dg.boundary_unit_vectors(m, fi)
    leak = 0.0
    for j in range(prob.nd):
        P = psi[j].reshape(m.ny, m.nx, 4)
        ox, oy, wj = prob.dirs[j, 0], prob.dirs[j, 1], prob.w[j]
        leak += wj * abs(ox) * np.sum(P[:, -1 if ox > 0 else 0] * fint[1 if ox > 0 else 0, :m.ny])
        leak += wj * abs(oy) * np.sum(P[-1 if oy > 0 else 0, :] * fint[3 if oy > 0 else 2, :m.nx])
    absorb = np.sum((prob.sigma_t - prob.sigma_s) * phi.reshape(-1, 4)[:, 0]) * one
    total = np.sum(prob.G.reshape(-1, 4)[:, 0]) * one
    assert abs(absorb + leak - total) < 1e-11 * total


def test_outer_count_and_return_convention():
    prob = small_problem()
    out = si.fr_si_dsa(prob, 1e-8, max_outer=100)
    assert out["converged"] and len(out["history"]) == out["iters"]
    assert out["history"][-1] <= 1e-8 < out["history"][-2]
    assert np.array_equal(out["phi"], out["phis"][-1])


# ---------------- MIP diffusion form ----------------

def test_mip_symmetric_positive_definite():
    m = dg.Mesh(5, 4, 0.0, 1.0, 0.0, 1.0)
    rng = np.random.default_rng(1)
    st = rng.uniform(0.1, 100.0, m.ncell)
    ss = st * rng.uniform(0.0, 1.0, m.ncell)
    A = dsa.mip_matrix(m, st, ss).toarray()
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


def test_mip_consistency_for_linear_functions():
    """For u linear and continuous, D constant, sigma_a = 0: jumps vanish and the flux
    terms cancel the cell integrals, so (A u)_k = 0 on cells away from the boundary."""
    m = dg.Mesh(6, 5, 0.0, 1.2, 0.0, 1.0)
    st = 3.0 * np.ones(m.ncell)
    A = dsa.mip_matrix(m, st, st)
    for gx, gy in [(1.0, 0.0), (0.0, 1.0), (0.7, -1.3)]:
        u = np.zeros((m.ny, m.nx, 4))
        for b in range(m.ny):
            for a in range(m.nx):
                # u = gx x + gy y: mean and the two linear moments of the cell
                sq = np.sqrt(m.hx * m.hy)
                u[b, a, 0] = (gx * m.xc(a) + gy * m.yc(b)) * sq
                u[b, a, 1] = gx * m.hx / (2 * np.sqrt(3)) * sq
                u[b, a, 2] = gy * m.hy / (2 * np.sqrt(3)) * sq
        r = (A @ u.reshape(-1)).reshape(m.ny, m.nx, 4)
        assert np.abs(r[1:-1, 1:-1]).max() < 1e-12


def test_mip_constant_absorption():
    """u = 1, D arbitrary, no boundary in reach: (A u)_k = sigma_a (1, eta_k)."""
    m = dg.Mesh(5, 5)
    rng = np.random.default_rng(2)
    st = rng.uniform(1.0, 10.0, m.ncell)
    ss = st * 0.4
    A = dsa.mip_matrix(m, st, ss)
    u = np.zeros((m.ncell, 4)); u[:, 0] = np.sqrt(m.hx * m.hy)
    r = (A @ u.reshape(-1)).reshape(m.ny, m.nx, 4)
    sa = (st - ss).reshape(m.ny, m.nx)
    assert np.abs(r[1:-1, 1:-1, 0] - sa[1:-1, 1:-1] * np.sqrt(m.hx * m.hy)).max() < 1e-12
    assert np.abs(r[1:-1, 1:-1, 1:]).max() < 1e-12
