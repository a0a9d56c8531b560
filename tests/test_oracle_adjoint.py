"""Pins of the oracle's discrete adjoint and cross-section gradients (project addition)."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import adjoint, dg, quadrature, si


def problem(n=6, seed=3):
    m = dg.Mesh(n, n)
    d, w = quadrature.cl_quadrature(8, 4)
    rng = np.random.default_rng(seed)
    sa = np.exp(np.log(0.5) + 0.5 * rng.normal(size=m.ncell))
    ss = 2.0 * np.ones(m.ncell)
    bc = np.zeros((4, n, 2)); bc[0, n // 2, 0] = np.sqrt(m.hy)
    return si.Problem(m, d, w, sa + ss, ss, np.zeros(m.ndof), bc)


def test_adjoint_flux_equals_transposed_coupled_solve():
    prob = problem()
    rng = np.random.default_rng(0)
    bc_adj = rng.uniform(0, 1, (4, prob.mesh.nx, 2))
    bnd = dg.boundary_unit_vectors(prob.mesh, bc_adj)
    phi_mu, _ = adjoint.adjoint_si_dsa(prob, bnd, 1e-14)
    A = si.coupled_matrix(prob)
    # right-hand side of the normalised adjoint: outflow-side terms per ordinate
    rhs = np.concatenate([dg.boundary_vector(prob.mesh, bnd, -prob.dirs[j, 0], -prob.dirs[j, 1])
                          for j in range(prob.nd)])
    # A^T lambda = diag(w) rhs, mu = lambda / w
    wrep = np.repeat(prob.w, prob.mesh.ndof)
    lam = spla.spsolve(A.T.tocsc(), wrep * rhs)
    mu = (lam / wrep).reshape(prob.nd, -1)
    assert np.abs(prob.w @ mu - phi_mu).max() < 1e-11 * np.abs(phi_mu).max()


def test_gradients_match_central_differences():
    prob = problem()
    J_obs = np.zeros((4, prob.mesh.nx))
    r = adjoint.loss_and_grad(prob, J_obs)
    cells = [0, 7, 20, 35]
    fd_a = adjoint.fd_grad_sigma_a(prob, J_obs, cells, h=1e-6)
    assert np.abs(fd_a - r["grad_sigma_a"][cells]).max() < 1e-5 * np.abs(fd_a).max()
    ss = prob.sigma_s
    fd_s = []
    for c in cells:
        v = []
        for sg in (1.0, -1.0):
            s2 = ss.copy(); s2[c] += sg * 1e-6
            v.append(adjoint.loss(adjoint.with_sigma(prob, sigma_s=s2), J_obs)[0])
        fd_s.append((v[0] - v[1]) / 2e-6)
    fd_s = np.array(fd_s)
    assert np.abs(fd_s - r["grad_sigma_s"][cells]).max() < 1e-5 * np.abs(fd_s).max()


def test_exit_currents_of_constant_state():
    """psi = c in a uniform absorber with inflow c: every face sees J = c sum_j w_j (Omega.n)^+."""
    m = dg.Mesh(4, 4)
    d, w = quadrature.cl_quadrature(8, 4)
    c, st = 0.8, 1.3
    G = np.zeros((m.ncell, 4)); G[:, 0] = st * c * np.sqrt(m.hx * m.hy)
    bc = np.zeros((4, 4, 2)); bc[0:2, :, 0] = c * np.sqrt(m.hy); bc[2:4, :, 0] = c * np.sqrt(m.hx)
    prob = si.Problem(m, d, w, st * np.ones(m.ncell), np.zeros(m.ncell), G.reshape(-1), bc)
    psi = adjoint.all_psi(prob, np.zeros(m.ndof))
    J = adjoint.exit_currents(prob, psi)
    half_range = c * np.sum(w * np.maximum(d[:, 0], 0.0))
    assert np.allclose(J, half_range, rtol=1e-13)
