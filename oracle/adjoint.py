"""Discrete adjoint and cross-section gradients of the oracle (a project addition).

The paper has no adjoint; this follows from the discrete system eq. (mat-vec-a):
    (D_j + Sigma_t) psi_j - Sigma_s sum_i w_i psi_i = G + g_j^bc   for all j.
For a functional L(psi) the multiplier lambda_j = w_j mu_j solves
    (D_j + Sigma_t)^T mu_j - Sigma_s Phi_mu = (dL/dpsi_j) / w_j,  Phi_mu = sum_i w_i mu_i,
which is again an SI-DSA problem (the diffusion correction is symmetric and the same).
With sigma_t = sigma_s + sigma_a per cell c:
    dL/dsigma_a,c = - sum_j w_j <mu_j, psi_j>_c
    dL/dsigma_s,c = dL/dsigma_a,c + <Phi_mu, phi>_c.

Detector functional: for every boundary face e (sides L, R, B, T) the exit partial
current averaged over the face,
    J_e = sum_j w_j (Omega_j . n_e)^+ |e|^{-1} int_e psi_j ds   (interior trace),
and L = 1/2 sum_e (J_e - J_e^obs)^2.  Then (dL/dpsi_j)/w_j is the outflow-side
boundary term of the transposed sweep with face data (J_e - J_e^obs)/|e|, so the
adjoint is solved with the transposed sweep of oracle/csweep.c.
"""
import numpy as np

from . import dg, si, sweep


def face_integrals(mesh):
    """int_e eta_k ds for every boundary face: [4 sides, max(nx,ny), 4]."""
    m = max(mesh.nx, mesh.ny)
    bc = np.zeros((4, m, 2))
    for s in range(4):
        flen = mesh.hy if s < 2 else mesh.hx
        bc[s, :, 0] = np.sqrt(flen)           # g = 1 on every face: g_0 = int l_0 = sqrt(h)
    return dg.boundary_unit_vectors(mesh, bc)


def face_lengths(mesh):
    m = max(mesh.nx, mesh.ny)
    L = np.zeros((4, m))
    L[0:2, :mesh.ny] = mesh.hy
    L[2:4, :mesh.nx] = mesh.hx
    return L


def exit_currents(prob, psi):
    """J_e for all boundary faces from psi [N, ndof]; zero-padded [4, max(nx,ny)]."""
    mesh = prob.mesh
    fi = face_integrals(mesh)
    flen = face_lengths(mesh)
    P = psi.reshape(prob.nd, mesh.ny, mesh.nx, 4)
    J = np.zeros((4, max(mesh.nx, mesh.ny)))
    for j in range(prob.nd):
        ox, oy = prob.dirs[j, 0], prob.dirs[j, 1]
        wj = prob.w[j]
        if ox < 0:   # exits through the left side (n = -x)
            J[0, :mesh.ny] += wj * (-ox) * np.einsum("bk,bk->b", P[j, :, 0, :], fi[0, :mesh.ny])
        if ox > 0:
            J[1, :mesh.ny] += wj * ox * np.einsum("bk,bk->b", P[j, :, -1, :], fi[1, :mesh.ny])
        if oy < 0:
            J[2, :mesh.nx] += wj * (-oy) * np.einsum("ak,ak->a", P[j, 0, :, :], fi[2, :mesh.nx])
        if oy > 0:
            J[3, :mesh.nx] += wj * oy * np.einsum("ak,ak->a", P[j, -1, :, :], fi[3, :mesh.nx])
    with np.errstate(invalid="ignore", divide="ignore"):
        J = np.where(flen > 0, J / np.where(flen > 0, flen, 1.0), 0.0)
    return J


def all_psi(prob, phi, nthreads=0):
    """psi_j for every ordinate from a converged scalar flux (one sweep, eq. (SI))."""
    src = prob.sig_s4 * phi + prob.G
    psi, _ = sweep.sweep(prob.mesh, prob.dirs, np.arange(prob.nd), prob.sigma_t, src, prob.bnd,
                         want_psi=True, nthreads=nthreads)
    return psi


def adjoint_si_dsa(prob, bnd_adj, eps, max_outer=500, nthreads=0):
    """Solve the adjoint system by SI-DSA with transposed sweeps; returns Phi_mu."""
    phi_prev = np.zeros(prob.mesh.ndof)
    for n in range(1, max_outer + 1):
        src = prob.sig_s4 * phi_prev
        _, phi_star = sweep.sweep(prob.mesh, prob.dirs, np.arange(prob.nd), prob.sigma_t, src,
                                  bnd_adj, want_psi=False, w=prob.w, transpose=True,
                                  nthreads=nthreads)
        if np.max(np.abs(phi_star - phi_prev)) <= eps:
            return phi_star, n
        phi_prev = phi_star + prob.dsa().correction(phi_star, phi_prev)
    raise RuntimeError("adjoint SI-DSA did not converge")


def loss(prob, J_obs, eps=1e-13, nthreads=0):
    fr = si.fr_si_dsa(prob, eps, max_outer=2000, nthreads=nthreads)
    psi = all_psi(prob, fr["phi"], nthreads)
    J = exit_currents(prob, psi)
    return 0.5 * float(np.sum((J - J_obs) ** 2)), J, fr["phi"], psi


def loss_and_grad(prob, J_obs, eps=1e-13, nthreads=0):
    """L, J and dL/dsigma_a, dL/dsigma_s per cell, by the discrete adjoint."""
    L, J, phi, psi = loss(prob, J_obs, eps, nthreads)
    mesh = prob.mesh
    flen = face_lengths(mesh)
    wface = np.where(flen > 0, (J - J_obs) / np.where(flen > 0, flen, 1.0), 0.0)
    bc_adj = np.zeros((4, max(mesh.nx, mesh.ny), 2))
    bc_adj[:, :, 0] = wface * np.sqrt(np.where(flen > 0, flen, 0.0))
    bnd_adj = dg.boundary_unit_vectors(mesh, bc_adj)
    phi_mu, _ = adjoint_si_dsa(prob, bnd_adj, eps, nthreads=nthreads)
    mu, _ = sweep.sweep(mesh, prob.dirs, np.arange(prob.nd), prob.sigma_t, prob.sig_s4 * phi_mu,
                        bnd_adj, want_psi=True, transpose=True, nthreads=nthreads)
    prod = np.einsum("j,jck->c", prob.w, (mu * psi).reshape(prob.nd, mesh.ncell, 4))
    g_a = -prod
    g_s = g_a + np.einsum("ck,ck->c", phi_mu.reshape(-1, 4), phi.reshape(-1, 4))
    return dict(loss=L, J=J, grad_sigma_a=g_a, grad_sigma_s=g_s, phi=phi, phi_adj=phi_mu,
                bc_adj=bc_adj)


def with_sigma(prob, sigma_a=None, sigma_s=None):
    sa = prob.sigma_t - prob.sigma_s if sigma_a is None else sigma_a
    ss = prob.sigma_s if sigma_s is None else sigma_s
    return si.Problem(prob.mesh, prob.dirs, prob.w, sa + ss, ss, prob.G, prob.bc)


def fd_grad_sigma_a(prob, J_obs, cells, h=1e-6, eps=1e-13, nthreads=0):
    """Central finite differences of L in sigma_a at the given cells."""
    sa = prob.sigma_t - prob.sigma_s
    out = []
    for c in cells:
        vals = []
        for sgn in (1.0, -1.0):
            s2 = sa.copy(); s2[c] += sgn * h
            vals.append(loss(with_sigma(prob, sigma_a=s2), J_obs, eps, nthreads)[0])
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)
