"""Implicit time marching of the oracle: backward Euler (the extension outlined in Sec. 3.7).

Test infrastructure only: the GPU library never imports this package.

With unit particle speed, a backward Euler step of size dt of
    d psi/dt + Omega . grad psi + sigma_t psi = sigma_s phi + Q
is, after the S_N-DG discretisation of Sec. 2.1, eq. (mat-vec-a) with the total cross
section Sigma_t + M/dt and the extra right-hand side M psi_j^m / dt for ordinate j.  M, the
mass matrix of the orthonormal Legendre basis, is the identity, so the step is the steady
problem with sigma_t + 1/dt per cell and the angular source psi_j^m / dt.  The SI-DSA of
Sec. 2.2 (full rank) or the low-rank SI-DSA of Sec. 3 solves it; the DSA acts on the
step's cross sections (sigma_a + 1/dt, D = 1/(3 (sigma_t + 1/dt))).

Readings (also implemented by the GPU library):
  * unit speed (the paper writes the step's operator as Sigma_t + M/dt);
  * the step's psi^{m+1}: full rank, the psi of the last SI sweep (the one that gives the
    returned phi^{n,*}); low rank, X S V^T of the truncation after the last outer
    iteration (Sec. 3.3: one truncation after the outer loop is enough to carry psi);
  * the low-rank step starts every outer iteration from an empty basis, as the steady
    solve does; psi^m enters only through the right-hand side.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import lowrank, si, sweep


def step_problem(prob, dt):
    """The steady problem of one step: sigma_t + 1/dt, the same sigma_s, Q and inflow."""
    return si.Problem(prob.mesh, prob.dirs, prob.w, prob.sigma_t + 1.0 / dt, prob.sigma_s,
                      prob.G, prob.bc)


def fr_step(prob, dt, psi_prev, eps_si, max_outer=200, phi0=None, use_dsa=True):
    """Full-rank SI-DSA of one step; every ordinate j is swept with
    Sigma_s phi + G + psi_prev[j] / dt.  Returns dict(phi, psi, iters, converged, history)."""
    p2 = step_problem(prob, dt)
    n = prob.mesh.ndof
    extra = np.zeros((prob.nd, n)) if psi_prev is None else np.asarray(psi_prev) / dt
    phi_prev = np.zeros(n) if phi0 is None else np.asarray(phi0, dtype=np.float64).copy()
    hist = []
    phi_star, psi = phi_prev, None
    for it in range(1, max_outer + 1):
        src = p2.sig_s4 * phi_prev + p2.G
        psi = np.concatenate([sweep.sweep(p2.mesh, p2.dirs, [j], p2.sigma_t, src + extra[j],
                                          p2.bnd, want_psi=True)[0] for j in range(p2.nd)])
        phi_star = p2.w @ psi
        d = float(np.max(np.abs(phi_star - phi_prev)))
        hist.append(d)
        if d <= eps_si:
            return dict(phi=phi_star, psi=psi, iters=it, converged=True, history=hist)
        phi_prev = phi_star + p2.dsa().correction(phi_star, phi_prev) if use_dsa else phi_star
    return dict(phi=phi_star, psi=psi, iters=max_outer, converged=False, history=hist)


def brute_force_step(prob, dt, psi_prev):
    """Direct sparse solve of the step's coupled system (tiny grids only)."""
    p2 = step_problem(prob, dt)
    n = prob.mesh.ndof
    extra = np.zeros((prob.nd, n)) if psi_prev is None else np.asarray(psi_prev) / dt
    rhs = np.concatenate([p2.G + p2.g_bc(j) + extra[j] for j in range(p2.nd)])
    psi = spla.spsolve(si.coupled_matrix(p2), rhs).reshape(p2.nd, n)
    return psi, p2.w @ psi


def lr_step(prob, dt, psi_prev, eps_si, p, q, eps_res, eps_diff, eps_svd, rand, **kw):
    """Low-rank SI-DSA of one step (Alg. 1 with the angular source); psi of the step from
    the truncated factors, psi = (X S V^T)^T [N_Omega][ndof]."""
    p2 = step_problem(prob, dt)
    extra = None if psi_prev is None else np.asarray(psi_prev) / dt
    out = lowrank.lr_si_dsa(p2, eps_si, p, q, eps_res, eps_diff, eps_svd, rand, extra=extra, **kw)
    out["psi"] = (out["X"] @ np.diag(out["S"]) @ out["V"].T).T
    return out
