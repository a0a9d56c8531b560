"""Full-rank SI-DSA of the oracle (Sec. 2.2, eqs. (SI), (DSA); outer test as in Alg. 1).

Readings (both here and in the GPU library):
  * the outer stopping test is taken on the un-accelerated SI iterate before the DSA
    step, ||phi^{n,*} - phi^{n-1}||_inf <= eps_si, as Alg. 1 writes it, so that full-
    and low-rank iteration counts compare; the sup norm is over the coefficient
    vector (the bold phi of eq. (mat-vec-a));
  * at the break phi^{n,*} is returned, and the iteration count includes that last
    SI step;
  * the DSA right-hand side is Sigma_s (phi^{n,*} - phi^{n-1}) (the phi^{(n)} of
    eq. (DSA) read as the previous iterate), and phi^{n} = phi^{n,*} + delta.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg, dsa, sweep


class Problem:
    """Discrete S_N-DG problem, eq. (mat-vec-a): mesh, quadrature, cross sections, sources."""

    def __init__(self, mesh, dirs, w, sigma_t, sigma_s, G, bc=None):
        self.mesh = mesh
        self.dirs = np.asarray(dirs, dtype=np.float64)
        self.w = np.asarray(w, dtype=np.float64)
        self.sigma_t = np.asarray(sigma_t, dtype=np.float64).reshape(-1)
        self.sigma_s = np.asarray(sigma_s, dtype=np.float64).reshape(-1)
        self.G = np.asarray(G, dtype=np.float64).reshape(-1)
        self.bc = bc
        self.bnd = dg.boundary_unit_vectors(mesh, bc)
        assert self.sigma_t.size == mesh.ncell and self.G.size == mesh.ndof
        self.nd = len(self.w)
        self.sig_s4 = np.repeat(self.sigma_s, 4)
        self.sig_t4 = np.repeat(self.sigma_t, 4)
        self._dsa = None

    def dsa(self):
        if self._dsa is None:
            self._dsa = dsa.DSA(self.mesh, self.sigma_t, self.sigma_s)
        return self._dsa

    def g_bc(self, j):
        return dg.boundary_vector(self.mesh, self.bnd, self.dirs[j, 0], self.dirs[j, 1])

    def operator(self, j):
        """D_j + Sigma_t assembled for direction j (eq. (mat-vec-a))."""
        return (dg.assemble_transport(self.mesh, self.dirs[j, 0], self.dirs[j, 1])
                + dg.cell_sigma_diag(self.mesh, self.sigma_t)).tocsr()


def si_step(prob, phi_prev, nthreads=0):
    """One SI step, eq. (SI): sweep every ordinate with Sigma_s phi^{n-1} + G~_j."""
    src = prob.sig_s4 * phi_prev + prob.G
    _, phi_star = sweep.sweep(prob.mesh, prob.dirs, np.arange(prob.nd), prob.sigma_t, src,
                              prob.bnd, want_psi=False, w=prob.w, nthreads=nthreads)
    return phi_star


def fr_si_dsa(prob, eps_si, max_outer=100, phi0=None, use_dsa=True, nthreads=0):
    """Full-rank SI-DSA.  Returns dict(phi, iters, converged, history, phis)."""
    phi_prev = np.zeros(prob.mesh.ndof) if phi0 is None else np.asarray(phi0, dtype=np.float64).copy()
    hist, phis = [], []
    phi_star = phi_prev
    for n in range(1, max_outer + 1):
        phi_star = si_step(prob, phi_prev, nthreads)
        d = float(np.max(np.abs(phi_star - phi_prev)))
        hist.append(d)
        phis.append(phi_star)
        if d <= eps_si:
            return dict(phi=phi_star, iters=n, converged=True, history=hist, phis=phis)
        phi_prev = phi_star + prob.dsa().correction(phi_star, phi_prev) if use_dsa else phi_star
    return dict(phi=phi_star, iters=max_outer, converged=False, history=hist, phis=phis)


def coupled_matrix(prob):
    """The whole system of eq. (mat-vec-a), unknowns [psi_1; ...; psi_N] (tiny grids only).

    Block (j, i) = delta_ij (D_j + Sigma_t) - w_i Sigma_s.
    """
    nd, n = prob.nd, prob.mesh.ndof
    blocks = [[None] * nd for _ in range(nd)]
    Ss = sp.diags(prob.sig_s4)
    for j in range(nd):
        for i in range(nd):
            blk = -prob.w[i] * Ss
            if i == j:
                blk = blk + prob.operator(j)
            blocks[j][i] = blk
    return sp.bmat(blocks, format="csc")


def brute_force(prob):
    """Direct sparse solve of the coupled system; returns (psi [N, ndof], phi)."""
    nd, n = prob.nd, prob.mesh.ndof
    rhs = np.concatenate([prob.G + prob.g_bc(j) for j in range(nd)])
    x = spla.spsolve(coupled_matrix(prob), rhs)
    psi = x.reshape(nd, n)
    return psi, prob.w @ psi
