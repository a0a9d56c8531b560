"""Diffusion synthetic acceleration of the oracle (Sec. 2.2, eqs. (DSA), (diffusion-correction)).

The paper uses a "fully consistent" diffusion discretisation defined in an external
reference that is not available.  Reading used here (both in this oracle and in the
GPU library): the modified interior penalty (MIP) symmetric DG-Q1 form of Wang and
Ragusa for
    -div(D grad dphi) + sigma_a dphi = sigma_s (phi^{n,*} - phi^{n-1}),
with D = 1/(3 sigma_t) per cell (1/(3 sigma_s) as printed is singular where
sigma_s = 0; sum_j w_j Omega_x^2 = 1/3 makes 1/3 the quadrature-consistent factor).
On the same orthonormal Q1 basis as the transport (oracle.dg) the bilinear form is

  b(u, v) = sum_K (D grad u, grad v)_K + (sigma_a u, v)_K
          + sum_{interior e} k_e ([[u]],[[v]])_e + ({{D d_n u}},[[v]])_e + ([[u]],{{D d_n v}})_e
          + sum_{boundary e} k_e (u, v)_e - 1/2 (D d_n u, v)_e - 1/2 (u, D d_n v)_e

with n pointing from the "-" to the "+" cell, [[u]] = u+ - u-, {{.}} the average,
n outward on the boundary, and the penalty
    k_e = max(1/4, (C/2)(D-/h- + D+/h+))   (interior),   max(1/4, C D-/h-)  (boundary),
h the cell width normal to the face and C = 4 p (p+1) = 8 for Q1.
The correction dphi solves b(dphi, v) = (sigma_s (phi* - phi_prev), v); the oracle
solves it by a sparse LU (scipy), i.e. exactly up to rounding.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg

C_IP = 8.0


def _grad_vals(xi, ze, hx, hy):
    return dg.grad_eta(xi, ze, hx, hy)


def mip_matrix(mesh, sigma_t, sigma_s, c_ip=C_IP):
    """Assemble the MIP matrix [b(eta_l, eta_k)]_{k,l} (rows = test functions)."""
    nx, ny, hx, hy = mesh.nx, mesh.ny, mesh.hx, mesh.hy
    sigma_t = np.asarray(sigma_t, dtype=np.float64).reshape(ny, nx)
    sigma_s = np.asarray(sigma_s, dtype=np.float64).reshape(ny, nx)
    if np.any(sigma_t <= 0):
        raise ValueError("DSA needs sigma_t > 0 in every cell")
    D = 1.0 / (3.0 * sigma_t)
    sa = sigma_t - sigma_s
    g = dg.GAUSS2
    # cell stiffness for D = 1 (shared by all cells of the uniform mesh)
    Kc = np.zeros((4, 4))
    for xi in g:
        for ze in g:
            gx, gy = _grad_vals(xi, ze, hx, hy)
            Kc += (np.outer(gx, gx) + np.outer(gy, gy)) * (hx / 2) * (hy / 2)
    Mc = dg.cell_mass(hx, hy)
    rows, cols, vals = [], [], []

    def add(dofs_r, dofs_c, blk):
        rows.append(np.repeat(dofs_r, len(dofs_c)))
        cols.append(np.tile(dofs_c, len(dofs_r)))
        vals.append(blk.reshape(-1))

    def dofs(a, b):
        return 4 * (b * nx + a) + np.arange(4)

    for b in range(ny):
        for a in range(nx):
            add(dofs(a, b), dofs(a, b), D[b, a] * Kc + sa[b, a] * Mc)
    # interior vertical faces: "-" = (a, b), "+" = (a+1, b), n = +x
    for b in range(ny):
        for a in range(nx - 1):
            Dm, Dp = D[b, a], D[b, a + 1]
            kap = max(0.25, 0.5 * c_ip * (Dm / hx + Dp / hx))
            blk = np.zeros((8, 8))
            for ze in g:
                em, ep = dg.eta(1.0, ze, hx, hy), dg.eta(-1.0, ze, hx, hy)
                gm = dg.grad_eta(1.0, ze, hx, hy)[0]
                gp = dg.grad_eta(-1.0, ze, hx, hy)[0]
                jump = np.concatenate([-em, ep])
                avg = np.concatenate([0.5 * Dm * gm, 0.5 * Dp * gp])
                blk += (kap * np.outer(jump, jump) + np.outer(jump, avg) + np.outer(avg, jump)) * (hy / 2)
            d8 = np.concatenate([dofs(a, b), dofs(a + 1, b)])
            add(d8, d8, blk)
    # interior horizontal faces: "-" = (a, b), "+" = (a, b+1), n = +y
    for b in range(ny - 1):
        for a in range(nx):
            Dm, Dp = D[b, a], D[b + 1, a]
            kap = max(0.25, 0.5 * c_ip * (Dm / hy + Dp / hy))
            blk = np.zeros((8, 8))
            for xi in g:
                em, ep = dg.eta(xi, 1.0, hx, hy), dg.eta(xi, -1.0, hx, hy)
                gm = dg.grad_eta(xi, 1.0, hx, hy)[1]
                gp = dg.grad_eta(xi, -1.0, hx, hy)[1]
                jump = np.concatenate([-em, ep])
                avg = np.concatenate([0.5 * Dm * gm, 0.5 * Dp * gp])
                blk += (kap * np.outer(jump, jump) + np.outer(jump, avg) + np.outer(avg, jump)) * (hx / 2)
            d8 = np.concatenate([dofs(a, b), dofs(a, b + 1)])
            add(d8, d8, blk)
    # boundary faces (outward normal)
    for b in range(ny):
        for a in range(nx):
            for side in ("L", "R", "B", "T"):
                if side == "L" and a != 0: continue
                if side == "R" and a != nx - 1: continue
                if side == "B" and b != 0: continue
                if side == "T" and b != ny - 1: continue
                h = hx if side in ("L", "R") else hy
                flen = hy if side in ("L", "R") else hx
                kap = max(0.25, c_ip * D[b, a] / h)
                blk = np.zeros((4, 4))
                for s in g:
                    if side == "L": xi, ze, n = -1.0, s, (-1.0, 0.0)
                    elif side == "R": xi, ze, n = 1.0, s, (1.0, 0.0)
                    elif side == "B": xi, ze, n = s, -1.0, (0.0, -1.0)
                    else: xi, ze, n = s, 1.0, (0.0, 1.0)
                    e = dg.eta(xi, ze, hx, hy)
                    gx, gy = dg.grad_eta(xi, ze, hx, hy)
                    dn = D[b, a] * (n[0] * gx + n[1] * gy)
                    blk += (kap * np.outer(e, e) - 0.5 * np.outer(e, dn) - 0.5 * np.outer(dn, e)) * (flen / 2)
                add(dofs(a, b), dofs(a, b), blk)
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.ndof, mesh.ndof))


class DSA:
    """Factorised diffusion correction: delta = A_MIP^{-1} Sigma_s (phi* - phi_prev)."""

    def __init__(self, mesh, sigma_t, sigma_s, c_ip=C_IP):
        self.A = mip_matrix(mesh, sigma_t, sigma_s, c_ip).tocsc()
        self.lu = spla.splu(self.A)
        self.sig_s4 = np.repeat(np.asarray(sigma_s, dtype=np.float64).reshape(-1), 4)

    def correction(self, phi_star, phi_prev):
        rhs = self.sig_s4 * (phi_star - phi_prev)
        return self.lu.solve(rhs)
