"""Upwind DG-Q1 discretisation of the S_N equations on a 2D Cartesian mesh.

Follows Sec. 2.1 (weak form with upwind traces, the upwind-flux definition and the
boundary fluxes) and Appendix B (matrix definitions).  Everything here is computed
from the weak form by 2-point Gauss quadrature (exact for products of Q1
functions), not from closed-form cell matrices, so that it can be read against the
weak form directly.

Readings (the paper only says "an orthonormal basis", Sec. 2.1 / Appendix B):
  * cell basis: eta_{pq}(x, y) = l_p(x) l_q(y), with l_0 = 1/sqrt(h) and
    l_1 = sqrt(3) xi / sqrt(h), xi in [-1, 1] the cell-local coordinate;
    the local DOF index is k = 2 q + p (so k=1 is the x-linear mode);
  * global DOF index ((b * nx + a) * 4 + k) for cell (a, b), a along x, b along y;
  * isotropic inflow data g is given per boundary face segment by two face-Legendre
    moments g_m = int_face g l_m(s) ds (s = y on the left/right sides, s = x on the
    bottom/top sides, l_1 increasing with s); sides are ordered L, R, B, T;
  * the boundary term enters the right-hand side as +|Omega.n| int_face g eta_k
    on inflow faces (the sign printed in Appendix B for g^bc reproduces no constant
    state; the weak form of Sec. 2.1 with psi = g on inflow faces gives this sign).
"""
import numpy as np
import scipy.sparse as sp

GAUSS2 = np.array([-1.0 / np.sqrt(3.0), 1.0 / np.sqrt(3.0)])
SIDES = ("L", "R", "B", "T")


class Mesh:
    """Uniform Cartesian mesh of [x0,x1] x [y0,y1] with nx x ny cells (Sec. 2.1)."""

    def __init__(self, nx, ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
        self.nx, self.ny = int(nx), int(ny)
        self.x0, self.x1, self.y0, self.y1 = float(x0), float(x1), float(y0), float(y1)
        self.hx = (self.x1 - self.x0) / self.nx
        self.hy = (self.y1 - self.y0) / self.ny
        self.ncell = self.nx * self.ny
        self.ndof = 4 * self.ncell

    def xc(self, a):
        return self.x0 + (a + 0.5) * self.hx

    def yc(self, b):
        return self.y0 + (b + 0.5) * self.hy


def leg1(xi, h):
    """Orthonormal 1D Legendre basis on an interval of length h at local xi."""
    return np.array([1.0 / np.sqrt(h), np.sqrt(3.0) * xi / np.sqrt(h)])


def dleg1(h):
    """d/dx of the 1D basis (xi = 2 (x - xc) / h)."""
    return np.array([0.0, np.sqrt(3.0) * 2.0 / h / np.sqrt(h)])


def eta(xi, zeta, hx, hy):
    """Values of the four cell basis functions at local (xi, zeta); k = 2q + p."""
    lx, ly = leg1(xi, hx), leg1(zeta, hy)
    return np.array([lx[0] * ly[0], lx[1] * ly[0], lx[0] * ly[1], lx[1] * ly[1]])


def grad_eta(xi, zeta, hx, hy):
    """(d/dx, d/dy) of the four basis functions at local (xi, zeta)."""
    lx, ly = leg1(xi, hx), leg1(zeta, hy)
    dx, dy = dleg1(hx), dleg1(hy)
    gx = np.array([dx[0] * ly[0], dx[1] * ly[0], dx[0] * ly[1], dx[1] * ly[1]])
    gy = np.array([lx[0] * dy[0], lx[1] * dy[0], lx[0] * dy[1], lx[1] * dy[1]])
    return gx, gy


def cell_mass(hx, hy):
    """int_cell eta_k eta_l (identity for the orthonormal basis)."""
    m = np.zeros((4, 4))
    for xi in GAUSS2:
        for ze in GAUSS2:
            e = eta(xi, ze, hx, hy)
            m += np.outer(e, e) * (hx / 2) * (hy / 2)
    return m


# Face geometry on the reference cell: (outward normal, local coords along the face).
def _face_points(side):
    """Local (xi, zeta) of the 2 Gauss points on a face and the outward normal."""
    if side == "L":
        return [(-1.0, s) for s in GAUSS2], np.array([-1.0, 0.0])
    if side == "R":
        return [(1.0, s) for s in GAUSS2], np.array([1.0, 0.0])
    if side == "B":
        return [(s, -1.0) for s in GAUSS2], np.array([0.0, -1.0])
    if side == "T":
        return [(s, 1.0) for s in GAUSS2], np.array([0.0, 1.0])
    raise ValueError(side)


def _face_len(side, hx, hy):
    return hy if side in ("L", "R") else hx


def cell_transport(Ox, Oy, hx, hy):
    """Cell matrices of the upwind DG weak form for direction (Ox, Oy), Sec. 2.1.

    Returns (A, B) where, for test function eta_k (row) and trial eta_l (column),
      A[k, l] = -int_cell (Omega . grad eta_k) eta_l
                + sum_{outflow faces f} (Omega . n_f) int_f eta_k eta_l,
      B[side][k, l] = |Omega . n_f| int_f eta_k eta_l^nb     (inflow faces only),
    with eta_l^nb the neighbour's basis function evaluated on the shared face.  The
    cell equation is (A + sigma_t I) psi_c = rhs_c + sum_f B[f] psi_nb(f).
    """
    A = np.zeros((4, 4))
    for xi in GAUSS2:
        for ze in GAUSS2:
            gx, gy = grad_eta(xi, ze, hx, hy)
            e = eta(xi, ze, hx, hy)
            A -= np.outer(Ox * gx + Oy * gy, e) * (hx / 2) * (hy / 2)
    B = {}
    for side in SIDES:
        pts, n = _face_points(side)
        on = Ox * n[0] + Oy * n[1]
        L = _face_len(side, hx, hy)
        if on > 0:
            for (xi, ze) in pts:
                e = eta(xi, ze, hx, hy)
                A += on * np.outer(e, e) * (L / 2)
        elif on < 0:
            Bf = np.zeros((4, 4))
            for (xi, ze) in pts:
                e = eta(xi, ze, hx, hy)
                # the same physical point seen from the neighbour across the face
                if side in ("L", "R"):
                    xin, zen = (1.0 if side == "L" else -1.0), ze
                else:
                    xin, zen = xi, (1.0 if side == "B" else -1.0)
                enb = eta(xin, zen, hx, hy)
                Bf += (-on) * np.outer(e, enb) * (L / 2)
            B[side] = Bf
    return A, B


def face_moments_to_vals(gm, s_local, h):
    """Value of the face function with moments gm = (g_0, g_1) at face-local s."""
    return gm[0] / np.sqrt(h) + gm[1] * np.sqrt(3.0) * s_local / np.sqrt(h)


def boundary_unit_vectors(mesh, bc):
    """Per-side unit-flux boundary moments, int_f g eta_k ds, for every boundary cell.

    bc: array [4, max(nx,ny), 2] of face-Legendre moments (sides L, R, B, T), or None.
    Returns bnd [4, max(nx,ny), 4] with bnd[side, i, k] = int_{face i of side} g eta_k.
    The right-hand side of a direction gets |Omega . n| bnd[side] on its inflow sides
    (Appendix B, g^bc, with the sign of the weak form, see the module header).
    """
    m = max(mesh.nx, mesh.ny)
    bnd = np.zeros((4, m, 4))
    if bc is None:
        return bnd
    bc = np.asarray(bc, dtype=np.float64)
    hx, hy = mesh.hx, mesh.hy
    for si, side in enumerate(SIDES):
        pts, _ = _face_points(side)
        L = _face_len(side, hx, hy)
        count = mesh.ny if side in ("L", "R") else mesh.nx
        for i in range(count):
            acc = np.zeros(4)
            for (xi, ze) in pts:
                s_loc = ze if side in ("L", "R") else xi
                g = face_moments_to_vals(bc[si, i], s_loc, L)
                acc += g * eta(xi, ze, hx, hy) * (L / 2)
            bnd[si, i] = acc
    return bnd


def boundary_vector(mesh, bnd, Ox, Oy):
    """g_j^bc for direction (Ox, Oy): |Omega.n| bnd on the inflow sides (Appendix B)."""
    g = np.zeros((mesh.ny, mesh.nx, 4))
    if Ox > 0:
        g[:, 0, :] += Ox * bnd[0, :mesh.ny]
    elif Ox < 0:
        g[:, -1, :] += -Ox * bnd[1, :mesh.ny]
    if Oy > 0:
        g[0, :, :] += Oy * bnd[2, :mesh.nx]
    elif Oy < 0:
        g[-1, :, :] += -Oy * bnd[3, :mesh.nx]
    return g.reshape(-1)


def assemble_transport(mesh, Ox, Oy):
    """Sparse D(Omega) of eq. (mat-vec-a) without the cross section (Appendix B)."""
    A, B = cell_transport(Ox, Oy, mesh.hx, mesh.hy)
    nx, ny = mesh.nx, mesh.ny
    rows, cols, vals = [], [], []
    k4 = np.arange(4)
    for b in range(ny):
        for a in range(nx):
            c = b * nx + a
            r = 4 * c + k4
            rows.append(np.repeat(r, 4)); cols.append(np.tile(r, 4)); vals.append(A.reshape(-1))
            for side, Bf in B.items():
                na, nb = a, b
                if side == "L":
                    na -= 1
                elif side == "R":
                    na += 1
                elif side == "B":
                    nb -= 1
                else:
                    nb += 1
                if 0 <= na < nx and 0 <= nb < ny:
                    cn = nb * nx + na
                    rows.append(np.repeat(r, 4)); cols.append(np.tile(4 * cn + k4, 4))
                    vals.append(-Bf.reshape(-1))
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.ndof, mesh.ndof))


def cell_sigma_diag(mesh, sigma):
    """Sigma (Appendix B) for a per-cell constant cross section: diag(sigma_c) x I_4."""
    sigma = np.asarray(sigma, dtype=np.float64).reshape(-1)
    return sp.diags(np.repeat(sigma, 4))


def directional_operators(mesh):
    """D_x^-, D_x^+, D_y^-, D_y^+ of eq. (upwind-operator) / Appendix B.

    D_j = Omega_x D_x^{-/+} + Omega_y D_y^{-/+} with '-' for a non-negative
    component.  D_x^- is D((1,0)); for Omega_x < 0, Omega_x D_x^+ = D((Omega_x, 0)),
    hence D_x^+ = -D((-1, 0)).
    """
    Dxm = assemble_transport(mesh, 1.0, 0.0)
    Dxp = -assemble_transport(mesh, -1.0, 0.0)
    Dym = assemble_transport(mesh, 0.0, 1.0)
    Dyp = -assemble_transport(mesh, 0.0, -1.0)
    return Dxm, Dxp, Dym, Dyp


def source_moments_box(mesh, value, box, nq=4):
    """Moments G_k = int_cell G eta_k (Appendix B) of G = value on an axis box.

    box = (xlo, xhi, ylo, yhi).  Integrated exactly: Gauss rule on the part of each
    cell inside the box (the integrand is polynomial there).
    """
    xlo, xhi, ylo, yhi = box
    xg, wg = np.polynomial.legendre.leggauss(nq)
    G = np.zeros((mesh.ny, mesh.nx, 4))
    for b in range(mesh.ny):
        ya, yb = mesh.y0 + b * mesh.hy, mesh.y0 + (b + 1) * mesh.hy
        lo_y, hi_y = max(ya, ylo), min(yb, yhi)
        if hi_y <= lo_y:
            continue
        for a in range(mesh.nx):
            xa, xb = mesh.x0 + a * mesh.hx, mesh.x0 + (a + 1) * mesh.hx
            lo_x, hi_x = max(xa, xlo), min(xb, xhi)
            if hi_x <= lo_x:
                continue
            acc = np.zeros(4)
            for i in range(nq):
                x = 0.5 * (lo_x + hi_x) + 0.5 * (hi_x - lo_x) * xg[i]
                for j in range(nq):
                    y = 0.5 * (lo_y + hi_y) + 0.5 * (hi_y - lo_y) * xg[j]
                    xi = 2 * (x - mesh.xc(a)) / mesh.hx
                    ze = 2 * (y - mesh.yc(b)) / mesh.hy
                    acc += value * eta(xi, ze, mesh.hx, mesh.hy) * wg[i] * wg[j] \
                        * 0.25 * (hi_x - lo_x) * (hi_y - lo_y)
            G[b, a] = acc
    return G.reshape(-1)


def source_moments_function(mesh, f, nq=6):
    """Moments int_cell f eta_k of a smooth source f(x, y) by an nq x nq Gauss rule."""
    xg, wg = np.polynomial.legendre.leggauss(nq)
    G = np.zeros((mesh.ny, mesh.nx, 4))
    for b in range(mesh.ny):
        for a in range(mesh.nx):
            acc = np.zeros(4)
            for i in range(nq):
                for j in range(nq):
                    x = mesh.xc(a) + 0.5 * mesh.hx * xg[i]
                    y = mesh.yc(b) + 0.5 * mesh.hy * xg[j]
                    acc += f(x, y) * eta(xg[i], xg[j], mesh.hx, mesh.hy) * wg[i] * wg[j] \
                        * 0.25 * mesh.hx * mesh.hy
            G[b, a] = acc
    return G.reshape(-1)
