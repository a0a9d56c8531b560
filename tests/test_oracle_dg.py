"""Pins of the oracle's DG-Q1 discretisation and transport sweep (Sec. 2.1-2.2, Appendix B)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dg, quadrature, sweep


def rand_problem(nx=5, ny=4, seed=0):
    m = dg.Mesh(nx, ny, 0.0, 1.3, -0.2, 0.5)
    d, w = quadrature.cl_quadrature(8, 4)
    rng = np.random.default_rng(seed)
    sig = rng.uniform(0.3, 3.0, m.ncell)
    src = rng.normal(size=m.ndof)
    bnd = dg.boundary_unit_vectors(m, rng.normal(size=(4, max(nx, ny), 2)))
    return m, d, w, sig, src, bnd


def test_mass_is_identity():
    assert np.allclose(dg.cell_mass(0.3, 0.7), np.eye(4), atol=1e-15)


def test_sweep_equals_direct_solve():
    """One upwind pass solves (D_j + Sigma_t) psi = rhs exactly (Sec. 2.2)."""
    m, d, w, sig, src, bnd = rand_problem()
    psi, phi = sweep.sweep(m, d, np.arange(len(w)), sig, src, bnd, w=w)
    for j in range(len(w)):
        A = (dg.assemble_transport(m, d[j, 0], d[j, 1]) + dg.cell_sigma_diag(m, sig)).tocsc()
        x = spla.spsolve(A, src + dg.boundary_vector(m, bnd, d[j, 0], d[j, 1]))
        assert np.abs(x - psi[j]).max() < 1e-13 * max(1.0, np.abs(x).max())
    assert np.abs(phi - w @ psi).max() < 1e-14


def test_transposed_sweep_and_reverse_identity():
    """(D_j+Sigma_t)^T solve; D(Omega)^T = D(-Omega); adjoint sweep = sweep of -Omega."""
    m, d, w, sig, src, bnd = rand_problem(seed=1)
    rv = quadrature.reverse_index(8, 4)
    for j in range(0, len(w), 3):
        A = (dg.assemble_transport(m, d[j, 0], d[j, 1]) + dg.cell_sigma_diag(m, sig)).tocsc()
        Ar = dg.assemble_transport(m, d[rv[j], 0], d[rv[j], 1]) + dg.cell_sigma_diag(m, sig)
        assert abs(A.T - Ar).max() < 1e-13
        mu, _ = sweep.sweep(m, d, [j], sig, src, bnd, transpose=True)
        rhs = src + dg.boundary_vector(m, bnd, -d[j, 0], -d[j, 1])
        assert np.abs(spla.spsolve(A.T.tocsc(), rhs) - mu[0]).max() < 1e-12
        fw, _ = sweep.sweep(m, d, [rv[j]], sig, src, bnd)
        assert np.abs(fw[0] - mu[0]).max() < 1e-12
        # dot-product test <b2, A^{-1} b1> = <A^{-T} b2, b1>
        b1 = np.random.default_rng(j).normal(size=m.ndof)
        y1, _ = sweep.sweep(m, d, [j], sig, b1, None)
        y2, _ = sweep.sweep(m, d, [j], sig, src, None, transpose=True)
        assert abs(src @ y1[0] - y2[0] @ b1) < 1e-12 * abs(src @ y1[0])


def test_quadrant_decomposition():
    """D_j = Omega_x D_x^{-/+} + Omega_y D_y^{-/+}, eq. (upwind-operator); (D_x^-)^T = -D_x^+."""
    m = dg.Mesh(4, 3, 0.0, 1.0, 0.0, 2.0)
    Dxm, Dxp, Dym, Dyp = dg.directional_operators(m)
    assert abs(Dxm.T + Dxp).max() < 1e-13 and abs(Dym.T + Dyp).max() < 1e-13
    for ox, oy in [(0.3, 0.5), (0.3, -0.5), (-0.3, 0.5), (-0.7, -0.1)]:
        D = dg.assemble_transport(m, ox, oy)
        E = ox * (Dxm if ox >= 0 else Dxp) + oy * (Dym if oy >= 0 else Dyp)
        assert abs(D - E).max() < 1e-13


def test_block_lower_triangular_in_upwind_order():
    """Sec. 2.2: ordered along the upwind direction the operator is block lower triangular."""
    m = dg.Mesh(4, 3)
    for ox, oy in [(0.3, 0.5), (-0.3, 0.5), (0.3, -0.5), (-0.3, -0.5)]:
        D = dg.assemble_transport(m, ox, oy).toarray()
        order = []
        for ib in range(m.ny):
            b = ib if oy > 0 else m.ny - 1 - ib
            for ia in range(m.nx):
                a = ia if ox > 0 else m.nx - 1 - ia
                order.append(b * m.nx + a)
        perm = np.concatenate([4 * c + np.arange(4) for c in order])
        P = D[np.ix_(perm, perm)]
        for r in range(m.ncell - 1):
            assert np.abs(P[4 * r:4 * r + 4, 4 * (r + 1):]).max() == 0.0


def test_constant_state():
    """sigma_s = 0, G = sigma_t c, inflow g = c  =>  psi_j = c everywhere, all j."""
    m = dg.Mesh(6, 5, 0.0, 2.0, 0.0, 1.0)
    d, w = quadrature.cl_quadrature(8, 4)
    c = 1.7
    sig = np.random.default_rng(2).uniform(0.5, 4.0, m.ncell)
    G = np.zeros((m.ncell, 4)); G[:, 0] = sig * c * np.sqrt(m.hx * m.hy)
    bc = np.zeros((4, 6, 2)); bc[0:2, :, 0] = c * np.sqrt(m.hy); bc[2:4, :, 0] = c * np.sqrt(m.hx)
    psi, _ = sweep.sweep(m, d, np.arange(32), sig, G.reshape(-1), dg.boundary_unit_vectors(m, bc))
    exp = np.zeros((m.ncell, 4)); exp[:, 0] = c * np.sqrt(m.hx * m.hy)
    assert np.abs(psi - exp.reshape(-1)).max() < 1e-14


def test_pade_transmission_pin():
    """Pure absorber, left inflow 1, bottom inflow = the 1D DG profile: in cell a the
    coefficients are sqrt(hx hy) T^a (tau+6, -sqrt3 tau, 0, 0)/(tau^2+4tau+6) with the
    (1,2) Pade transmission T = (6-2tau)/(tau^2+4tau+6), tau = sigma hx / Omega_x.
    (Derived by hand from the cell equations of Sec. 2.1.)"""
    nx, ny = 7, 3
    m = dg.Mesh(nx, ny, 0.0, 0.7, 0.0, 0.3)
    sig = 2.5
    d = np.array([[0.6, 0.3, np.sqrt(1 - 0.45)]])
    tau = sig * m.hx / 0.6
    den = tau * tau + 4 * tau + 6
    T = (6 - 2 * tau) / den
    prof = np.array([[T ** a * (tau + 6) / den, -np.sqrt(3) * tau * T ** a / den] for a in range(nx)])
    bc = np.zeros((4, nx, 2))
    bc[0, :ny, 0] = np.sqrt(m.hy)                 # g = 1 on the left side
    bc[2, :, :] = np.sqrt(m.hx) * prof            # 1D profile on the bottom side
    psi, _ = sweep.sweep(m, d, [0], sig * np.ones(m.ncell), np.zeros(m.ndof),
                         dg.boundary_unit_vectors(m, bc))
    P = psi[0].reshape(ny, nx, 4)
    for b in range(ny):
        for a in range(nx):
            exp = np.sqrt(m.hx * m.hy) * np.array([prof[a, 0], prof[a, 1], 0.0, 0.0])
            assert np.abs(P[b, a] - exp).max() < 1e-14


def test_attenuation_converges_to_exponential():
    """Purely absorbing medium: the DG solution tends to exp(-sigma_t s) with O(h^2)."""
    sig, ox, oy = 3.0, 0.8, 0.4
    errs = []
    for n in (8, 16, 32, 64):
        m = dg.Mesh(n, 2, 0.0, 1.0, 0.0, 2.0 / n)
        d = np.array([[ox, oy, np.sqrt(1 - ox * ox - oy * oy)]])
        # exact psi = exp(-sig x/ox) is y-independent: bottom data = its face moments
        xg, wg = np.polynomial.legendre.leggauss(8)
        bc = np.zeros((4, n, 2))
        bc[0, :2, 0] = np.sqrt(m.hy)
        for a in range(n):
            x = m.xc(a) + 0.5 * m.hx * xg
            f = np.exp(-sig * x / ox)
            bc[2, a, 0] = np.sum(wg * f / np.sqrt(m.hx)) * m.hx / 2
            bc[2, a, 1] = np.sum(wg * f * np.sqrt(3) * xg / np.sqrt(m.hx)) * m.hx / 2
        psi, _ = sweep.sweep(m, d, [0], sig * np.ones(m.ncell), np.zeros(m.ndof),
                             dg.boundary_unit_vectors(m, bc))
        avg = psi[0].reshape(2, n, 4)[0, :, 0] / np.sqrt(m.hx * m.hy)
        xa, xb = np.arange(n) * m.hx, (np.arange(n) + 1) * m.hx
        exact = (np.exp(-sig * xa / ox) - np.exp(-sig * xb / ox)) * ox / sig / m.hx
        errs.append(np.sqrt(np.mean((avg - exact) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.8, (errs, rates)


def test_sweep_particle_balance():
    """Test function 1 in the weak form: sigma_t int psi + outflow - inflow = int rhs."""
    m, d, w, sig, src, bnd = rand_problem(seed=5)
    psi, _ = sweep.sweep(m, d, np.arange(len(w)), sig, src, bnd)
    one = np.zeros((m.ncell, 4)); one[:, 0] = np.sqrt(m.hx * m.hy)
    fi = np.zeros((4, max(m.nx, m.ny), 2))
    fi[0:2, :, 0] = np.sqrt(m.hy); fi[2:4, :, 0] = np.sqrt(m.hx)
    fint = dg.boundary_unit_vectors(m, fi)            # int_face eta_k
    for j in range(len(w)):
        P = psi[j].reshape(m.ny, m.nx, 4)
        ox, oy = d[j, 0], d[j, 1]
        out = 0.0
        out += abs(ox) * np.sum(P[:, -1 if ox > 0 else 0, :] * fint[1 if ox > 0 else 0, :m.ny])
        out += abs(oy) * np.sum(P[-1 if oy > 0 else 0, :, :] * fint[3 if oy > 0 else 2, :m.nx])
        inflow = np.sum(dg.boundary_vector(m, bnd, ox, oy).reshape(-1, 4) * one)
        lhs = np.sum(sig[:, None] * psi[j].reshape(-1, 4) * one) + out - inflow
        rhs = np.sum(src.reshape(-1, 4) * one)
        assert abs(lhs - rhs) < 1e-12 * (1 + abs(rhs))


# ---------------------------------------------------------------------------
# Source moments G_k = int_cell G eta_k (Appendix B), pinned by closed forms.
# With xi = 2 (x - x_c)/h_x and zeta = 2 (y - y_c)/h_y the orthonormal basis is
# (1, sqrt3 xi, sqrt3 zeta, 3 xi zeta) / sqrt(h_x h_y), local index k = 2q + p, so a
# separable source f(x) g(y) has moments (1/sqrt(h_x h_y)) * Fx_p * Fy_q with
#   F_0 = int f,  F_1 = sqrt3 int xi f.
# ---------------------------------------------------------------------------

def _box_1d(lo, hi, c, h):
    """Moments (int 1, sqrt3 int xi) of the indicator of [lo, hi] over one cell."""
    if hi <= lo:
        return 0.0, 0.0
    xl, xh = 2.0 * (lo - c) / h, 2.0 * (hi - c) / h      # xi at the ends
    return hi - lo, np.sqrt(3.0) * 0.25 * h * (xh * xh - xl * xl)


def test_box_source_fully_covered_cell():
    """A cell inside the box gets (v sqrt(h_x h_y), 0, 0, 0): the only mode of a constant."""
    m = dg.Mesh(6, 5, 0.0, 1.2, -0.5, 0.5)
    v = 2.5
    G = dg.source_moments_box(m, v, (-1.0, 2.0, -1.0, 1.0)).reshape(m.ny, m.nx, 4)
    expect = np.array([v * np.sqrt(m.hx * m.hy), 0.0, 0.0, 0.0])
    assert np.abs(G - expect).max() < 1e-14


def test_box_source_partial_cells_closed_form():
    """Cells cut by the box: separable linear moments of the covered rectangle."""
    m = dg.Mesh(7, 5, -0.3, 1.1, 0.2, 0.9)
    box = (0.137, 0.61, 0.33, 0.77)
    v = 1.7
    G = dg.source_moments_box(m, v, box).reshape(m.ny, m.nx, 4)
    s = 1.0 / np.sqrt(m.hx * m.hy)
    n_cut = 0
    for b in range(m.ny):
        y0, y1 = m.y0 + b * m.hy, m.y0 + (b + 1) * m.hy
        fy = _box_1d(max(y0, box[2]), min(y1, box[3]), 0.5 * (y0 + y1), m.hy)
        for a in range(m.nx):
            x0, x1 = m.x0 + a * m.hx, m.x0 + (a + 1) * m.hx
            fx = _box_1d(max(x0, box[0]), min(x1, box[1]), 0.5 * (x0 + x1), m.hx)
            want = v * s * np.array([fx[0] * fy[0], fx[1] * fy[0], fx[0] * fy[1], fx[1] * fy[1]])
            assert np.abs(G[b, a] - want).max() < 1e-14 * max(1.0, v)
            n_cut += int(abs(fx[1]) > 0 or abs(fy[1]) > 0)
    assert n_cut >= 8          # the box really cuts cells on all four sides
    # total source = v * area of the box (the zeroth moments times sqrt(h_x h_y))
    tot = G[:, :, 0].sum() * np.sqrt(m.hx * m.hy)
    assert abs(tot - v * (box[1] - box[0]) * (box[3] - box[2])) < 1e-14


def _gauss_1d(lo, hi, c, h, alpha, x0):
    """Moments (int e, sqrt3 int xi e) of e(x) = exp(-alpha (x - x0)^2) over [lo, hi]:
    int e = sqrt(pi/alpha)/2 [erf(sqrt(alpha)(x - x0))],
    int (x - x0) e = -[e]/(2 alpha),  and xi = 2 ((x - x0) + (x0 - c))/h."""
    import math
    ra = math.sqrt(alpha)
    i0 = 0.5 * math.sqrt(math.pi / alpha) * (math.erf(ra * (hi - x0)) - math.erf(ra * (lo - x0)))
    i1 = -(math.exp(-alpha * (hi - x0) ** 2) - math.exp(-alpha * (lo - x0) ** 2)) / (2.0 * alpha)
    return i0, np.sqrt(3.0) * 2.0 / h * (i1 + (x0 - c) * i0)


def test_function_source_gaussian_closed_form():
    """Moments of exp(-alpha ((x-cx)^2 + (y-cy)^2)) are products of erf integrals."""
    m = dg.Mesh(9, 7, -1.0, 1.0, -0.8, 0.6)
    alpha, cx, cy, amp = 30.0, 0.13, -0.21, 1.9
    f = lambda x, y: amp * np.exp(-alpha * ((x - cx) ** 2 + (y - cy) ** 2))
    G = dg.source_moments_function(m, f, nq=12).reshape(m.ny, m.nx, 4)
    s = 1.0 / np.sqrt(m.hx * m.hy)
    for b in range(m.ny):
        y0, y1 = m.y0 + b * m.hy, m.y0 + (b + 1) * m.hy
        fy = _gauss_1d(y0, y1, 0.5 * (y0 + y1), m.hy, alpha, cy)
        for a in range(m.nx):
            x0, x1 = m.x0 + a * m.hx, m.x0 + (a + 1) * m.hx
            fx = _gauss_1d(x0, x1, 0.5 * (x0 + x1), m.hx, alpha, cx)
            want = amp * s * np.array([fx[0] * fy[0], fx[1] * fy[0], fx[0] * fy[1], fx[1] * fy[1]])
            assert np.abs(G[b, a] - want).max() < 1e-12 * amp


def test_function_source_polynomial_exact():
    """A bilinear f is reproduced exactly by its four moments (Q1 projection = identity),
    and a quadratic in x has the Legendre-l2 part dropped: int x^2 eta_0 by hand."""
    m = dg.Mesh(4, 3, 0.0, 2.0, 1.0, 2.5)
    f = lambda x, y: 0.7 - 1.3 * x + 2.1 * y + 0.4 * x * y
    G = dg.source_moments_function(m, f, nq=3).reshape(m.ny, m.nx, 4)
    for b in range(m.ny):
        for a in range(m.nx):
            xc, yc = m.xc(a), m.yc(b)
            # f in the local variables: f = A + B xi + C zeta + D xi zeta
            Bx, Cy = 0.5 * m.hx, 0.5 * m.hy
            A = f(xc, yc)
            B = (-1.3 + 0.4 * yc) * Bx
            C = (2.1 + 0.4 * xc) * Cy
            D = 0.4 * Bx * Cy
            # <f, eta_k> = sqrt(h_x h_y) * (A, B/sqrt3, C/sqrt3, D/3)
            want = np.sqrt(m.hx * m.hy) * np.array([A, B / np.sqrt(3.0), C / np.sqrt(3.0), D / 3.0])
            assert np.abs(G[b, a] - want).max() < 1e-13
    g = lambda x, y: x * x + 0.0 * y
    G2 = dg.source_moments_function(m, g, nq=3).reshape(m.ny, m.nx, 4)
    for a in range(m.nx):
        x0, x1 = a * m.hx, (a + 1) * m.hx
        want0 = (x1 ** 3 - x0 ** 3) / 3.0 * m.hy / np.sqrt(m.hx * m.hy)
        assert abs(G2[0, a, 0] - want0) < 1e-13
