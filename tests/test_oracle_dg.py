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
