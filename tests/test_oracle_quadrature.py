"""Pins of the oracle's CL quadrature (Appendix A) against closed forms."""
import math

import numpy as np
import pytest

from oracle import quadrature as Q

RULES = [(4, 2), (8, 4), (16, 8), (32, 8), (32, 16), (64, 16)]


def sphere_monomial(a, b, c):
    """(1/4pi) int_{S^2} x^a y^b z^c dOmega, closed form by Gamma functions."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    g = math.gamma
    val = 2.0 * g((a + 1) / 2) * g((b + 1) / 2) * g((c + 1) / 2) / g((a + b + c + 3) / 2)
    return val / (4.0 * math.pi)


@pytest.mark.parametrize("nt,nz", RULES)
def test_weights_and_moments(nt, nz):
    d, w = Q.cl_quadrature(nt, nz)
    assert d.shape == (nt * nz, 3)
    assert abs(w.sum() - 1.0) < 1e-14
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    assert np.abs(w @ d).max() < 1e-15
    for k in range(3):
        assert abs(w @ d[:, k] ** 2 - 1.0 / 3.0) < 1e-14
    assert abs(w @ (d[:, 0] * d[:, 1])) < 1e-15


@pytest.mark.parametrize("N", [2, 3, 4, 6, 8])
def test_exact_to_degree_2N_minus_1(N):
    """CL(2N, N) integrates every monomial of degree <= 2N - 1 exactly.

    Appendix A states degree 2N; an N-point Gauss rule in Omega_z and a 2N-point
    uniform azimuthal rule are exact only to degree 2N - 1 (z^{2N} is not), which is
    what this pins (recorded as a reading of Appendix A).
    """
    d, w = Q.cl_quadrature(2 * N, N)
    for a in range(2 * N):
        for b in range(2 * N - a):
            for c in range(2 * N - a - b):
                q = w @ (d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c)
                assert abs(q - sphere_monomial(a, b, c)) < 1e-13, (a, b, c)
    q = w @ d[:, 2] ** (2 * N)
    assert abs(q - sphere_monomial(0, 0, 2 * N)) > 1e-6


def test_gauss_nodes_textbook():
    """2- and 3-point Gauss-Legendre nodes and weights (textbook values)."""
    d, w = Q.cl_quadrature(4, 2)
    assert np.allclose(np.unique(np.round(d[:, 2], 15)), [-1 / math.sqrt(3), 1 / math.sqrt(3)])
    d, w = Q.cl_quadrature(4, 3)
    mu = d[::4, 2]
    assert np.allclose(mu, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w[::4] * 4, [5 / 18, 8 / 18, 5 / 18])


def test_azimuths():
    d, _ = Q.cl_quadrature(8, 2)
    th = np.arctan2(d[:8, 1], d[:8, 0]) % (2 * np.pi)
    assert np.allclose(th, (2 * np.arange(1, 9) - 1) * np.pi / 8)


@pytest.mark.parametrize("nt,nz", RULES)
def test_twin_and_reverse(nt, nz):
    d, w = Q.cl_quadrature(nt, nz)
    tw, rv = Q.twin_index(nt, nz), Q.reverse_index(nt, nz)
    assert np.allclose(d[tw, :2], d[:, :2], atol=1e-15) and np.allclose(d[tw, 2], -d[:, 2])
    assert np.allclose(d[rv], -d, atol=1e-15)
    assert np.allclose(w[rv], w) and np.allclose(w[tw], w)
    assert sorted(rv) == list(range(nt * nz)) and sorted(tw) == list(range(nt * nz))


def test_no_axis_aligned_directions():
    """With N_theta = 0 mod 4 no direction has Omega_x = 0 or Omega_y = 0."""
    for nt, nz in RULES:
        d, _ = Q.cl_quadrature(nt, nz)
        assert np.abs(d[:, :2]).min() > 1e-3
