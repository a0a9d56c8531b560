"""Chebyshev-Legendre angular quadrature CL(N_theta, N_z)  (paper, Appendix A).

The rule is the tensor product of the N_z-point Gauss-Legendre rule in Omega_z on
[-1, 1], with weights normalised to sum to one, and the N_theta-point uniform
(Chebyshev) rule on the circle, theta_j = (2j - 1) pi / N_theta for j = 1..N_theta,
each with weight 1/N_theta.  Directions are
    Omega = (cos(theta) sqrt(1 - mu^2), sin(theta) sqrt(1 - mu^2), mu).

Ordering (a reading; the paper only writes j = (j1, j2)): the flat 0-based index is
    j = j2 * N_theta + j1,
with j2 running over the Gauss nodes in ascending mu and j1 over theta.
"""
import numpy as np


def cl_quadrature(n_theta, n_z):
    """Return (dirs [N,3], weights [N]) of CL(n_theta, n_z), Appendix A.

    Weights sum to 1 (normalised S_N weights, Sec. 2.1, the sum of omega_j is one).
    """
    if n_theta < 1 or n_z < 1:
        raise ValueError("CL rule needs n_theta >= 1 and n_z >= 1")
    mu, wz = np.polynomial.legendre.leggauss(n_z)       # ascending nodes on [-1, 1]
    wz = wz / 2.0                                         # normalised: sums to 1
    j1 = np.arange(1, n_theta + 1)
    theta = (2.0 * j1 - 1.0) * np.pi / n_theta            # theta_j = 2 j pi/N - pi/N
    wt = np.full(n_theta, 1.0 / n_theta)
    dirs = np.empty((n_z * n_theta, 3))
    w = np.empty(n_z * n_theta)
    for a in range(n_z):
        s = np.sqrt(1.0 - mu[a] ** 2)
        for b in range(n_theta):
            j = a * n_theta + b
            dirs[j] = (np.cos(theta[b]) * s, np.sin(theta[b]) * s, mu[a])
            w[j] = wz[a] * wt[b]
    return dirs, w


def twin_index(n_theta, n_z):
    """Index of the direction with the same (Omega_x, Omega_y) and opposite Omega_z.

    In 2D X-Y geometry the transport operator depends only on (Omega_x, Omega_y)
    (Sec. 2.1, eq. (upwind-operator)), so a direction and its twin share psi.
    """
    j = np.arange(n_theta * n_z)
    j2, j1 = j // n_theta, j % n_theta
    return (n_z - 1 - j2) * n_theta + j1


def reverse_index(n_theta, n_z):
    """Index of -Omega_j; the CL rule is symmetric under Omega -> -Omega (Appendix A)."""
    if n_theta % 2:
        raise ValueError("the reverse map needs an even n_theta")
    j = np.arange(n_theta * n_z)
    j2, j1 = j // n_theta, j % n_theta
    return (n_z - 1 - j2) * n_theta + (j1 + n_theta // 2) % n_theta
