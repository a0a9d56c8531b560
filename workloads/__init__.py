"""Seeded synthetic workloads shared by the tests, the bench and the oracle.

This module holds NO arithmetic of the method: it only describes problems (grid,
domain, quadrature sizes, per-cell cross sections, where the sources are, solver
settings) and draws the random numbers the method consumes.  Moments of sources,
quadrature rules and every step of the solvers are computed separately by the
oracle (oracle/) and by the GPU library (paper_2603_25233_amd/).

The paper's media are analytic (Sec. 4); the five workloads here are synthetic media
of the sizes and structure the benchmark configurations name:

  small_fr       32x32 cells, CL(16,8), sigma_t = 1, sigma_s = 0.99, Q = 1 on
                 [0.4,0.6]^2, vacuum, full-rank SI-DSA to 1e-8.
  checkerboard   256x256 cells, CL(32,16); 8x8 checkerboard of 32x32-cell blocks,
                 block (I,J) diffusive if I+J is even (sigma_t = 1/eps,
                 sigma_s = 1/eps - 0.1 eps, eps = 1e-3), else absorbing
                 (sigma_t = sigma_a = 10); Q = 1 on the block-sized square centred in
                 the domain, [7/16, 9/16]^2; p = 4, q = 32; eps_si = 1e-6,
                 eps_res = eps_diff = 1e-7, eps_svd = 1e-8.
  tomography     256x256 cells, CL(32,8); sigma_a = exp(log 0.1 + 0.5 z) with z a
                 Gaussian-smoothed (8 cells, periodic), re-standardised white noise;
                 sigma_s = 5; 16 boundary point sources (unit isotropic inflow on one
                 boundary face at cells 32, 96, 160, 224 of each side); detectors on
                 all 4 x 256 boundary faces.
  multiscale     1024x1024 cells, CL(64,16); log sigma_t = mu + z with z smoothed at
                 32 cells, mu = ln 100 - 1/2 (arithmetic mean 100); sigma_s = 0.999
                 sigma_t; Q = 1 everywhere; p = 1, q = 8.
  lattice        stand-in for Sec. 4.2's lattice (geometry only in a figure): [0,5]^2,
                 80x80 cells, CL(32,16), 5x5 board of scattering / absorbing unit blocks,
                 Q = 1 in the central (scattering) block; p = 1, q = 8.
The paper's own examples (Sec. 4), on [-1,1]^2 with no absorption (sigma_t = sigma_s),
vacuum boundaries and the Gaussian source exp(-100 (x^2 + y^2)), p = 1, q = 8:
  homogeneous         Sec. 4.1: sigma_s in {0.1, 1, 10, 100}, 16L x 16L cells, CL(8L, 4L).
  variable_scattering Sec. 4.3: sigma_s = 99.9 r^4 (r^2 - 2)^2 + 0.1 for r <= 1, else 100
                      (at the cell centre), 80 x 80 cells, CL(40, 20).
  pin_cell            Sec. 4.4: sigma_s = 0.1 on |x|, |y| <= 0.5, else 100 (at the cell
                      centre; the 80 x 80 mesh resolves the square exactly), CL(32, 16).
The Gaussian source is described twice: `source_gauss` = (amplitude, alpha, centre) for
the library's closed-form moments and `source_fn`, a callable the oracle integrates with
its own quadrature.
A workload can be shrunk (`scaled`) for tests that must finish in seconds; the
structure (block pattern, source placement relative to the domain) is kept.
"""
import numpy as np
from scipy.ndimage import gaussian_filter

SIDE_L, SIDE_R, SIDE_B, SIDE_T = 0, 1, 2, 3


def random_stream(seed, n=1 << 20):
    """uint64 random numbers consumed by the greedy random sampling, in order."""
    return np.random.default_rng(seed).integers(0, np.iinfo(np.uint64).max, size=n,
                                               dtype=np.uint64, endpoint=True)


def smoothed_normal(shape, width_cells, seed):
    """White noise, Gaussian-filtered with periodic wrap, re-standardised to N(0,1)."""
    z = np.random.default_rng(seed).standard_normal(shape)
    z = gaussian_filter(z, sigma=width_cells, mode="wrap")
    z = (z - z.mean()) / z.std()
    return z


class Workload(dict):
    """A problem description.  Keys:
    nx, ny, domain (x0,x1,y0,y1), n_theta, n_z, sigma_t [ny,nx], sigma_s [ny,nx],
    source_boxes [(value, (xlo,xhi,ylo,yhi)), ...], inflow_faces [(side, index, value)],
    eps_si, max_outer, and for the low-rank solver p, q, eps_res, eps_diff, eps_svd,
    eps_mgs, m_max, seed.
    """

    @property
    def n_dirs(self):
        return self["n_theta"] * self["n_z"]

    @property
    def ncell(self):
        return self["nx"] * self["ny"]


def small_fr(n=32, n_theta=16, n_z=8):
    sig_t = np.ones((n, n)); sig_s = 0.99 * np.ones((n, n))
    return Workload(name="small_fr", nx=n, ny=n, domain=(0.0, 1.0, 0.0, 1.0), n_theta=n_theta,
                    n_z=n_z, sigma_t=sig_t, sigma_s=sig_s,
                    source_boxes=[(1.0, (0.4, 0.6, 0.4, 0.6))], inflow_faces=[],
                    eps_si=1e-8, max_outer=200, p=1, q=8, eps_res=1e-9, eps_diff=1e-9,
                    eps_svd=1e-10, eps_mgs=1e-10, m_max=4, seed=11)


def checkerboard(n=256, n_theta=32, n_z=16, blocks=8, eps=1e-3, p=4, q=32):
    bs = n // blocks
    I = np.arange(n) // bs
    diff = ((I[:, None] + I[None, :]) % 2) == 0
    sig_t = np.where(diff, 1.0 / eps, 10.0)
    sig_s = np.where(diff, 1.0 / eps - 0.1 * eps, 0.0)
    half = 0.5 / blocks
    box = (0.5 - half, 0.5 + half, 0.5 - half, 0.5 + half)
    return Workload(name="checkerboard", nx=n, ny=n, domain=(0.0, 1.0, 0.0, 1.0),
                    n_theta=n_theta, n_z=n_z, sigma_t=sig_t, sigma_s=sig_s,
                    source_boxes=[(1.0, box)], inflow_faces=[], eps_si=1e-6, max_outer=100,
                    p=p, q=q, eps_res=1e-7, eps_diff=1e-7, eps_svd=1e-8, eps_mgs=1e-10,
                    m_max=4, seed=22)


def tomography(n=256, n_theta=32, n_z=8, seed=44, smooth=8.0, sigma_s=5.0):
    z = smoothed_normal((n, n), smooth * n / 256.0, seed)
    sig_a = np.exp(np.log(0.1) + 0.5 * z)
    sig_s = sigma_s * np.ones((n, n))
    return Workload(name="tomography", nx=n, ny=n, domain=(0.0, 1.0, 0.0, 1.0), n_theta=n_theta,
                    n_z=n_z, sigma_t=sig_a + sig_s, sigma_s=sig_s, source_boxes=[],
                    inflow_faces=[], eps_si=1e-12, max_outer=2000, seed=seed)


def tomography_sources(n=256):
    """16 point sources: (side, face index) with unit isotropic inflow."""
    idx = [n // 8, 3 * n // 8, 5 * n // 8, 7 * n // 8]
    return [(s, i) for s in (SIDE_L, SIDE_R, SIDE_B, SIDE_T) for i in idx]


def multiscale(n=1024, n_theta=64, n_z=16, seed=55, corr=32.0, log_std=1.0, c=0.999, p=1, q=8):
    z = smoothed_normal((n, n), corr * n / 1024.0, seed)
    mu = np.log(100.0) - 0.5 * log_std ** 2
    sig_t = np.exp(mu + log_std * z)
    return Workload(name="multiscale", nx=n, ny=n, domain=(0.0, 1.0, 0.0, 1.0), n_theta=n_theta,
                    n_z=n_z, sigma_t=sig_t, sigma_s=c * sig_t,
                    source_boxes=[(1.0, (0.0, 1.0, 0.0, 1.0))], inflow_faces=[],
                    eps_si=1e-6, max_outer=100, p=p, q=q, eps_res=1e-7, eps_diff=1e-7,
                    eps_svd=1e-8, eps_mgs=1e-10, m_max=4, seed=seed)


def lattice(n=80, n_theta=32, n_z=16, blocks=5, seed=88, p=1, q=8):
    """Stand-in for the lattice medium of Sec. 4.2, whose geometry is given only in a
    figure: [0, 5]^2, 80 x 80 cells, CL(32, 16); a blocks x blocks board of unit squares,
    block (I, J) scattering (sigma_t = sigma_s = 1) when I + J is even and absorbing
    (sigma_t = sigma_a = 10) otherwise, except the central block, which holds the
    isotropic source Q = 1 and scatters; vacuum boundaries."""
    bs = n // blocks
    I = np.arange(n) // bs
    scat = ((I[:, None] + I[None, :]) % 2) == 0
    c = blocks // 2
    scat[c * bs:(c + 1) * bs, c * bs:(c + 1) * bs] = True
    sig_t = np.where(scat, 1.0, 10.0)
    sig_s = np.where(scat, 1.0, 0.0)
    L = float(blocks)
    box = (c * 1.0, c + 1.0, c * 1.0, c + 1.0)
    return Workload(name="lattice", nx=n, ny=n, domain=(0.0, L, 0.0, L), n_theta=n_theta,
                    n_z=n_z, sigma_t=sig_t, sigma_s=sig_s, source_boxes=[(1.0, box)],
                    inflow_faces=[], eps_si=1e-6, max_outer=100, p=p, q=q, eps_res=1e-7,
                    eps_diff=1e-7, eps_svd=1e-8, eps_mgs=1e-10, m_max=4, seed=seed)


def homogeneous(sigma, L):
    """Sec. 4.1 medium on [-1,1]^2: sigma_a = 0, sigma_s = sigma, 16L x 16L, CL(8L, 4L).

    The Gaussian source exp(-100 (x^2 + y^2)) is returned as a callable; each side
    integrates its moments itself.
    """
    n = 16 * L
    return Workload(name="homogeneous", nx=n, ny=n, domain=(-1.0, 1.0, -1.0, 1.0),
                    n_theta=8 * L, n_z=4 * L, sigma_t=sigma * np.ones((n, n)),
                    sigma_s=sigma * np.ones((n, n)), source_boxes=[], inflow_faces=[],
                    source_fn=gaussian_source, source_gauss=(1.0, 100.0, (0.0, 0.0)),
                    eps_si=1e-6, max_outer=100, p=1, q=8, eps_res=1e-7, eps_diff=1e-7,
                    eps_svd=1e-8, eps_mgs=1e-10, m_max=4, seed=33)


def gaussian_source(x, y):
    """The isotropic source of Sec. 4, exp(-100 (x^2 + y^2))."""
    return np.exp(-100.0 * (x * x + y * y))


def _cell_centres(n, lo=-1.0, hi=1.0):
    h = (hi - lo) / n
    c = lo + h * (np.arange(n) + 0.5)
    return np.meshgrid(c, c, indexing="xy")  # [y][x]


def _paper_example(name, sig_s, n, n_theta, n_z, seed, p=1, q=8):
    return Workload(name=name, nx=n, ny=n, domain=(-1.0, 1.0, -1.0, 1.0), n_theta=n_theta,
                    n_z=n_z, sigma_t=sig_s.copy(), sigma_s=sig_s, source_boxes=[],
                    inflow_faces=[], source_fn=gaussian_source,
                    source_gauss=(1.0, 100.0, (0.0, 0.0)), eps_si=1e-6, max_outer=100, p=p,
                    q=q, eps_res=1e-7, eps_diff=1e-7, eps_svd=1e-8, eps_mgs=1e-10, m_max=4,
                    seed=seed)


def variable_scattering(n=80, n_theta=40, n_z=20, seed=66, p=1, q=8):
    """Sec. 4.3: smooth transition from sigma_s = 0.1 at the centre to 100 outside r = 1."""
    x, y = _cell_centres(n)
    r2 = x * x + y * y
    sig = np.where(r2 <= 1.0, 99.9 * r2 * r2 * (r2 - 2.0) ** 2 + 0.1, 100.0)
    return _paper_example("variable_scattering", sig, n, n_theta, n_z, seed, p, q)


def pin_cell(n=80, n_theta=32, n_z=16, seed=77, p=1, q=8):
    """Sec. 4.4: sigma_s = 0.1 on the central square |x|, |y| <= 0.5, 100 elsewhere."""
    x, y = _cell_centres(n)
    sig = np.where((np.abs(x) <= 0.5) & (np.abs(y) <= 0.5), 0.1, 100.0)
    return _paper_example("pin_cell", sig, n, n_theta, n_z, seed, p, q)
