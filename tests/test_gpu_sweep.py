"""GPU parity of rte_sweep / rte_adjoint_sweep against the oracle sweep (Sec. 2.2).

FP64: element-wise to 1e-13 relative to the field's max.  Mixed (FP32 sweep): 1e-5
relative, the precision target for the mixed path; the per-cell closed-form solve
loses at most ~2e-6 in FP32 over sigma, a, b in [1e-3, 1e4] (checked on the host),
and errors do not grow along the sweep for a contractive upwind transmission.
Grids span several 64-row waves with ragged tails; every quadrant, heterogeneous
cross sections, linear inflow data, both directions-per-workgroup paths, and both output
paths (the LDS write-back ring for plans of 64 or more ordinates, direct stores below).
"""
import numpy as np
import pytest

from oracle import dg, quadrature, sweep as osweep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def make(nx, ny, nt, nz, seed, domain=(0.0, 1.3, -0.4, 0.9)):
    import paper_2603_25233_amd as R
    rng = np.random.default_rng(seed)
    sig_t = np.exp(rng.uniform(np.log(0.05), np.log(2000.0), (ny, nx)))
    src = rng.normal(size=(ny, nx, 4))
    bc = rng.normal(size=(4, max(nx, ny), 2))
    d, w = R.cl_quadrature(nt, nz)
    prob = R.Problem(nx, ny, domain, d, w, sig_t, 0.5 * sig_t, G=None, bc=bc)
    m = dg.Mesh(nx, ny, *domain)
    do, wo = quadrature.cl_quadrature(nt, nz)
    return prob, m, do, wo, sig_t, src, bc


def oracle_sweep(m, do, sig_t, src, bc, sel, transpose=False, w=None):
    bnd = dg.boundary_unit_vectors(m, bc)
    return osweep.sweep(m, do, sel, sig_t.reshape(-1), src.reshape(-1), bnd,
                        want_psi=True, w=w, transpose=transpose)


# (13, 300, 16, 4): 64 ordinates over 300 rows, the write-back ring with five write-back
# wavefronts and a short end chunk in every row (13 columns); (7, 400, 16, 4): the
# thread budget leaves fewer write-back wavefronts than 64-row blocks (two blocks each;
# with FP32 the last two wavefronts' rows are all past the grid), rows shorter than one
# FP32 chunk
# (6, 1000, 16, 8): two rows per compute thread with 128 ordinates: the output ring does
# not fit, every cell leaves through the paired direct stores (aligned 64-byte pairs of
# a row's consecutive cells; with nx = 6 every row starts on a pair boundary, with
# nx = 7 below every other row starts on the second cell of a pair)
# (3, 800, 32, 16): 512 ordinates over two rows per thread: two FP64 directions per
# workgroup, psi in aligned pairs of cells per row and direction
CASES = [(37, 70, 8, 4), (64, 64, 16, 8), (5, 129, 8, 2), (130, 3, 4, 2), (1, 1, 4, 2),
         (13, 300, 16, 4), (7, 400, 16, 4), (6, 1000, 16, 8), (7, 777, 16, 4), (3, 800, 32, 16)]


@pytest.mark.parametrize("nx,ny,nt,nz", CASES)
def test_sweep_fp64_matches_oracle(nx, ny, nt, nz):
    import paper_2603_25233_amd as R
    prob, m, do, wo, sig_t, src, bc = make(nx, ny, nt, nz, seed=nx * 1000 + ny)
    sel = np.arange(len(wo))[::-1].copy()          # reversed order: slots != ordinate ids
    psi, _ = R.sweep(prob, sel, torch.as_tensor(src, device="cuda"))
    ref, _ = oracle_sweep(m, do, sig_t, src, bc, sel)
    got = psi.cpu().numpy().reshape(len(sel), -1)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert (np.abs(got - ref) / scale).max() < 1e-13


@pytest.mark.parametrize("nx,ny,nt,nz", CASES[:3])
def test_adjoint_sweep_fp64_matches_oracle(nx, ny, nt, nz):
    import paper_2603_25233_amd as R
    prob, m, do, wo, sig_t, src, bc = make(nx, ny, nt, nz, seed=7 + nx)
    sel = np.arange(len(wo))
    mu, _ = R.adjoint_sweep(prob, sel, torch.as_tensor(src, device="cuda"))
    ref, _ = oracle_sweep(m, do, sig_t, src, bc, sel, transpose=True)
    got = mu.cpu().numpy().reshape(len(sel), -1)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert (np.abs(got - ref) / scale).max() < 1e-13


@pytest.mark.parametrize("nx,ny,nt,nz", [(20, 30, 32, 16), (9, 40, 64, 32), (33, 17, 8, 4),
                                         (13, 300, 16, 4), (7, 400, 16, 4), (5, 1024, 16, 8),
                                         (3, 800, 32, 16)])
def test_scalar_flux_accumulation(nx, ny, nt, nz):
    """phi = sum_j w_j psi_j through the partial-sum path (1, 2 and 4 directions per group;
    (3, 800, 32, 16): 512 ordinates over two rows per thread, two FP64 directions per
    workgroup with two input slots)."""
    import paper_2603_25233_amd as R
    prob, m, do, wo, sig_t, src, bc = make(nx, ny, nt, nz, seed=3)
    sel = np.arange(len(wo))
    _, phi = R.sweep(prob, sel, torch.as_tensor(src, device="cuda"), want_psi=False, want_phi=True)
    _, ref = oracle_sweep(m, do, sig_t, src, bc, sel, w=wo)
    got = phi.cpu().numpy().reshape(-1)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("nx,ny,nt,nz", [(37, 70, 8, 4), (64, 64, 16, 8), (9, 40, 64, 32),
                                         (13, 300, 16, 4), (7, 400, 16, 4)])
def test_sweep_fp32_within_mixed_tolerance(nx, ny, nt, nz):
    import paper_2603_25233_amd as R
    prob, m, do, wo, sig_t, src, bc = make(nx, ny, nt, nz, seed=11)
    sel = np.arange(len(wo))
    psi, phi = R.sweep(prob, sel, torch.as_tensor(src, device="cuda"), want_phi=True, mixed=True)
    assert psi.dtype == torch.float32
    ref, refphi = oracle_sweep(m, do, sig_t, src, bc, sel, w=wo)
    got = psi.cpu().double().numpy().reshape(len(sel), -1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5
    assert np.linalg.norm(phi.cpu().double().numpy().reshape(-1) - refphi) / np.linalg.norm(refphi) < 1e-5


def test_max_rows_and_repeatability():
    """ny = 1024 (one thread per row, 16 waves); two runs are bitwise identical."""
    import paper_2603_25233_amd as R
    prob, m, do, wo, sig_t, src, bc = make(3, 1024, 4, 2, seed=5)
    sel = np.arange(len(wo))
    s = torch.as_tensor(src, device="cuda")
    a, pa = R.sweep(prob, sel, s, want_phi=True)
    b, pb = R.sweep(prob, sel, s, want_phi=True)
    assert torch.equal(a, b) and torch.equal(pa, pb)
    ref, _ = oracle_sweep(m, do, sig_t, src, bc, sel)
    got = a.cpu().numpy().reshape(len(sel), -1)
    assert (np.abs(got - ref) / np.abs(ref).max(axis=1, keepdims=True)).max() < 1e-13


def test_rejects_bad_input():
    import paper_2603_25233_amd as R
    prob, m, do, wo, sig_t, src, bc = make(4, 4, 4, 2, seed=1)
    with pytest.raises(R.RTEError):
        R.sweep(prob, [0, 99], torch.as_tensor(src, device="cuda"))
    big = R.Problem(2, 1025, (0, 1, 0, 1), do, wo, np.ones((1025, 2)), np.zeros((1025, 2)))
    with pytest.raises(R.RTEError):
        R.sweep(big, [0], torch.zeros((1025, 2, 4), dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("mixed", [False, True])
def test_plan_matches_one_shot(mixed):
    """A plan made with the scalar-flux workspace: psi-writing and phi-only executions
    match the one-shot entry point bit for bit, repeated executions included."""
    import paper_2603_25233_amd as R
    prob, m, do, wo, sig_t, src, bc = make(23, 41, 32, 16, seed=13)
    sel = np.arange(len(wo))
    dt = torch.float32 if mixed else torch.float64
    s = torch.as_tensor(src, device="cuda").to(dt).contiguous()
    psi_ref, _ = R.sweep(prob, sel, s, mixed=mixed)
    _, phi_ref = R.sweep(prob, sel, s, want_psi=False, want_phi=True, mixed=mixed)
    plan = R.SweepPlan(prob, sel, mixed=mixed, want_phi=True)
    psi = torch.empty_like(psi_ref)
    phi = torch.empty_like(phi_ref)
    for _ in range(2):
        plan.execute(s, psi=psi)
        plan.execute(s, phi=phi)
        torch.cuda.synchronize()
        assert torch.equal(psi, psi_ref)
        assert torch.equal(phi, phi_ref)
    plan.close()
