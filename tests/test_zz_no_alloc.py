"""rte_sweep_noalloc (static device workspace, no allocation) against rte_sweep: same
plan and kernels, so psi and phi must agree bit for bit; two calls in a row, the second
smaller, and a request beyond the workspace rejected on the host."""
import numpy as np
import pytest

import workloads as W
from tests.common import gpu_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(wl, sel, mixed):
    import paper_2603_25233_amd as R
    gp = gpu_problem(wl)
    dt = torch.float32 if mixed else torch.float64
    rng = np.random.default_rng(wl["nx"] * 7 + len(sel))
    src = torch.as_tensor(rng.uniform(0.0, 1.0, (wl["ny"], wl["nx"], 4)), device="cuda").to(dt)
    ref_psi, ref_phi = R.sweep(gp, sel, src, want_psi=True, want_phi=True, mixed=mixed)
    ref_only_phi = R.sweep(gp, sel, src, want_psi=False, want_phi=True, mixed=mixed)[1]
    psi = torch.full_like(ref_psi, float("nan"))
    phi = torch.full_like(ref_phi, float("nan"))
    R.sweep_noalloc(gp, sel, src, psi=psi, phi=phi, mixed=mixed)
    phi2 = torch.full_like(ref_phi, float("nan"))
    R.sweep_noalloc(gp, sel, src, phi=phi2, mixed=mixed)
    torch.cuda.synchronize()
    assert torch.equal(psi, ref_psi)
    assert torch.equal(phi, ref_phi)
    assert torch.equal(phi2, ref_only_phi)


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "fp32"])
def test_noalloc_sweep_matches_rte_sweep_twice(mixed):
    # first call: 40 x 24 cells (ragged), 96 ordinates with inflow data; second: smaller
    wl = W.checkerboard(n=40, n_theta=16, n_z=6, blocks=4)
    wl = W.Workload(wl, ny=24, sigma_t=wl["sigma_t"][:24], sigma_s=wl["sigma_s"][:24])
    _case(wl, np.arange(96), mixed)
    wl2 = W.small_fr(n=12, n_theta=8, n_z=4)
    _case(wl2, np.array([5, 0, 17, 31, 5]), mixed)


def test_noalloc_sweep_rejects_oversized_workspace():
    import paper_2603_25233_amd as R
    n = 1024
    wl = W.small_fr(n=n, n_theta=8, n_z=4)
    gp = gpu_problem(wl)
    src = torch.zeros((n, n, 4), dtype=torch.float64, device="cuda")
    phi = torch.zeros((n, n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(R.RTEError, match="scratch"):
        R.sweep_noalloc(gp, np.arange(32), src, phi=phi)
