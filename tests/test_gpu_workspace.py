"""Workspace reuse between calls: buffers released by one call are kept by the library and
handed to later calls (on the same or another stream) after the call's stream has
finished with them.  Reused workspace must not change a result: repeated solves and sweeps
are bitwise equal, across problem sizes, streams and an emptied cache."""
import numpy as np
import pytest

import workloads as W
from tests.common import gpu_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_repeated_calls_reuse_workspace_bitwise():
    import paper_2603_25233_amd as R
    big = gpu_problem(W.Workload(W.checkerboard(n=64, n_theta=16, n_z=4)))
    small = gpu_problem(W.Workload(W.small_fr(n=12, n_theta=8, n_z=4)))
    kw = dict(full_rank=1, eps_si=1e-10, eps_dsa=1e-12, max_outer=200)
    ref = R.solve(big, **kw)["phi"].clone()
    ref_small = R.solve(small, **kw)["phi"].clone()
    for _ in range(2):
        assert torch.equal(R.solve(big, **kw)["phi"], ref)
        assert torch.equal(R.solve(small, **kw)["phi"], ref_small)
    # a sweep on a side stream after solves on the default stream
    src = (big.sigma_s[..., None] * ref + big.G).contiguous()
    d = np.arange(big.n_dirs)
    want = R.sweep(big, d, src, want_psi=False, want_phi=True)[1].clone()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        got = R.sweep(big, d, src, want_psi=False, want_phi=True)[1]
    side.synchronize()
    assert torch.equal(got, want)
    R.release_cached_memory()
    assert torch.equal(R.solve(big, **kw)["phi"], ref)
