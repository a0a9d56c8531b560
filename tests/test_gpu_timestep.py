"""Backward Euler steps (the implicit time marching of Sec. 3.7) through the C ABI
(rte_backward_euler_step) against the oracle's steps, two steps chained on each side:
each side feeds its own psi^{m+1} into its next step.

Bars: full rank, phi and psi within 1e-10 (rel-L2) and equal outer counts; low rank,
identical sample logs, equal outer counts and truncation ranks, phi within 1e-10 and the
factors X S V^T within 1e-9 (the FP64 bars of the steady solves).
"""
import numpy as np
import pytest

import workloads as W
from oracle import timestep as ots
from tests.common import gpu_problem, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def psi_of(out):
    """psi [N_Omega][ndof] from the factors the library returns."""
    X, S, V = (out[k].cpu().numpy() for k in ("X", "S", "V"))
    return (X.T @ np.diag(S) @ V).T


def wide(nx, ny, n_theta, n_z):
    wl = W.Workload(W.small_fr(n=nx, n_theta=n_theta, n_z=n_z))
    wl["ny"] = ny
    wl["sigma_t"] = np.ones((ny, nx)); wl["sigma_s"] = 0.99 * np.ones((ny, nx))
    return wl


# Every step after the first sweeps with one source per class: 16 classes use the small
# plans' direct stores, 64 classes the LDS output ring, and 800 rows with 64 classes the
# line-grouped stores of two rows per thread.
FR_STEP_CASES = [
    ("small12_cl8x4_dt0.05", W.Workload(W.small_fr(n=12, n_theta=8, n_z=4)), 0.05),
    ("small12_cl8x4_dt2", W.Workload(W.small_fr(n=12, n_theta=8, n_z=4)), 2.0),
    ("small12_cl16x8_ring", W.Workload(W.small_fr(n=12, n_theta=16, n_z=8)), 0.1),
    ("rows800_cl16x8_grouped", wide(3, 800, 16, 8), 0.1),
]


@pytest.mark.parametrize("name,wl,dt", FR_STEP_CASES, ids=[c[0] for c in FR_STEP_CASES])
def test_full_rank_steps(name, wl, dt):
    import paper_2603_25233_amd as R
    op, gp = oracle_problem(wl), gpu_problem(wl)
    kw = dict(full_rank=1, eps_si=1e-12, eps_dsa=1e-13, max_outer=200)
    o1 = ots.fr_step(op, dt, None, 1e-12)
    o2 = ots.fr_step(op, dt, o1["psi"], 1e-12)
    g1 = R.backward_euler_step(gp, dt, None, **kw)
    g2 = R.backward_euler_step(gp, dt, (g1["X"], g1["S"], g1["V"]), **kw)
    for o, g in ((o1, g1), (o2, g2)):
        assert g["converged"] and g["iters"] == o["iters"]
        assert rel_l2(g["phi"].cpu().numpy(), o["phi"]) < 1e-10
        assert rel_l2(psi_of(g), o["psi"]) < 1e-10
    # the step moved the solution: psi^2 differs from psi^1
    assert rel_l2(o2["psi"], o1["psi"]) > 1e-3


LR_STEP_CASES = [
    ("multiscale10_cl16x4", W.multiscale(n=10, n_theta=16, n_z=4, corr=3.0), 0.1, 2, 8),
    ("multiscale12_cl16x8", W.multiscale(n=12, n_theta=16, n_z=8, corr=4.0, seed=7), 0.02, 1, 8),
]


@pytest.mark.parametrize("name,wl,dt,p,q", LR_STEP_CASES, ids=[c[0] for c in LR_STEP_CASES])
def test_low_rank_steps(name, wl, dt, p, q):
    import paper_2603_25233_amd as R
    wl = W.Workload(wl)
    op, gp = oracle_problem(wl), gpu_problem(wl)
    th = dict(p=p, q=q, eps_res=1e-8, eps_diff=1e-8, eps_svd=1e-9)
    eps_si = 1e-7
    o1 = ots.lr_step(op, dt, None, eps_si, rand=W.random_stream(wl["seed"]), **th)
    o2 = ots.lr_step(op, dt, o1["psi"], eps_si, rand=W.random_stream(wl["seed"] + 1), **th)
    kw = dict(full_rank=0, eps_si=eps_si, eps_mgs=1e-10, eps_dsa=1e-13, **th)
    g1 = R.backward_euler_step(gp, dt, None, rand=W.random_stream(wl["seed"]), **kw)
    g2 = R.backward_euler_step(gp, dt, (g1["X"], g1["S"], g1["V"]),
                               rand=W.random_stream(wl["seed"] + 1), **kw)
    for o, g in ((o1, g1), (o2, g2)):
        olog = [c for outer in o["logs"] for e in outer for c in e["samples"]]
        assert list(g["sample_log"]) == olog
        assert g["iters"] == o["iters"]
        assert list(g["trunc_ranks"]) == list(o["ranks"])
        assert rel_l2(g["phi"].cpu().numpy(), o["phi"]) < 1e-10
        assert rel_l2(psi_of(g), o["psi"]) < 1e-9


def test_step_rejects_bad_arguments():
    import paper_2603_25233_amd as R
    wl = W.Workload(W.small_fr(n=6, n_theta=8, n_z=2))
    gp = gpu_problem(wl)
    kw = dict(full_rank=1, eps_si=1e-10)
    for dt in (0.0, -1.0, float("inf")):
        with pytest.raises(R.RTEError):
            R.backward_euler_step(gp, dt, None, **kw)
    with pytest.raises(R.RTEError):
        R.backward_euler_step(gp, 0.1, None, mixed=True, **kw)
    g = R.backward_euler_step(gp, 0.1, None, **kw)
    # twins of a class must carry the same psi
    V = g["V"].clone()
    V[0, 0] += 1.0
    twin = int(np.nonzero(V[0].cpu().numpy() > 0.5)[0][-1])
    assert twin != 0
    with pytest.raises(R.RTEError):
        R.backward_euler_step(gp, 0.1, (g["X"], g["S"], V), **kw)
    # the output must not overlap psi^m
    with pytest.raises(R.RTEError):
        Xall = torch.zeros((gp.n_dirs * 2, gp.ndof), dtype=torch.float64, device=gp.device)
        Xall[:g["X"].shape[0]] = g["X"]
        # X_prev and X the same memory: call the library directly
        import ctypes
        from paper_2603_25233_amd import rte
        call = rte._Call(gp, None, None, False, 16, dict(kw))
        S = torch.ones(gp.n_dirs, dtype=torch.float64, device=gp.device)
        Vo = torch.zeros((gp.n_dirs, gp.n_dirs), dtype=torch.float64, device=gp.device)
        phi = torch.empty((gp.ny, gp.nx, 4), dtype=torch.float64, device=gp.device)
        cp = gp.c()
        code = rte.lib().rte_backward_euler_step(
            ctypes.byref(cp), ctypes.byref(call.prm), 0.1, g["S"].numel(), rte._dptr(Xall),
            rte._dptr(g["S"].contiguous()), rte._dptr(g["V"].contiguous()), None, rte._dptr(phi),
            rte._dptr(Xall), rte._dptr(S), rte._dptr(Vo), ctypes.byref(call.res), rte._stream())
        rte._check(code)
