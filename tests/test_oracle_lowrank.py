"""Pins of the oracle's low-rank SI-DSA (Alg. 1, Alg. 2, Sec. 3.2-3.4) and metrics (Sec. 4)."""
import json
import os

import numpy as np
import pytest

from oracle import dg, lowrank, metrics, quadrature, si
from workloads import random_stream

HERE = os.path.dirname(os.path.abspath(__file__))


def problem(nx=8, ny=8, nt=8, nz=4, sig_t=2.0, c=0.9, hetero=True, seed=0):
    m = dg.Mesh(nx, ny)
    d, w = quadrature.cl_quadrature(nt, nz)
    rng = np.random.default_rng(seed)
    st = sig_t * (rng.uniform(0.5, 2.0, m.ncell) if hetero else np.ones(m.ncell))
    G = dg.source_moments_box(m, 1.0, (0.3, 0.55, 0.4, 0.7))
    return si.Problem(m, d, w, st, c * st, G)


def test_draw_partial_fisher_yates():
    s = lowrank.RandomStream(np.array([0, 0, 0], dtype=np.uint64))
    assert lowrank.draw(s, [5, 1, 9, 3], 3) == [1, 3, 5]          # u = 0 keeps the order
    top = np.iinfo(np.uint64).max
    s = lowrank.RandomStream(np.array([top, top], dtype=np.uint64))
    # i=0 swaps slots 0,3 -> [9,3,5,1]; i=1 swaps slots 1,3 -> [9,1,5,3]
    assert lowrank.draw(s, [1, 3, 5, 9], 2) == [9, 1]
    s = lowrank.RandomStream(random_stream(3, 1000))
    for _ in range(50):
        pool = sorted(set(np.random.default_rng(_).integers(0, 100, 30).tolist()))
        out = lowrank.draw(s, pool, 7)
        assert len(set(out)) == len(out) == min(7, len(pool)) and set(out) <= set(pool)


def test_order_key_breaks_rounding_level_ties():
    k = lowrank.order_key
    a = 0.1234567
    assert k(a) == k(a * (1 + 1e-15)) == k(a * (1 - 1e-15))     # rounding noise: tie
    assert k(a * (1 + 1e-8)) > k(a) > k(a * (1 - 1e-8))          # real differences order
    assert k(1.0) > k(0.9999999) and k(0.5) < k(0.5000001)
    assert k(0.0) < k(1e-300)
    m = 1.0 - 2.0 ** -40                                          # rounds up to the next binade
    assert k(m) == k(1.0)
    vals = np.random.default_rng(0).uniform(1e-8, 1.0, 2000)
    keys = [k(v) for v in sorted(vals)]
    assert keys == sorted(keys)


def test_truncation_rank():
    s = np.array([10.0, 1.0, 1e-3, 1e-9, 1e-12])
    tot = s.sum()
    assert lowrank.truncation_rank(s, 0.0) == 5
    assert lowrank.truncation_rank(s, 1e-8) == 3          # tail 1e-9 + 1e-12 <= 1e-8 * tot
    assert lowrank.truncation_rank(s, (1e-3 + 1e-9 + 1e-12) / tot) == 2
    assert lowrank.truncation_rank(s, 1.0) == 0


def test_low_rank_at_full_rank_equals_full_rank():
    """Every ordinate sampled (replay, eps_res = 0) => phi_LR^{n,*} = phi_FR^{n,*} each outer."""
    prob = problem()
    nd = prob.nd
    K = len(lowrank.direction_classes(prob.dirs)[1])
    assert K == nd // 2
    rep = [[list(range(i, min(i + 3, K))) for i in range(0, K, 3)]] * 60
    fr = si.fr_si_dsa(prob, 1e-9)
    lr = lowrank.lr_si_dsa(prob, 1e-9, p=3, q=4, eps_res=0.0, eps_diff=0.0, eps_svd=0.0,
                           rand=random_stream(1), replay=rep)
    assert fr["iters"] == lr["iters"]
    assert np.abs(np.array(fr["history"]) - np.array(lr["history"])).max() < 1e-13
    assert np.abs(fr["phi"] - lr["phi"]).max() < 1e-13
    assert all(r <= nd // 2 for r in lr["ranks"])        # twins are linearly dependent


def test_infinite_medium_has_rank_one():
    m = dg.Mesh(6, 6)
    d, w = quadrature.cl_quadrature(8, 4)
    st, ss, Q = 2.0, 1.0, 1.0
    G = np.zeros((m.ncell, 4)); G[:, 0] = Q * np.sqrt(m.hx * m.hy)
    bc = np.zeros((4, 6, 2)); bc[0:2, :, 0] = Q / (st - ss) * np.sqrt(m.hy); bc[2:4, :, 0] = Q / (st - ss) * np.sqrt(m.hx)
    prob = si.Problem(m, d, w, st * np.ones(m.ncell), ss * np.ones(m.ncell), G.reshape(-1), bc)
    lr = lowrank.lr_si_dsa(prob, 1e-10, p=1, q=8, eps_res=1e-11, eps_diff=1e-11, eps_svd=1e-8,
                           rand=random_stream(2))
    assert lr["converged"] and lr["ranks"][-1] == 1


def run_one_inner(prob, p=2, q=6, seed=4):
    ops = lowrank.operators(prob)
    solver = lowrank.LowRankSI(prob, ops, p, q, 1e-9, 1e-9)
    phi_prev = np.zeros(prob.mesh.ndof)
    src = prob.sig_s4 * phi_prev + prob.G
    solver.run(src, phi_prev, lowrank.RandomStream(random_stream(seed)))
    return solver, ops, src


def test_basis_orthonormal_and_R_reproduces_snapshots():
    prob = problem()
    s, ops, src = run_one_inner(prob)
    X = s.X
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-12
    from oracle import sweep
    for c, col in s.coef.items():
        psi, _ = sweep.sweep(prob.mesh, prob.dirs, [s.reps[c]], prob.sigma_t, src, prob.bnd)
        assert np.abs(X[:, :col.size] @ col - psi[0]).max() < 1e-12 * np.abs(psi).max()


def test_incremental_operators_equal_fresh_projection():
    prob = problem()
    s, ops, src = run_one_inner(prob)
    X = s.X
    for name, M in [("Sig_t", s.T), ("Dxm", s.Dxm), ("Dxp", s.Dxp), ("Dym", s.Dym), ("Dyp", s.Dyp)]:
        fresh = X.T @ (ops[name] @ X)
        assert np.abs(M - fresh).max() < 1e-12 * max(1.0, np.abs(fresh).max()), name
    assert np.abs(s.b_src - X.T @ src).max() < 1e-13
    assert np.abs(s.b_side - (X.T @ ops["gside"].T).T).max() < 1e-13


def test_galerkin_is_exact_for_twins():
    """Twins share (Omega_x, Omega_y): the twin of a sampled ordinate is in span(X), and
    the class map pairs exactly the twins of the CL rule."""
    prob = problem()
    s, ops, src = run_one_inner(prob)
    tw = quadrature.twin_index(8, 4)
    cls, reps = lowrank.direction_classes(prob.dirs)
    assert np.array_equal(cls, cls[tw]) and len(reps) == prob.nd // 2
    scale = np.linalg.norm(src)
    for c in list(s.coef):
        t = int(tw[s.reps[c]])
        assert s.residual_norm(t, s.galerkin(t)) < 1e-12 * scale


def test_svd_without_truncation_reproduces_XC():
    prob = problem()
    s, ops, src = run_one_inner(prob)
    Xn, S, V, _ = s.truncate(0.0)
    assert np.abs(Xn @ np.diag(S) @ V.T - s.X @ s.C).max() < 1e-12 * np.abs(s.X @ s.C).max()


def test_mgs2a_double_projection_keeps_orthogonality():
    """Nearly dependent snapshots: Alg. 2 keeps ||X^T X - I|| at rounding level."""
    prob = problem(nx=6, ny=6)
    ops = lowrank.operators(prob)
    sv = lowrank.LowRankSI(prob, ops, 1, 1, 0, 0)
    rng = np.random.default_rng(0)
    base = rng.normal(size=(prob.mesh.ndof, 5))
    sv.X = np.zeros((prob.mesh.ndof, 0)); sv.mgs_failures = 0; sv.breakdowns = 0
    for i in range(12):
        v = base @ rng.normal(size=5) + 1e-7 * rng.normal(size=prob.mesh.ndof)
        sv.mgs2a_append(v)
    X = sv.X
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-12


def test_lowrank_matches_full_rank_iterations():
    """Sec. 4 observation used as a soft pin: same outer count, phi difference << eps."""
    prob = problem(nx=12, ny=12, nt=16, nz=4, sig_t=5.0, c=0.99)
    fr = si.fr_si_dsa(prob, 1e-7)
    lr = lowrank.lr_si_dsa(prob, 1e-7, p=1, q=8, eps_res=1e-8, eps_diff=1e-8, eps_svd=1e-9,
                           rand=random_stream(5))
    assert fr["iters"] == lr["iters"]
    assert np.abs(fr["phi"] - lr["phi"]).max() < 1e-7


def test_compression_ratio_printed_values():
    rows = json.load(open(os.path.join(HERE, "golden", "compression_ratio.json")))["rows"]
    for row in rows:
        cr = metrics.compression_ratio(row["rank"], 4 * row["cells"], row["n_theta"] * row["n_z"])
        assert abs(100 * cr - row["cr_percent"]) < 0.006, row["cite"]


# ---------------------------------------------------------------------------
# Basis-update variants of Sec. 4.2 (MGS-QR, full QR).  Each spans the same space as
# MGS2-A, so on the same sampled classes (the MGS2-A run's decisions replayed) the
# Galerkin solutions and the scalar flux agree; the full-QR basis is orthonormal and
# reproduces every sampled snapshot through its R column.
# ---------------------------------------------------------------------------

def _replay_of(ref):
    return [[e["samples"] for e in outer] for outer in ref["logs"]]


@pytest.mark.parametrize("variant", ["mgs_qr", "full_qr"])
def test_basis_variants_match_mgs2a_on_same_samples(variant):
    prob = problem(nx=8, ny=8, nt=8, nz=4, c=0.95)
    kw = dict(p=2, q=5, eps_res=1e-9, eps_diff=1e-9, eps_svd=1e-10)
    ref = lowrank.lr_si_dsa(prob, 1e-9, rand=random_stream(4), **kw)
    got = lowrank.lr_si_dsa(prob, 1e-9, rand=random_stream(4), replay=_replay_of(ref),
                            basis_update=variant, **kw)
    assert got["iters"] == ref["iters"]
    assert np.linalg.norm(got["phi"] - ref["phi"]) < 1e-10 * np.linalg.norm(ref["phi"])
    for a, b in zip(got["history"], ref["history"]):
        assert abs(a - b) <= 1e-9 * b + 1e-15
    X = got["Xfull"]
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-12
    n_batches = sum(len(outer) for outer in ref["logs"])
    if variant == "full_qr":
        assert got["full_qrs"] == n_batches           # one full QR per inner iteration
    else:
        assert 0 <= got["full_qrs"] <= n_batches


def test_full_qr_reproduces_snapshots_and_counts():
    """With the greedy choice (no replay): R columns reproduce the sampled snapshots,
    the basis is orthonormal and nested spans give the same flux as MGS2-A."""
    prob = problem(nx=6, ny=6, nt=8, nz=4, c=0.9, seed=2)
    ops = lowrank.operators(prob)
    lr = lowrank.LowRankSI(prob, ops, 2, 4, 1e-10, 1e-10, basis_update="full_qr")
    src = prob.sig_s4 * np.zeros(prob.mesh.ndof) + prob.G
    lr.run(src, np.zeros(prob.mesh.ndof), lowrank.RandomStream(random_stream(8)))
    X = lr.X
    assert np.abs(X.T @ X - np.eye(X.shape[1])).max() < 1e-13
    for c, psi in lr.snaps:
        assert np.linalg.norm(X @ lr.coef[c] - psi) < 1e-12 * np.linalg.norm(psi)
    assert lr.full_qrs == len(lr.log)
    # the projected operators equal a fresh projection of the final basis
    assert np.abs(lr.T - X.T @ (ops["Sig_t"] @ X)).max() < 1e-12 * np.abs(lr.T).max()


def test_mgs_qr_takes_full_qrs_when_the_test_fails():
    """eps_mgs below any attainable orthogonality forces a full QR at every snapshot
    after the first; the flux is unchanged and every full QR is counted."""
    prob = problem(nx=8, ny=8, nt=8, nz=4, c=0.95)
    kw = dict(p=1, q=4, eps_res=1e-9, eps_diff=1e-9, eps_svd=1e-10)
    ref = lowrank.lr_si_dsa(prob, 1e-9, rand=random_stream(6), **kw)
    got = lowrank.lr_si_dsa(prob, 1e-9, rand=random_stream(6), replay=_replay_of(ref),
                            basis_update="mgs_qr", eps_mgs=1e-300, **kw)
    n_snap = sum(len(e["samples"]) for outer in ref["logs"] for e in outer)
    n_first = len(ref["logs"])                        # the first snapshot of each outer
    assert got["full_qrs"] >= n_snap - n_first - got["breakdowns"] - 2 * len(ref["logs"])
    assert got["full_qrs"] > 0
    assert np.linalg.norm(got["phi"] - ref["phi"]) < 1e-10 * np.linalg.norm(ref["phi"])


def test_deim_indices_small_example_by_hand():
    """v_1 = (1, 0, 2): largest entry in row 2.  v_2 = (0, 1, 1) interpolated at row 2 by
    0.5 v_1 leaves rho = (-0.5, 1, 0): row 1."""
    V = np.array([[1.0, 0.0], [0.0, 1.0], [2.0, 1.0]])
    assert lowrank.deim_indices(V) == [2, 1]
    # sign and scale of a column do not move the points
    assert lowrank.deim_indices(V * np.array([-3.0, 0.5])) == [2, 1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_deim_indices_are_the_row_pivots_of_partial_pivoting_lu(seed):
    """The DEIM residual of column l is column l of the Schur complement after l steps of
    Gaussian elimination, so the DEIM points are LAPACK's partial-pivoting row pivots."""
    import scipy.linalg as sla
    V = np.random.default_rng(seed).standard_normal((40, 12))
    P, _, _ = sla.lu(V)
    perm = np.argmax(P, axis=0)          # (P^T V)[i] = V[perm[i]]
    assert lowrank.deim_indices(V) == list(perm[:12])
    # the points interpolate: the DEIM projector reproduces every column of V
    idx = lowrank.deim_indices(V)
    proj = V @ np.linalg.solve(V[idx], V[idx])
    assert np.abs(proj - V).max() < 1e-12
    # early stop after the first 5 points
    assert lowrank.deim_indices(V, stop=lambda ix: len(ix) >= 5) == list(perm[:5])


def test_deim_sampling_converges_to_full_rank():
    """DEIM sampling (Remark in Sec. 3.2) reaches the full-rank fixed point within the
    inner thresholds, samples each class at most once per outer iteration, and takes a
    different sample sequence from the greedy random subsampling."""
    prob = problem(nx=8, ny=8, nt=8, nz=4)
    fr = si.fr_si_dsa(prob, 1e-10)
    kw = dict(p=2, q=4, eps_res=1e-10, eps_diff=1e-10, eps_svd=1e-11)
    de = lowrank.lr_si_dsa(prob, 1e-10, rand=random_stream(4), sampling="deim", **kw)
    gr = lowrank.lr_si_dsa(prob, 1e-10, rand=random_stream(4), **kw)
    assert de["converged"] and de["iters"] == fr["iters"]
    assert np.abs(de["phi"] - fr["phi"]).max() < 1e-8 * np.abs(fr["phi"]).max()
    for outer in de["logs"]:
        seq = [c for e in outer for c in e["samples"]]
        assert len(seq) == len(set(seq))
    assert [e["samples"] for e in de["logs"][0]] != [e["samples"] for e in gr["logs"][0]]
