#!/usr/bin/env python3
"""Benchmark of the sweep-based (low-rank) SI-DSA hot path on one MI355X.

Metric: angle-cell-DOF sweep updates per second (one update = one DG degree of
freedom of one cell for one swept direction), plus the low-rank SI-DSA time to
tolerance next to the full-rank SI-DSA on the same GPU.

Workload of the headline line: the large multiscale medium, 1024 x 1024 DG-Q1 cells
(4,194,304 DOF), CL(64,16) with 1024 ordinates, log-normal sigma_t (mean 100, log-std 1,
correlation 32 cells), scattering ratio 0.999, uniform Q = 1, vacuum boundaries
(workloads.multiscale), FP64.  One step:
  1. a full-angle transport sweep writing psi for all 1024 ordinates (34.4 GB FP64);
  2. full-rank SI-DSA to eps_si = 1e-6 (one sweep per (Omega_x, Omega_y) class per outer
     iteration, DSA conjugate gradients to 1e-12).
value = all sweep updates of the timed steps / their wall time (inputs resident in HBM).
After the timed region, once each: the low-rank SI-DSA (p = 1, q = 8) in FP64 and the
mixed form, the full-rank solve in the mixed form, the 256 x 256 checkerboard (p = 4,
q = 32) as a secondary workload, and the oracle on the host (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--only step|sweep|sweep_large|paper|copy]
                    [--no-lr] [--no-secondary] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector (256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz)
# FP64 flops of one cell solve of the sweep (the closed-form 4x4 solve: right-hand side,
# determinant, refined reciprocal, two block products, outflow traces) and its weighted
# contribution to the scalar flux, plus the fixed-order reduction of the group partial
# sums: 93 + 4 per cell and swept direction (FMA = 2).
SWEEP_FLOPS_PER_CELL_DIR = 97


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_2603_25233_amd", "csrc", "sweep.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(profile="sweep_multiscale1024_pmc.md"):
    """HBM bytes per launch of a sweep from a committed rocprofv3 --pmc summary, or None
    when it is missing or taken on a different sweep kernel source."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = re.search(r"sweep\.hip sha256\[:16\]:\s*([0-9a-f]+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not h or not t or h.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def large_sweep(args, R, W, torch, dev):
    """The psi-writing full-angle sweep on the 1024x1024, CL(64,16) multiscale medium:
    1024 ordinates, 2047 anti-diagonal steps, FP64 psi of 34.4 GB (written once)."""
    wl = W.multiscale()
    dirs, wts = R.cl_quadrature(wl["n_theta"], wl["n_z"])
    prob = R.Problem(wl["nx"], wl["ny"], wl["domain"], dirs, wts, wl["sigma_t"], wl["sigma_s"])
    ncell, ndirs = wl["nx"] * wl["ny"], len(wts)
    dt = torch.float32 if args.mixed else torch.float64
    wsize = 4 if args.mixed else 8
    src = torch.ones((wl["ny"], wl["nx"], 4), dtype=dt, device=dev)  # uniform Q = 1
    psi = torch.empty((ndirs, wl["ny"], wl["nx"], 4), dtype=dt, device=dev)
    plan = R.SweepPlan(prob, np.arange(ndirs), mixed=args.mixed)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.execute(src, psi=psi)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        plan.execute(src, psi=psi)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    alg = ncell * (4 * wsize * ndirs + 4 * wsize + 8)
    updates = 4 * ncell * ndirs
    print(json.dumps({"metric": "angle-cell-DOF sweep updates/s (psi sweep only)",
                      "value": updates / (ms * 1e-3), "unit": "angle-cell-DOF updates/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                      "dtype": "f32" if args.mixed else "f64", "data": "synthetic",
                      "config": {"workload": "multiscale 1024x1024 DG-Q1, CL(64,16) 1024 ordinates, "
                                             "log-normal sigma_t, c=0.999, psi sweep only"},
                      "roofline": {"bound": "hbm", "achieved": alg / (ms * 1e-3) / 1e9,
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                   "algorithmic_bytes_per_launch": alg}}))


def effective_rank(s, eps):
    """Smallest l with sum_{i > l} s_i <= eps sum_i s_i (the truncation rule of the solver)."""
    tail = np.concatenate([np.cumsum(s[::-1])[::-1][1:], [0.0]])
    return int(np.argmax(tail <= eps * s.sum())) + 1


def paper_examples(R, W, torch, dev):
    """Full-rank and low-rank SI-DSA (FP64) on the paper's own media: Sec. 4.1 (homogeneous,
    L = 2..5, sigma_s in {0.1, 1, 10, 100}), Sec. 4.3 (variable scattering) and Sec. 4.4
    (pin cell); p = 1, q = 8, eps_SI = 1e-6.  Per case one JSON line: iterations, ranks,
    ||phi_LR - phi_FR||_2, compression ratio, times, and the effective rank of the
    full-rank angular flux (its truncated SVD with the solver's rule and eps_SVD = 1e-8)."""
    cases = [("sec4.1 homogeneous sigma_s=%g L=%d" % (sg, L), W.homogeneous(sg, L))
             for L in (2, 3, 4, 5) for sg in (0.1, 1.0, 10.0, 100.0)]
    cases += [("sec4.3 variable scattering", W.variable_scattering()),
              # fully greedy selection: every unsampled ordinate class a candidate (400
              # classes of CL(40,20), Omega_z twins folded)
              ("sec4.3 variable scattering, fully greedy", W.variable_scattering(q=400)),
              ("sec4.4 pin cell", W.pin_cell())]
    for name, wl in cases:
        d, w = R.cl_quadrature(wl["n_theta"], wl["n_z"])
        amp, alpha, centre = wl["source_gauss"]
        G = R.gaussian_source_moments(wl["nx"], wl["ny"], wl["domain"], amp, alpha, centre)
        prob = R.Problem(wl["nx"], wl["ny"], wl["domain"], d, w, wl["sigma_t"], wl["sigma_s"], G=G)
        kw = dict(eps_si=wl["eps_si"], max_outer=wl["max_outer"], eps_dsa=1e-12)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fr = R.solve(prob, full_rank=1, **kw)
        torch.cuda.synchronize()
        t_fr = time.perf_counter() - t0
        t0 = time.perf_counter()
        lr = R.solve(prob, rand=W.random_stream(wl["seed"]), full_rank=0, p=wl["p"], q=wl["q"],
                     eps_res=wl["eps_res"], eps_diff=wl["eps_diff"], eps_svd=wl["eps_svd"],
                     eps_mgs=wl["eps_mgs"], m_max=wl["m_max"], trunc_every_outer=False, **kw)
        torch.cuda.synchronize()
        t_lr = time.perf_counter() - t0
        # full-rank angular flux: one sweep of the converged source
        src = (prob.sigma_s[..., None] * fr["phi"] + prob.G).contiguous()
        psi, _ = R.sweep(prob, np.arange(len(w)), src)
        s = np.linalg.svd(psi.reshape(len(w), -1).cpu().numpy().T, compute_uv=False)
        nd = prob.ndof
        diff = (lr["phi"] - fr["phi"]).double().cpu().numpy().reshape(-1)
        print(json.dumps({"example": name, "cells": "%dx%d" % (wl["nx"], wl["ny"]),
                          "ordinates": len(w), "p": wl["p"], "q": wl["q"],
                          "fr_iters": fr["iters"], "lr_iters": lr["iters"], "lr_rank": lr["rank"],
                          "fr_effective_rank": effective_rank(s, wl["eps_svd"]),
                          "phi_lr_minus_fr_l2": float(np.linalg.norm(diff)),
                          "phi_lr_minus_fr_rel_l2": float(np.linalg.norm(diff) / np.linalg.norm(
                              fr["phi"].double().cpu().numpy())),
                          "compression_ratio": lr["rank"] * (nd + len(w) + 1) / (nd * len(w)),
                          "lr_angles_swept": int(sum(lr["swept"])),
                          "fr_time_s": t_fr, "lr_time_s": t_lr, "data": "synthetic",
                          "dtype": "f64"}), flush=True)



def lr_against_fr(R, W, torch, prob, wl, fr, seed, p, q, eps_res, eps_diff, eps_svd, eps_si,
                  max_outer, t_fr):
    """One FP64 low-rank solve against a converged full-rank one: the metrics of the paper's
    tables (rank, ||phi_LR - phi_FR||_2, C-R, iterations, speedup = full-rank time / low-rank
    time, largest oversampling ratio).  The tables' psi column is not reproduced: the factors
    hold the angular flux of the last SI step's source, and the full-rank solve does not keep
    the angular flux of its own last sweep to compare with."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lr = R.solve(prob, rand=W.random_stream(seed), full_rank=0, p=p, q=q, eps_res=eps_res,
                 eps_diff=eps_diff, eps_svd=eps_svd, eps_mgs=wl["eps_mgs"], m_max=wl["m_max"],
                 eps_si=eps_si, max_outer=max_outer, eps_dsa=1e-12)
    torch.cuda.synchronize()
    t_lr = time.perf_counter() - t0
    nd, nw = prob.ndof, prob.n_dirs
    dphi = float(torch.linalg.norm(lr["phi"].reshape(-1) - fr["phi"].reshape(-1)))
    over = [float(b) / float(a) - 1.0 for a, b in zip(lr["trunc_ranks"], lr["ranks"]) if a > 0]
    return dict(rank=lr["rank"], phi_lr_minus_fr_l2=dphi,
                compression_ratio=lr["rank"] * (nd + nw + 1) / (nd * nw), fr_iters=fr["iters"],
                lr_iters=lr["iters"], lr_converged=lr["converged"], speedup_fr_over_lr=t_fr / t_lr,
                lr_time_s=t_lr, max_oversampling=max(over) if over else None)


def paper_tables(R, W, torch):
    """The paper's robustness and threshold studies on its media (FP64): Sec. 4.3's p and q
    sweeps on the variable-scattering medium, Sec. 4.4's eight random seeds on the pin cell,
    and Sec. 4.2's inner-threshold scan (eps_res = eps_diff = 1e-3 .. 1e-7, eps_SVD = 0.1
    eps_res, eps_SI = 5e-5, at most 25 outer iterations) on the lattice stand-in.  One JSON
    line per run with the columns of the paper's tables."""
    def setup(wl):
        d, w = R.cl_quadrature(wl["n_theta"], wl["n_z"])
        if wl.get("source_gauss") is not None:
            amp, alpha, centre = wl["source_gauss"]
            G = R.gaussian_source_moments(wl["nx"], wl["ny"], wl["domain"], amp, alpha, centre)
        else:
            G = R.box_source_moments(wl["nx"], wl["ny"], wl["domain"], wl["source_boxes"])
        return R.Problem(wl["nx"], wl["ny"], wl["domain"], d, w, wl["sigma_t"], wl["sigma_s"], G=G)

    def reference(prob, eps_si, max_outer):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fr = R.solve(prob, full_rank=1, eps_si=eps_si, max_outer=max_outer, eps_dsa=1e-12)
        torch.cuda.synchronize()
        return fr, time.perf_counter() - t0

    wl = W.variable_scattering()
    prob = setup(wl)
    fr, t_fr = reference(prob, wl["eps_si"], wl["max_outer"])
    for p, q in ((1, 4), (1, 8), (1, 12), (1, 16), (2, 8), (3, 8)):
        m = lr_against_fr(R, W, torch, prob, wl, fr, wl["seed"], p, q, wl["eps_res"],
                          wl["eps_diff"], wl["eps_svd"], wl["eps_si"], wl["max_outer"], t_fr)
        print(json.dumps({"table": "sec4.3 variable scattering, p and q", "p": p, "q": q, **m,
                          "dtype": "f64", "data": "synthetic"}), flush=True)
    del prob
    wl = W.pin_cell()
    prob = setup(wl)
    fr, t_fr = reference(prob, wl["eps_si"], wl["max_outer"])
    runs = []
    for k in range(8):
        m = lr_against_fr(R, W, torch, prob, wl, fr, wl["seed"] + 1000 * (k + 1), wl["p"],
                          wl["q"], wl["eps_res"], wl["eps_diff"], wl["eps_svd"], wl["eps_si"],
                          wl["max_outer"], t_fr)
        runs.append(m)
        print(json.dumps({"table": "sec4.4 pin cell, random seeds", "run": k, **m, "dtype": "f64",
                          "data": "synthetic"}), flush=True)
    stats = {}
    for key in ("rank", "phi_lr_minus_fr_l2", "compression_ratio",
                "fr_iters", "lr_iters", "speedup_fr_over_lr"):
        v = np.array([r[key] for r in runs], dtype=np.float64)
        stats[key] = {"mean": float(v.mean()), "sd": float(v.std(ddof=1)), "min": float(v.min()),
                      "max": float(v.max())}
    print(json.dumps({"table": "sec4.4 pin cell, statistics of 8 seeds", **stats}), flush=True)
    del prob
    wl = W.lattice()
    prob = setup(wl)
    fr, t_fr = reference(prob, 5e-5, 25)
    for eps in (1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        m = lr_against_fr(R, W, torch, prob, wl, fr, wl["seed"], wl["p"], wl["q"], eps, eps,
                          0.1 * eps, 5e-5, 25, t_fr)
        print(json.dumps({"table": "sec4.2 lattice stand-in, inner thresholds", "eps_res": eps,
                          "eps_diff": eps, "eps_svd": 0.1 * eps, "eps_si": 5e-5, **m,
                          "dtype": "f64", "data": "synthetic"}), flush=True)


def basis_update_ablation(R, W, torch):
    """Sec. 4.2's comparison of basis updates (MGS2-A, MGS-QR, full QR) and the DEIM
    sampling of the Remark in Sec. 3.2 on the lattice stand-in (80 x 80, CL(32,16), p = 1,
    q = 8), FP64, next to the full-rank solve: one JSON line per variant with time, angles
    swept, rank, iterations, full-QR count and the flux difference to full rank."""
    wl = W.lattice()
    prob = make_problem(R, wl)
    kw = dict(eps_si=wl["eps_si"], max_outer=wl["max_outer"], eps_dsa=1e-12)
    fr = R.solve(prob, full_rank=1, **kw)
    nd, ndirs = prob.ndof, prob.n_dirs
    runs = [("mgs2a", "greedy"), ("mgs_qr", "greedy"), ("full_qr", "greedy"), ("mgs2a", "deim")]
    for variant, sampling in runs:
        lr = R.solve(prob, rand=W.random_stream(wl["seed"]), full_rank=0, p=wl["p"], q=wl["q"],
                     eps_res=wl["eps_res"], eps_diff=wl["eps_diff"], eps_svd=wl["eps_svd"],
                     eps_mgs=wl["eps_mgs"], m_max=wl["m_max"], basis_update=variant,
                     sampling=sampling, trunc_every_outer=False, **kw)
        diff = (lr["phi"] - fr["phi"]).double().cpu().numpy().reshape(-1)
        print(json.dumps({"ablation": "basis update (Sec. 4.2) and DEIM sampling (Remark in "
                                      "Sec. 3.2), lattice stand-in 80x80 CL(32,16)",
                          "variant": variant, "sampling": sampling,
                          "angles_swept": lr["n_swept"], "lr_time_s": lr["ms_total"] / 1e3,
                          "fr_time_s": fr["ms_total"] / 1e3,
                          "speedup_fr_over_lr": fr["ms_total"] / lr["ms_total"],
                          "rank": lr["rank"], "lr_iters": lr["iters"], "fr_iters": fr["iters"],
                          "full_qrs": lr["full_qrs"], "mgs_failures": lr["mgs_failures"],
                          "phi_lr_minus_fr_l2": float(np.linalg.norm(diff)),
                          "compression_ratio": lr["rank"] * (nd + ndirs + 1) / (nd * ndirs),
                          "dtype": "f64", "data": "synthetic"}), flush=True)


def tomography_run(R, W, torch, n_fd=8):
    """The adjoint workload at size: 256 x 256 cells, CL(32,8) (256 ordinates), log-normal
    sigma_a smoothed over 8 cells, sigma_s = 5, 16 boundary point sources (4 per side),
    exit currents on all 4 x 256 boundary faces; observations from a second seed's medium.
    Loss and gradient (forward and adjoint SI-DSA to 1e-12 per source) are timed; the
    gradient with respect to sigma_a is checked against FP64 central differences
    (h = 1e-6) on n_fd seeded random cells.  One JSON line."""
    wl, wtrue = W.tomography(), W.tomography(seed=45)
    n = wl["nx"]
    dirs, wts = R.cl_quadrature(wl["n_theta"], wl["n_z"])
    srcs = W.tomography_sources(n)
    bcs = np.stack([R.inflow_moments(n, n, wl["domain"], [(sd, i, 1.0)]) for sd, i in srcs])
    base = R.Problem(n, n, wl["domain"], dirs, wts, wl["sigma_t"], wl["sigma_s"])
    btrue = R.Problem(n, n, wl["domain"], dirs, wts, wtrue["sigma_t"], wtrue["sigma_s"])
    kw = dict(eps_si=1e-12, eps_dsa=1e-13)
    with torch.no_grad():
        _, J_obs = R.detector_misfit_batch(btrue.sigma_t - btrue.sigma_s, btrue.sigma_s, btrue, bcs,
                                           np.zeros((len(srcs), 4, n)), **kw)
    sa = (base.sigma_t - base.sigma_s).clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L, J = R.detector_misfit_batch(sa, base.sigma_s, base, bcs, J_obs, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = sa.grad.reshape(-1).cpu().numpy()
    cells = np.random.default_rng(64).choice(n * n, n_fd, replace=False)
    h = 1e-6
    fd = []
    with torch.no_grad():
        for c in cells:
            vals = []
            for sgn in (1.0, -1.0):
                s2 = (base.sigma_t - base.sigma_s).clone().reshape(-1)
                s2[c] += sgn * h
                vals.append(R.detector_misfit_batch(s2.reshape(n, n), base.sigma_s, base, bcs,
                                                    J_obs, **kw)[0].item())
            fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    err = np.abs(fd - g[cells])
    worst = int(np.argmax(err / np.abs(fd)))
    # The 1e-4 bar is on the error relative to the gradient's scale (its largest entry).
    # Per cell, a central difference of a loss L resolves a gradient entry only down to
    # its rounding floor (~eps |L| / h, a few 1e-16 here): the per-cell ratio is reported
    # with the size of the entry it was taken at.
    print(json.dumps({"workload": "tomography 256x256 DG-Q1, CL(32,8) 256 ordinates, 16 boundary "
                                  "point sources, 1024 boundary detectors, sigma_s = 5, log-normal "
                                  "sigma_a (smoothed over 8 cells)",
                      "loss": L.item(), "detectors": int(J.shape[0] * J.shape[1] * J.shape[2]),
                      "forward_s": t1 - t0, "adjoint_and_gradient_s": t2 - t1,
                      "fd_cells": int(n_fd), "fd_h": h,
                      "grad_vs_fd_max_abs": float(err.max()),
                      "fd_rounding_floor": float(np.finfo(np.float64).eps * abs(L.item()) / h),
                      "grad_vs_fd_rel_to_max_grad": float(err.max() / np.abs(g).max()),
                      "target_rel_to_max_grad": 1e-4,
                      "grad_vs_fd_max_rel_per_cell": float(err[worst] / abs(fd[worst])),
                      "grad_at_that_cell_rel_to_max_grad": float(abs(g[cells][worst]) / np.abs(g).max()),
                      "dtype": "f64", "data": "synthetic"}), flush=True)


def lowrank_run(R, W, torch):
    """One low-rank SI-DSA solve (FP64, p = 4, q = 32) on the 256 x 256 checkerboard, for
    profiling the basis kernels at ranks up to 256.  One JSON line."""
    wl = W.checkerboard()
    prob = make_problem(R, wl)
    lr = lr_solve(R, W, prob, wl)
    print(json.dumps({"workload": "checkerboard 256x256, CL(32,16), p = 4, q = 32, FP64 low rank",
                      "time_to_tol_s": lr["ms_total"] / 1e3, "outer_iters": lr["iters"],
                      "rank": lr["rank"], "basis_before_truncation": [int(x) for x in lr["ranks"]],
                      "angles_swept": lr["n_swept"],
                      "phases_ms": {"sweep": lr["ms_sweep"], "lowrank": lr["ms_lowrank"],
                                    "dsa": lr["ms_dsa"]}}), flush=True)


def timestep_run(R, W, torch, steps=3, dt=0.01):
    """Backward Euler time marching (Sec. 3.7) on the 256 x 256 checkerboard, CL(32,16):
    `steps` steps of size dt from psi = 0 with the box source on, full rank and low rank
    (p = 4, q = 32), each step's SI-DSA to 1e-6.  One JSON line per method with the time
    per step, outer iterations, ranks and the final flux difference between the two."""
    wl = W.checkerboard()
    prob = make_problem(R, wl)
    kw = dict(eps_si=wl["eps_si"], max_outer=wl["max_outer"], eps_dsa=1e-12)
    lr_kw = dict(p=wl["p"], q=wl["q"], eps_res=wl["eps_res"], eps_diff=wl["eps_diff"],
                 eps_svd=wl["eps_svd"], eps_mgs=wl["eps_mgs"], m_max=wl["m_max"],
                 trunc_every_outer=False)
    phis = {}
    for method in ("full_rank", "low_rank"):
        prev, times, iters, ranks = None, [], [], []
        for m in range(steps):
            if method == "full_rank":
                out = R.backward_euler_step(prob, dt, prev, full_rank=1, **kw)
            else:
                out = R.backward_euler_step(prob, dt, prev, full_rank=0,
                                            rand=W.random_stream(wl["seed"] + m), **kw, **lr_kw)
            prev = (out["X"], out["S"], out["V"])
            times.append(out["ms_total"] / 1e3)
            iters.append(out["iters"])
            ranks.append(out["rank"])
        phis[method] = out["phi"]
        line = {"workload": "backward Euler, checkerboard 256x256, CL(32,16), dt = %g, %d steps "
                            "from psi = 0" % (dt, steps),
                "method": method, "step_time_s": times, "outer_iters": iters, "rank": ranks,
                "dtype": "f64", "data": "synthetic"}
        if method == "low_rank":
            d = (phis["low_rank"] - phis["full_rank"]).cpu().numpy()
            line["phi_lr_minus_fr_rel_l2"] = float(np.linalg.norm(d) /
                                                   np.linalg.norm(phis["full_rank"].cpu().numpy()))
        print(json.dumps(line), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_baseline(wl):
    """The oracle (test infrastructure) on the host, on bounded samples:
    - one full-angle SI sweep (phi only) of the headline medium with its plain-C sweep,
      the work of one full-rank outer iteration without folding;
    - the oracle's full-rank and low-rank SI-DSA time to tolerance on the 32 x 32,
      CL(16,8) medium, median of 3 runs."""
    import statistics
    from oracle import dg, quadrature, sweep as osweep, si as osi, lowrank as olr
    import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    x0, x1, y0, y1 = wl["domain"]
    m = dg.Mesh(wl["nx"], wl["ny"], x0, x1, y0, y1)
    d, w = quadrature.cl_quadrature(wl["n_theta"], wl["n_z"])
    G = sum(dg.source_moments_box(m, v, b) for v, b in wl["source_boxes"]) \
        if m.ncell <= 65536 else None
    if G is None:   # uniform Q = 1 over the whole domain: the constant's only moment
        G = np.zeros((m.ncell, 4)); G[:, 0] = np.sqrt(m.hx * m.hy); G = G.reshape(-1)
    sel = np.arange(len(w))
    sig = wl["sigma_t"].reshape(-1)
    osweep.sweep(m, d, sel[:2], sig, G, None, want_psi=False, w=w[:2], nthreads=threads)
    t0 = time.perf_counter()
    osweep.sweep(m, d, sel, sig, G, None, want_psi=False, w=w, nthreads=threads)
    dt = time.perf_counter() - t0
    ups = len(w) * m.ncell * 4
    small = W.small_fr()
    ms = dg.Mesh(small["nx"], small["ny"], *small["domain"])
    ds, ws = quadrature.cl_quadrature(small["n_theta"], small["n_z"])
    Gs = sum(dg.source_moments_box(ms, v, b) for v, b in small["source_boxes"])
    op = osi.Problem(ms, ds, ws, small["sigma_t"].reshape(-1), small["sigma_s"].reshape(-1), Gs)
    fr_t, lr_t = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        fr = osi.fr_si_dsa(op, small["eps_si"], max_outer=small["max_outer"], nthreads=threads)
        fr_t.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        lr = olr.lr_si_dsa(op, small["eps_si"], p=1, q=8, eps_res=small["eps_res"],
                           eps_diff=small["eps_diff"], eps_svd=small["eps_svd"],
                           rand=W.random_stream(small["seed"]), max_outer=small["max_outer"],
                           nthreads=threads, keep_factors=False)
        lr_t.append(time.perf_counter() - t0)
    return {"value": ups / dt, "unit": "angle-cell-DOF updates/s", "cores": threads,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "one full-angle phi-only SI sweep of the %dx%d, CL(%d,%d) medium (%d "
                      "ordinates, %.1f s), plain-C oracle sweep on %d threads"
                      % (wl["nx"], wl["ny"], wl["n_theta"], wl["n_z"], len(w), dt, threads),
            "time_to_tol_s": {"workload": "32x32, CL(16,8), sigma_s/sigma_t = 0.99, eps_si = 1e-8 "
                                          "(low rank p = 1, q = 8)",
                              "fr": statistics.median(fr_t), "lr": statistics.median(lr_t),
                              "fr_outer_iters": fr["iters"], "lr_outer_iters": lr["iters"]},
            "skipped": "the oracle's full solves of the 256x256 and 1024x1024 media (hours of "
                       "host time; the low-rank one needs X of ~17 GB)"}


def lr_solve(R, W, prob, wl, mixed=False, trunc_every_outer=False):
    """Low-rank SI-DSA as timed: one truncation, after the last outer iteration (the
    paper's single truncation, Sec. 3.3); trunc_every_outer also truncates after every
    inner loop to report r' and the oversampling per outer iteration."""
    return R.solve(prob, rand=W.random_stream(wl["seed"]), full_rank=0, p=wl["p"], q=wl["q"],
                   eps_si=wl["eps_si"], eps_res=wl["eps_res"], eps_diff=wl["eps_diff"],
                   eps_svd=wl["eps_svd"], eps_mgs=wl["eps_mgs"], m_max=wl["m_max"],
                   max_outer=wl["max_outer"], eps_dsa=1e-12, mixed=mixed,
                   trunc_every_outer=trunc_every_outer)


def rel(a, b):
    return float((a.double() - b.double()).norm() / b.double().norm())


def solver_report(fr, lr, nd, ndirs, wsize, lr_trunc=None):
    """lr_trunc: an untimed run of the same low-rank solve that truncated after every
    outer iteration (r' and oversampling per outer iteration)."""
    tr = lr_trunc["trunc_ranks"] if lr_trunc is not None else [lr["rank"]]
    rk = lr_trunc["ranks"] if lr_trunc is not None else lr["ranks"][-1:]
    return {
        "fr_time_to_tol_s": fr["ms_total"] / 1e3, "lr_time_to_tol_s": lr["ms_total"] / 1e3,
        "lr_speedup_vs_fr": fr["ms_total"] / lr["ms_total"],
        "fr_outer_iters": fr["iters"], "lr_outer_iters": lr["iters"],
        "fr_converged": fr["converged"], "lr_converged": lr["converged"],
        "lr_rank": lr["rank"], "lr_basis_before_truncation": [int(x) for x in lr["ranks"]],
        "lr_rank_after_truncation": [int(x) for x in tr],
        "lr_oversampling": [float((a - b) / b) if b else None for a, b in zip(rk, tr)],
        "lr_truncation_reported": "every outer iteration (untimed second run)"
                                  if lr_trunc is not None else "last outer iteration",
        "lr_angles_swept": lr["n_swept"], "fr_class_sweeps": fr["n_swept"],
        "lr_phi_vs_fr_rel_l2": rel(lr["phi"], fr["phi"]),
        "fr_phases_ms": {"sweep": fr["ms_sweep"], "dsa": fr["ms_dsa"], "total": fr["ms_total"]},
        "lr_phases_ms": {"sweep": lr["ms_sweep"], "lowrank": lr["ms_lowrank"],
                         "dsa": lr["ms_dsa"], "total": lr["ms_total"]},
        "compression_ratio": lr["rank"] * (nd + ndirs + 1) / (nd * ndirs),
        "storage_bytes": {"lr_factors": lr["rank"] * (nd + ndirs + 1) * wsize,
                          "fr_psi": nd * ndirs * wsize},
    }


def make_problem(R, wl):
    dirs, wts = R.cl_quadrature(wl["n_theta"], wl["n_z"])
    G = R.box_source_moments(wl["nx"], wl["ny"], wl["domain"], wl["source_boxes"])
    return R.Problem(wl["nx"], wl["ny"], wl["domain"], dirs, wts, wl["sigma_t"], wl["sigma_s"], G=G)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--only", choices=["step", "sweep", "sweep_large", "paper", "ablation",
                                       "paper_tables", "tomography", "lowrank", "timestep",
                                       "copy"],
                    default="step",
                    help="step: the headline line (default); "
                         "sweep: only the psi-writing full-angle sweep of the headline medium; "
                         "sweep_large: the same, one JSON line of its own (--mixed: FP32); "
                         "paper: the paper's own examples (Sec. 4.1, 4.3, 4.4), one JSON line each; "
                         "paper_tables: the paper's p/q, random-seed and inner-threshold studies; "
                         "ablation: MGS2-A / MGS-QR / full-QR basis updates (Sec. 4.2) and DEIM sampling; "
                         "tomography: loss and sigma gradient of the 16-source detector misfit "
                         "at 256x256 with a central-difference check; "
                         "lowrank: one FP64 low-rank solve of the 256x256 checkerboard (profiling); "
                         "timestep: backward Euler steps (Sec. 3.7), full and low rank, 256x256; "
                         "copy: a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lr", action="store_true",
                    help="skip the untimed low-rank and mixed-precision solves (profiling runs)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 256x256 checkerboard secondary workload")
    ap.add_argument("--mixed", action="store_true", help="sweep_large in FP32")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (the method runs on one MI355X here); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_25233_amd as R
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only == "copy":
        n = 1 << 27  # 1 GiB of float64
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.warmup + args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                          "launches": args.warmup + args.steps}))
        return
    if args.only == "sweep_large":
        large_sweep(args, R, W, torch, dev)
        return
    if args.only == "paper":
        paper_examples(R, W, torch, dev)
        return
    if args.only == "paper_tables":
        paper_tables(R, W, torch)
        return
    if args.only == "ablation":
        basis_update_ablation(R, W, torch)
        return
    if args.only == "tomography":
        tomography_run(R, W, torch)
        return
    if args.only == "lowrank":
        lowrank_run(R, W, torch)
        return
    if args.only == "timestep":
        timestep_run(R, W, torch)
        return

    wl = W.multiscale()
    prob = make_problem(R, wl)
    nd, ncell, ndirs = prob.ndof, wl["nx"] * wl["ny"], prob.n_dirs
    wsize = 8
    # isotropic right-hand side of one SI step from a seeded positive scalar flux
    phi0 = torch.as_tensor(np.random.default_rng(7).uniform(0, 1e-2, (wl["ny"], wl["nx"], 4)), device=dev)
    src = (prob.sigma_s[..., None] * phi0 + prob.G).contiguous()
    del phi0
    psi = torch.empty((ndirs, wl["ny"], wl["nx"], 4), dtype=torch.float64, device=dev)
    plan = R.SweepPlan(prob, np.arange(ndirs))
    stream = torch.cuda.current_stream()
    fr_kw = dict(full_rank=1, eps_si=wl["eps_si"], max_outer=wl["max_outer"], eps_dsa=1e-12)

    def sweep_once():
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        # A short spin keeps the GPU busy while the host enqueues the sweep, so that the
        # events bracket its kernels and not the host's launch latency.
        torch.cuda._sleep(200000)
        e0.record(stream)
        plan.execute(src, psi=psi)
        e1.record(stream)
        return e0, e1

    def step():
        out = {"events": sweep_once()}
        if args.only == "step":
            out["fr"] = R.solve(prob, **fr_kw)
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    sweep_ms = [o["events"][0].elapsed_time(o["events"][1]) for o in outs]
    k1_updates = ndirs * ncell * 4
    updates = args.steps * k1_updates
    k1_ms = float(np.mean(sweep_ms))
    # algorithmic bytes of the psi-writing sweep: psi written once, source and sigma_t read once
    k1_bytes = ncell * (4 * wsize * ndirs + 4 * wsize + 8)
    achieved = k1_bytes / (k1_ms * 1e-3) / 1e9
    line = {
        "metric": "angle-cell-DOF sweep updates/s + low-rank SI-DSA time-to-tol vs full-rank, 1 GPU",
        "unit": "angle-cell-DOF updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "multiscale 1024x1024 DG-Q1, CL(64,16) 1024 ordinates, log-normal "
                               "sigma_t (mean 100, log-std 1, correlation 32 cells), c = 0.999, "
                               "Q = 1, vacuum; step = psi sweep + full-rank SI-DSA to 1e-6",
                   "only": args.only},
        "psi_sweep": {"updates_per_s": k1_updates / (k1_ms * 1e-3), "ms": k1_ms,
                      "algorithmic_bytes": k1_bytes, "achieved_GBs": achieved,
                      "hbm_frac": achieved / HBM_PEAK_GBS},
    }
    if args.only == "step":
        fr = outs[-1]["fr"]
        for o in outs:
            updates += o["fr"]["n_swept"] * ncell * 4
        fr_sweep_ms = float(np.mean([o["fr"]["ms_sweep"] / o["fr"]["iters"] for o in outs]))
        line["fr"] = {"time_to_tol_s": float(np.median([o["fr"]["ms_total"] for o in outs])) / 1e3,
                      "outer_iters": fr["iters"], "converged": fr["converged"],
                      "class_sweeps_per_outer": fr["n_swept"] // fr["iters"],
                      "dsa_cg_iters": fr["dsa_iters"],
                      "phases_ms": {"sweep": fr["ms_sweep"], "dsa": fr["ms_dsa"],
                                    "total": fr["ms_total"]},
                      "sweep_ms_per_outer": fr_sweep_ms}
    line["value"] = updates / wall
    psi_roof = {"kernel": "psi sweep (diag_layout_kernel + sweep_kernel), full angle set",
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                "algorithmic_bytes_per_launch": k1_bytes}
    if args.only == "step":
        # The step's dominant kernel is the full-rank SI sweep (the phi-only sweep of one
        # ordinate per class: source, anti-diagonal layout, sweep, fixed-order reduction of
        # the group partial sums), timed by the solver with HIP events on its stream.
        fr_flops = SWEEP_FLOPS_PER_CELL_DIR * ncell * line["fr"]["class_sweeps_per_outer"]
        fr_tf = fr_flops / (fr_sweep_ms * 1e-3) / 1e12
        line["roofline"] = {"kernel": "full-rank SI sweep, phi only (source_kernel, diag_layout_kernel, "
                                      "sweep_kernel, reduce_quadrants_kernel, gather_quadrants_kernel), 512 class sweeps",
                            "bound": "alu", "achieved": fr_tf, "peak": FP64_PEAK_TFLOPS,
                            "unit": "TFLOP/s", "frac": fr_tf / FP64_PEAK_TFLOPS,
                            "traffic": measured_traffic("fr_sweep_multiscale1024_pmc.md"),
                            "algorithmic_flops_per_launch": fr_flops, "ms_per_launch": fr_sweep_ms}
        line["roofline_psi_sweep"] = psi_roof
    else:
        line["roofline"] = psi_roof
    plan.close()
    del psi
    torch.cuda.empty_cache()
    if args.only == "step" and not args.no_lr:
        lr = lr_solve(R, W, prob, wl)
        line["lowrank"] = solver_report(fr, lr, nd, ndirs, wsize)
        print(json.dumps({"progress": "low-rank FP64 done", "s": lr["ms_total"] / 1e3}),
              file=sys.stderr, flush=True)
        frm = R.solve(prob, mixed=True, **fr_kw)
        lrm = lr_solve(R, W, prob, wl, mixed=True)
        line["mixed"] = {
            "fr_time_to_tol_s": frm["ms_total"] / 1e3, "lr_time_to_tol_s": lrm["ms_total"] / 1e3,
            "fr_outer_iters": frm["iters"], "lr_outer_iters": lrm["iters"], "lr_rank": lrm["rank"],
            "fr_phi_vs_fp64_fr_rel_l2": rel(frm["phi"], fr["phi"]),
            "lr_phi_vs_fp64_lr_rel_l2": rel(lrm["phi"], lr["phi"]),
            "lr_phi_vs_fp64_fr_rel_l2": rel(lrm["phi"], fr["phi"]),
            "target_rel_l2": 1e-5,
        }
        del lr, lrm, frm
    del prob
    torch.cuda.empty_cache()
    if args.only == "step" and not args.no_secondary:
        wl2 = W.checkerboard()
        p2 = make_problem(R, wl2)
        fr2 = R.solve(p2, full_rank=1, eps_si=wl2["eps_si"], max_outer=wl2["max_outer"], eps_dsa=1e-12)
        lr2 = lr_solve(R, W, p2, wl2)
        lr2t = lr_solve(R, W, p2, wl2, trunc_every_outer=True)
        line["secondary"] = dict(
            workload="checkerboard 256x256 DG-Q1, CL(32,16) 512 ordinates, 8x8 diffusive/absorbing "
                     "blocks, p = 4, q = 32, eps_si = 1e-6",
            **solver_report(fr2, lr2, p2.ndof, p2.n_dirs, 8, lr_trunc=lr2t))
        del p2
    if not args.no_cpu_baseline and args.only == "step":
        line["cpu_baseline"] = oracle_baseline(wl)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
