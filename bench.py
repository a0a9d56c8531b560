#!/usr/bin/env python3
"""Benchmark of the sweep-based (low-rank) SI-DSA hot path on one MI355X.

Metric: angle-cell-DOF sweep updates per second (one update = one DG degree of
freedom of one cell for one swept direction), plus the low-rank SI-DSA time to
tolerance next to the full-rank SI-DSA on the same GPU.

One step = one pass of the whole hot path over the 256x256-cell checkerboard
workload (CL(32,16), 512 ordinates, FP64; see workloads.checkerboard):
  1. a full-angle transport sweep writing psi for all 512 ordinates (rte_sweep plan);
  2. full-rank SI-DSA to eps_si = 1e-6;
  3. low-rank SI-DSA (p = 4, q = 32, eps_res = eps_diff = 1e-7, eps_svd = 1e-8).
value = all sweep updates of the step / step wall time (inputs resident in HBM).

    python bench.py [--steps K] [--warmup W] [--only sweep|step] [--no-cpu-baseline]
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


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_2603_25233_amd", "csrc", "sweep.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the psi-writing sweep from the committed rocprofv3 --pmc
    summary, or None when it is missing or taken on a different sweep kernel source."""
    path = os.path.join(ROOT, "profiles", "sweep_checkerboard_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = re.search(r"sweep\.hip sha256\[:16\]:\s*([0-9a-f]+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not h or not t or h.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def cpu_baseline(wl, n_sweeps):
    """The oracle's plain-C sweep (test infrastructure) on a bounded sample of the same
    workload: n_sweeps full-angle FP64 sweeps writing psi."""
    from oracle import dg, quadrature, sweep as osweep
    x0, x1, y0, y1 = wl["domain"]
    m = dg.Mesh(wl["nx"], wl["ny"], x0, x1, y0, y1)
    d, w = quadrature.cl_quadrature(wl["n_theta"], wl["n_z"])
    G = sum(dg.source_moments_box(m, v, b) for v, b in wl["source_boxes"])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sel = np.arange(len(w))
    osweep.sweep(m, d, sel[:4], wl["sigma_t"].reshape(-1), G, None, want_psi=True, nthreads=threads)
    t0 = time.perf_counter()
    for _ in range(n_sweeps):
        osweep.sweep(m, d, sel, wl["sigma_t"].reshape(-1), G, None, want_psi=True, nthreads=threads)
    dt = time.perf_counter() - t0
    ups = n_sweeps * len(w) * m.ncell * 4
    return {"value": ups / dt, "unit": "angle-cell-DOF updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d full-angle FP64 sweeps writing psi (%d ordinates, %dx%d cells), "
                      "plain-C oracle sweep, %.1f s" % (n_sweeps, len(w), wl["nx"], wl["ny"], dt)}


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
                     eps_mgs=wl["eps_mgs"], m_max=wl["m_max"], **kw)
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--only", choices=["step", "sweep", "sweep_large", "paper", "copy"], default="step",
                    help="sweep: only the psi-writing full-angle sweep (profiling); "
                         "sweep_large: the same on the 1024x1024, CL(64,16) multiscale medium "
                         "(34.4 GB of FP64 psi), one JSON line of its own; "
                         "paper: the paper's own examples (Sec. 4.1, 4.3, 4.4), one JSON line each; "
                         "copy: a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=10)
    ap.add_argument("--mixed", action="store_true", help="mixed-precision solvers and sweep")
    ap.add_argument("--no-mixed-report", action="store_true",
                    help="skip the untimed mixed-precision solves reported next to the FP64 ones")
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

    wl = W.checkerboard()
    dirs, wts = R.cl_quadrature(wl["n_theta"], wl["n_z"])
    G = R.box_source_moments(wl["nx"], wl["ny"], wl["domain"], wl["source_boxes"])
    prob = R.Problem(wl["nx"], wl["ny"], wl["domain"], dirs, wts, wl["sigma_t"], wl["sigma_s"], G=G)
    nd, ncell, ndirs = prob.ndof, wl["nx"] * wl["ny"], len(wts)
    dt = torch.float32 if args.mixed else torch.float64
    wsize = 4 if args.mixed else 8
    # isotropic right-hand side of one SI step from a seeded positive scalar flux
    phi0 = torch.as_tensor(np.random.default_rng(7).uniform(0, 1e-3, (wl["ny"], wl["nx"], 4)), device=dev)
    src = (prob.sigma_s[..., None] * phi0 + prob.G).to(dt).contiguous()
    psi = torch.empty((ndirs, wl["ny"], wl["nx"], 4), dtype=dt, device=dev)
    plan = R.SweepPlan(prob, np.arange(ndirs), mixed=args.mixed)
    rand = W.random_stream(wl["seed"])
    stream = torch.cuda.current_stream()
    solve_kw = dict(eps_si=wl["eps_si"], max_outer=wl["max_outer"], eps_dsa=1e-12, mixed=args.mixed)

    def sweep_once():
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        # A short spin keeps the GPU busy while the host enqueues the sweep, so that the
        # events bracket its kernels and not the host's launch latency (after a solver run
        # the GPU is idle when the step starts).
        torch.cuda._sleep(200000)
        e0.record(stream)
        plan.execute(src, psi=psi)
        e1.record(stream)
        return e0, e1

    def step():
        out = {}
        e0, e1 = sweep_once()
        if args.only == "step":
            fr = R.solve(prob, full_rank=1, **solve_kw)
            lr = R.solve(prob, rand=rand, full_rank=0, p=wl["p"], q=wl["q"], eps_res=wl["eps_res"],
                         eps_diff=wl["eps_diff"], eps_svd=wl["eps_svd"], eps_mgs=wl["eps_mgs"],
                         m_max=wl["m_max"], **solve_kw)
            out.update(fr=fr, lr=lr)
        out["events"] = (e0, e1)
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
    res = {}
    if args.only == "step":
        fr_ms = [o["fr"]["ms_total"] for o in outs]
        lr_ms = [o["lr"]["ms_total"] for o in outs]
        fr, lr = outs[-1]["fr"], outs[-1]["lr"]
        for o in outs:
            updates += o["fr"]["iters"] * ndirs * ncell * 4 + o["lr"]["n_swept"] * ncell * 4
        diff = (lr["phi"] - fr["phi"]).double()
        res = {
            "fr_time_to_tol_s": float(np.median(fr_ms)) / 1e3,
            "lr_time_to_tol_s": float(np.median(lr_ms)) / 1e3,
            "lr_speedup_vs_fr": float(np.median(fr_ms) / np.median(lr_ms)),
            "fr_outer_iters": fr["iters"], "lr_outer_iters": lr["iters"],
            "lr_rank": lr["rank"], "lr_angles_swept": lr["n_swept"],
            "lr_phi_vs_fr_rel_l2": float(diff.norm() / fr["phi"].double().norm()),
            "fr_phases_ms": {"sweep": fr["ms_sweep"], "dsa": fr["ms_dsa"], "total": fr["ms_total"]},
            "lr_phases_ms": {"sweep": lr["ms_sweep"], "lowrank": lr["ms_lowrank"],
                             "dsa": lr["ms_dsa"], "total": lr["ms_total"]},
            "compression_ratio": lr["rank"] * (nd + ndirs + 1) / (nd * ndirs),
            "storage_bytes": {"lr_factors": lr["rank"] * (nd + ndirs + 1) * wsize,
                              "fr_psi": nd * ndirs * wsize},
        }
    k1_ms = float(np.mean(sweep_ms))
    # algorithmic bytes of the psi-writing sweep: psi written once, source and sigma_t read once
    k1_bytes = ncell * (4 * wsize * ndirs + 4 * wsize + 8)
    achieved = k1_bytes / (k1_ms * 1e-3) / 1e9
    traffic = measured_traffic() if not args.mixed else None
    line = {
        "metric": "angle-cell-DOF sweep updates/s + low-rank SI-DSA time-to-tol vs full-rank, 1 GPU",
        "value": updates / wall,
        "unit": "angle-cell-DOF updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.mixed else "f64", "data": "synthetic",
        "config": {"workload": "checkerboard 256x256 DG-Q1, CL(32,16) 512 ordinates, "
                               "8x8 diffusive/absorbing blocks, p=4 q=32, eps_si=1e-6",
                   "only": args.only},
        "sweep_kernel": {"updates_per_s": k1_updates / (k1_ms * 1e-3), "ms": k1_ms,
                         "launch": "diag_layout_kernel, then sweep_kernel: 1 ordinate per "
                                   "workgroup (512 workgroups, 2 per CU), 256 compute threads "
                                   "(one per row) + 2 staging wavefronts of 128 rows + 4 write-back wavefronts of 64 rows"},
        "roofline": {"kernel": "psi sweep (diag_layout_kernel + sweep_kernel), full angle set",
                     "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": k1_bytes},
    }
    line.update(res)
    if args.only == "step" and not args.mixed and not args.no_mixed_report:
        # the mixed-precision form (FP32 sweeps and basis, FP64 reductions, Galerkin, SVD,
        # DSA) once each, after the timed region, against this step's FP64 results
        mkw = dict(solve_kw, mixed=True)
        frm = R.solve(prob, full_rank=1, **mkw)
        lrm = R.solve(prob, rand=W.random_stream(wl["seed"]), full_rank=0, p=wl["p"], q=wl["q"],
                      eps_res=wl["eps_res"], eps_diff=wl["eps_diff"], eps_svd=wl["eps_svd"],
                      eps_mgs=wl["eps_mgs"], m_max=wl["m_max"], **mkw)
        fr, lr = outs[-1]["fr"], outs[-1]["lr"]
        nrm = lambda a, b: float((a.double() - b.double()).norm() / b.double().norm())
        line["mixed"] = {
            "fr_time_to_tol_s": frm["ms_total"] / 1e3, "lr_time_to_tol_s": lrm["ms_total"] / 1e3,
            "fr_outer_iters": frm["iters"], "lr_outer_iters": lrm["iters"], "lr_rank": lrm["rank"],
            "fr_phi_vs_fp64_fr_rel_l2": nrm(frm["phi"], fr["phi"]),
            "lr_phi_vs_fp64_lr_rel_l2": nrm(lrm["phi"], lr["phi"]),
            "lr_phi_vs_fp64_fr_rel_l2": nrm(lrm["phi"], fr["phi"]),
            "target_rel_l2": 1e-5,
        }
    if not args.no_cpu_baseline and args.only == "step":
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_sweeps)
    plan.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
