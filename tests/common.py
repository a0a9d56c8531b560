"""Builds the same seeded problem twice: once for the oracle (its own quadrature,
moments and assembly) and once for the HIP library (the library's own quadrature and
moments).  Only workload descriptions and random numbers are shared."""
import numpy as np

from oracle import dg, quadrature, si


def oracle_problem(wl, bc_faces=None):
    x0, x1, y0, y1 = wl["domain"]
    m = dg.Mesh(wl["nx"], wl["ny"], x0, x1, y0, y1)
    d, w = quadrature.cl_quadrature(wl["n_theta"], wl["n_z"])
    G = np.zeros(m.ndof)
    for val, box in wl.get("source_boxes", []):
        G += dg.source_moments_box(m, val, box)
    if wl.get("source_fn") is not None:
        G += dg.source_moments_function(m, wl["source_fn"], nq=12)
    bc = None
    if bc_faces:
        bc = np.zeros((4, max(m.nx, m.ny), 2))
        for side, i, val in bc_faces:
            bc[side, i, 0] += val * np.sqrt(m.hy if side < 2 else m.hx)
    return si.Problem(m, d, w, np.asarray(wl["sigma_t"]).reshape(-1),
                      np.asarray(wl["sigma_s"]).reshape(-1), G, bc)


def gpu_problem(wl, bc_faces=None, bc=None):
    import paper_2603_25233_amd as R
    d, w = R.cl_quadrature(wl["n_theta"], wl["n_z"])
    G = R.box_source_moments(wl["nx"], wl["ny"], wl["domain"], wl.get("source_boxes", []))
    if wl.get("source_gauss") is not None:
        amp, alpha, centre = wl["source_gauss"]
        G = G + R.gaussian_source_moments(wl["nx"], wl["ny"], wl["domain"], amp, alpha, centre)
    if bc is None and bc_faces:
        bc = R.inflow_moments(wl["nx"], wl["ny"], wl["domain"], bc_faces)
    return R.Problem(wl["nx"], wl["ny"], wl["domain"], d, w, wl["sigma_t"], wl["sigma_s"],
                     G=G, bc=bc)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
