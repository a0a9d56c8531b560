"""Transport sweep of the oracle (Sec. 2.2, "Transport sweeps"; eqs. (SI), (sampled-sweep)).

Python side: builds the per-direction 4x4 cell blocks from the weak form (oracle.dg)
and hands them to the plain-C pass in csweep.c.  The C pass is checked in the tests
against a sparse direct solve of the assembled (D_j + Sigma_t) on small grids.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import dg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csweep.c")
_LIB = os.path.join(_HERE, "_csweep.so")
_lib = None


def build(force=False):
    """Compile csweep.c with gcc (OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        lib.oracle_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P,
                                     P, P, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int]
        lib.oracle_sweep.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


_BLOCKS = {}


def direction_blocks(mesh, dirs, sel):
    """Cell blocks (A, Bx, By) of each selected direction from the weak form (Sec. 2.1)."""
    n = len(sel)
    A = np.zeros((n, 16)); Bx = np.zeros((n, 16)); By = np.zeros((n, 16))
    cache = _BLOCKS
    if len(cache) > 100000:
        cache.clear()
    for i, j in enumerate(sel):
        ox, oy = float(dirs[j, 0]), float(dirs[j, 1])
        key = (ox, oy, mesh.hx, mesh.hy)
        if key not in cache:
            Ac, B = dg.cell_transport(ox, oy, mesh.hx, mesh.hy)
            bx = B.get("L" if ox > 0 else "R", np.zeros((4, 4))) if ox != 0 else np.zeros((4, 4))
            by = B.get("B" if oy > 0 else "T", np.zeros((4, 4))) if oy != 0 else np.zeros((4, 4))
            cache[key] = (Ac.reshape(-1), bx.reshape(-1), by.reshape(-1))
        A[i], Bx[i], By[i] = cache[key]
    return A, Bx, By


def sweep(mesh, dirs, sel, sigma_t, src, bnd=None, want_psi=True, w=None,
          transpose=False, nthreads=0):
    """Solve (D_j + Sigma_t) psi_j = src + g_j^bc for each j in sel (eq. (SI)).

    src: isotropic right-hand side [ndof] (e.g. Sigma_s phi + G).  bnd: unit boundary
    moments from dg.boundary_unit_vectors (None = vacuum).  With transpose=True solves
    (D_j + Sigma_t)^T mu_j = src + (outflow-side boundary data) instead.
    Returns (psi [n_sel, ndof] or None, phi = sum_i w_i psi_i or None).
    """
    lib = _load()
    sel = np.asarray(sel, dtype=np.int64).reshape(-1)
    A, Bx, By = direction_blocks(mesh, dirs, sel)
    ox = np.ascontiguousarray(dirs[sel, 0], dtype=np.float64)
    oy = np.ascontiguousarray(dirs[sel, 1], dtype=np.float64)
    mb = max(mesh.nx, mesh.ny)
    if bnd is None:
        bnd = np.zeros((4, mb, 4))
    bnd = np.ascontiguousarray(bnd, dtype=np.float64)
    sig = np.ascontiguousarray(np.asarray(sigma_t, dtype=np.float64).reshape(-1))
    src = np.ascontiguousarray(np.asarray(src, dtype=np.float64).reshape(-1))
    assert src.size == mesh.ndof and sig.size == mesh.ncell
    psi = np.empty((len(sel), mesh.ndof)) if want_psi else None
    phi = None
    wsel = None
    if w is not None:
        phi = np.empty(mesh.ndof)
        wsel = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1))
        assert wsel.size == len(sel)
    rc = lib.oracle_sweep(mesh.nx, mesh.ny, len(sel), _ptr(ox), _ptr(oy), _ptr(A), _ptr(Bx),
                          _ptr(By), _ptr(sig), _ptr(src), _ptr(bnd), mb, _ptr(wsel), _ptr(psi),
                          _ptr(phi), int(bool(transpose)), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle sweep: allocation failed")
    return psi, phi
