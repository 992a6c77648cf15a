"""TEST INFRASTRUCTURE ONLY: FP64 CPU oracle for the FFT-based Poisson solve.

The oracle is a plain C implementation (``poisson_oracle.c``) of the solve in
FluTAS (arXiv 2204.08834), Section 3.3.1: textbook expansions along x and y
(DFTs for periodic axes, cosine / sine sums for Neumann / Dirichlet walls),
Gauss elimination (Thomas) along z for walls or a DFT along z when periodic,
the inverse expansions, and a zero-mean gauge when the constant is in the
operator's null space.  It shares no code with the GPU
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use it.

Arrays are numpy float64 of shape (nz, ny, nx), x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "poisson_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

PERIODIC = 0
NEUMANN = 1
DIRICHLET = 2

# Planted mistakes (mirrors the MUT_* constants in poisson_oracle.c).
MUTATIONS = {
    "fwd_sign_x": 1,
    "wall_row": 2,
    "half_angle": 3,
    "swap_dxdy": 4,
    "no_norm_y": 5,
    "no_gauge": 6,
    "drop_z": 7,
    "offdiag": 8,
    "idx_y": 9,
    "dir_row": 10,
    "cos_shift": 11,
    "sin_index": 12,
    "res_no_sqrt": 13,
    "lap_dir_x": 14,
    "lap_dir_y": 15,
    "res_no_mean": 16,
    "res_mean_dir": 17,
    "h_face": 18,
    "h_mean": 19,
}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build(force=True)
    lib = ctypes.CDLL(LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_solve_ex.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
    lib.oracle_solve_ex.restype = ctypes.c_int
    lib.oracle_solve_bc.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int] * 3 + [dp, dp, dp, dp, ctypes.c_int]
    lib.oracle_solve_bc.restype = ctypes.c_int
    lib.oracle_laplacian_bc.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int] * 3 + [dp, dp]
    lib.oracle_laplacian_bc.restype = ctypes.c_int
    lib.oracle_laplacian_bc_mut.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int] * 3 + [dp, dp, ctypes.c_int]
    lib.oracle_laplacian_bc_mut.restype = ctypes.c_int
    lib.oracle_residual_bc.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int] * 3 + [dp, dp, dp, dp, dp]
    lib.oracle_residual_bc.restype = ctypes.c_int
    lib.oracle_residual_bc_mut.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int] * 3 + [dp, dp, dp, dp, dp, ctypes.c_int]
    lib.oracle_residual_bc_mut.restype = ctypes.c_int
    lib.oracle_laplacian.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int, dp, dp]
    lib.oracle_laplacian.restype = ctypes.c_int
    lib.oracle_residual.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int, dp, dp, dp, dp, dp]
    lib.oracle_residual.restype = ctypes.c_int
    lib.oracle_divergence_bc.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int] * 3 + [dp, dp, dp, ctypes.c_double, dp]
    lib.oracle_divergence_bc.restype = ctypes.c_int
    lib.oracle_correct_bc.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [
        ctypes.c_int] * 3 + [dp, ctypes.c_double, dp, dp, dp]
    lib.oracle_correct_bc.restype = ctypes.c_int
    lib.oracle_solve_bc_h.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [dp] + [
        ctypes.c_int] * 3 + [dp, dp, dp, dp, ctypes.c_int]
    lib.oracle_solve_bc_h.restype = ctypes.c_int
    lib.oracle_laplacian_bc_h.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [dp] + [
        ctypes.c_int] * 3 + [dp, dp, ctypes.c_int]
    lib.oracle_laplacian_bc_h.restype = ctypes.c_int
    lib.oracle_residual_bc_h.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [dp] + [
        ctypes.c_int] * 3 + [dp, dp, dp, dp, dp, ctypes.c_int]
    lib.oracle_residual_bc_h.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim != 3:
        raise ValueError("expected a (nz, ny, nx) array")
    return f


def _cells(dz_cells, nz):
    h = np.ascontiguousarray(dz_cells, dtype=np.float64)
    if h.shape != (nz,):
        raise ValueError(f"dz_cells must hold nz = {nz} cell thicknesses")
    return h


def solve(f, dx, dy, dz, bc_z, mutation: int | str = 0, return_info: bool = False,
          bc_x: int = PERIODIC, bc_y: int = PERIODIC, dz_cells=None):
    """p with L p = f - mean(f), zero-mean, when no axis is Dirichlet; else
    L p = f.  Boundaries per axis: PERIODIC (0), NEUMANN (1), DIRICHLET (2).
    dz_cells: nz cell thicknesses of a z-stretched grid (walls in z; dz is
    then unused): the mean and the gauge are volume-weighted."""
    lib = _load()
    f = _check(f)
    nz, ny, nx = f.shape
    p = np.empty_like(f)
    mean = ctypes.c_double(0.0)
    mim = ctypes.c_double(0.0)
    mutation = _mutation(mutation)
    if dz_cells is not None:
        h = _cells(dz_cells, nz)
        rc = lib.oracle_solve_bc_h(nx, ny, nz, dx, dy, _ptr(h), int(bc_x), int(bc_y), int(bc_z),
                                   _ptr(f), _ptr(p), ctypes.byref(mean), ctypes.byref(mim),
                                   int(mutation))
    else:
        rc = lib.oracle_solve_bc(nx, ny, nz, dx, dy, dz, int(bc_x), int(bc_y), int(bc_z),
                                 _ptr(f), _ptr(p), ctypes.byref(mean), ctypes.byref(mim),
                                 int(mutation))
    if rc != 0:
        raise RuntimeError(f"oracle_solve failed ({rc})")
    if return_info:
        return p, {"rhs_mean": mean.value, "max_imag_ratio": mim.value}
    return p


def _mutation(m):
    return MUTATIONS[m] if isinstance(m, str) else int(m)


def laplacian(p, dx, dy, dz, bc_z, bc_x: int = PERIODIC, bc_y: int = PERIODIC,
              mutation: int | str = 0, dz_cells=None):
    """L p, the 7-point operator with the ghost rule of each axis (with
    dz_cells: the conservative z part on cells of those thicknesses)."""
    lib = _load()
    p = _check(p)
    nz, ny, nx = p.shape
    out = np.empty_like(p)
    if dz_cells is not None:
        h = _cells(dz_cells, nz)
        rc = lib.oracle_laplacian_bc_h(nx, ny, nz, dx, dy, _ptr(h), int(bc_x), int(bc_y),
                                       int(bc_z), _ptr(p), _ptr(out), _mutation(mutation))
    else:
        rc = lib.oracle_laplacian_bc_mut(nx, ny, nz, dx, dy, dz, int(bc_x), int(bc_y), int(bc_z),
                                         _ptr(p), _ptr(out), _mutation(mutation))
    if rc != 0:
        raise RuntimeError("oracle_laplacian failed")
    return out


def residual(f, p, dx, dy, dz, bc_z, return_field: bool = False, bc_x: int = PERIODIC,
             bc_y: int = PERIODIC, mutation: int | str = 0, dz_cells=None):
    """Relative residual ||(f - mean f) - L p||_2 / ||f - mean f||_2 (and Linf);
    the mean is removed only when no axis is Dirichlet (volume-weighted with
    dz_cells)."""
    lib = _load()
    f = _check(f)
    p = _check(p)
    nz, ny, nx = f.shape
    r = np.empty_like(f) if return_field else None
    l2 = ctypes.c_double()
    li = ctypes.c_double()
    if dz_cells is not None:
        h = _cells(dz_cells, nz)
        rc = lib.oracle_residual_bc_h(nx, ny, nz, dx, dy, _ptr(h), int(bc_x), int(bc_y),
                                      int(bc_z), _ptr(f), _ptr(p),
                                      _ptr(r) if r is not None else None, ctypes.byref(l2),
                                      ctypes.byref(li), _mutation(mutation))
    else:
        rc = lib.oracle_residual_bc_mut(nx, ny, nz, dx, dy, dz, int(bc_x), int(bc_y), int(bc_z),
                                        _ptr(f), _ptr(p), _ptr(r) if r is not None else None,
                                        ctypes.byref(l2), ctypes.byref(li), _mutation(mutation))
    if rc != 0:
        raise RuntimeError("oracle_residual failed")
    if return_field:
        return l2.value, li.value, r
    return l2.value, li.value


def divergence(u, v, w, dx, dy, dz, bc_z, alpha=1.0, bc_x: int = PERIODIC,
               bc_y: int = PERIODIC):
    """alpha * D u: cell divergence of face velocities (u east, v north, w top
    faces).  Per axis PERIODIC or NEUMANN (solid walls: the last face of the
    axis is the wall and, like the face below the first cell, carries no
    flux)."""
    lib = _load()
    u, v, w = _check(u), _check(v), _check(w)
    nz, ny, nx = u.shape
    f = np.empty_like(u)
    rc = lib.oracle_divergence_bc(nx, ny, nz, dx, dy, dz, int(bc_x), int(bc_y), int(bc_z),
                                  _ptr(u), _ptr(v), _ptr(w), float(alpha), _ptr(f))
    if rc != 0:
        raise RuntimeError("oracle_divergence failed")
    return f


def correct(u, v, w, psi, dx, dy, dz, bc_z, beta=1.0, bc_x: int = PERIODIC,
            bc_y: int = PERIODIC):
    """(u, v, w) - beta * G psi on the faces (copies; wall faces unchanged)."""
    lib = _load()
    u, v, w = _check(u).copy(), _check(v).copy(), _check(w).copy()
    psi = _check(psi)
    nz, ny, nx = u.shape
    rc = lib.oracle_correct_bc(nx, ny, nz, dx, dy, dz, int(bc_x), int(bc_y), int(bc_z),
                               _ptr(psi), float(beta), _ptr(u), _ptr(v), _ptr(w))
    if rc != 0:
        raise RuntimeError("oracle_correct failed")
    return u, v, w


def project(u, v, w, dx, dy, dz, bc_z, alpha=1.0, beta=1.0, bc_x: int = PERIODIC,
            bc_y: int = PERIODIC):
    """The projection around the solve: f = alpha D u, psi = the zero-mean
    solution of L psi = f - mean(f), and the corrected velocities."""
    f = divergence(u, v, w, dx, dy, dz, bc_z, alpha, bc_x=bc_x, bc_y=bc_y)
    psi = solve(f, dx, dy, dz, bc_z, bc_x=bc_x, bc_y=bc_y)
    return psi, correct(u, v, w, psi, dx, dy, dz, bc_z, beta, bc_x=bc_x, bc_y=bc_y)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))
