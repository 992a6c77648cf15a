"""ctypes binding of libpoisson.so (the C ABI in include/poisson.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory (float64 CUDA tensors of shape
(nz, ny, nx)) and the stream.  If the library is missing the binding raises;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpoisson.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED = -2
ERR_OUT_OF_MEMORY = -3
ERR_HIP = -4
ERR_NOT_CONVERGED = -5
ERR_NONFINITE = -6
ERR_TOO_LARGE = -7

BC_PERIODIC = 0
BC_NEUMANN = 1
BC_DIRICHLET = 2

FP64 = 0
FP32_REFINE = 1
FP32 = 2
_PREC = {"fp64": FP64, "fp32_refine": FP32_REFINE, "fp32": FP32}


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("bc_z", ctypes.c_int),
                ("precision", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_refine", ctypes.c_int), ("dz_cells", ctypes.POINTER(ctypes.c_double))]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("rhs_mean", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self):
        return {"iterations": self.iterations, "rel_residual": self.rel_residual,
                "rhs_mean": self.rhs_mean, "status": self.status}


class PassStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int),
                ("total_ms", ctypes.c_double), ("bytes_per_launch", ctypes.c_double)]


class PoissonError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {error_string(code)} ({code})" if what else error_string(code))


_lib = None

# every entry point of include/poisson.h
SYMBOLS = ["poisson_desc_init", "poisson_desc_validate", "poisson_workspace_bytes",
           "poisson_plan_create", "poisson_solve", "poisson_destroy",
           "poisson_batch_plan_create", "poisson_batch_solve", "poisson_error_string",
           "poisson_plan_set_timing", "poisson_plan_reset_timing", "poisson_plan_get_timing",
           "poisson_plan_set_graph", "poisson_plan_autotune", "poisson_plan_describe",
           "poisson_project", "poisson_solve_noalloc"]

# refinement-loop drivers of poisson_plan_set_graph
GRAPH_MODES = {"host": 0, "graph": 1, "device": 2}


def lib():
    """Load libpoisson.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2204_08834_amd.build` (HIP, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(Desc)
    L.poisson_desc_init.argtypes = [dp]
    L.poisson_desc_validate.argtypes = [dp]
    L.poisson_workspace_bytes.argtypes = [dp]
    L.poisson_workspace_bytes.restype = ctypes.c_size_t
    L.poisson_plan_create.argtypes = [dp, P, ctypes.POINTER(P)]
    L.poisson_solve.argtypes = [P, P, P, ctypes.POINTER(Stats)]
    L.poisson_destroy.argtypes = [P]
    L.poisson_batch_plan_create.argtypes = [dp, ctypes.c_int, P, ctypes.POINTER(P)]
    L.poisson_batch_solve.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P),
                                      ctypes.POINTER(Stats)]
    L.poisson_error_string.argtypes = [ctypes.c_int]
    L.poisson_error_string.restype = ctypes.c_char_p
    L.poisson_plan_set_timing.argtypes = [P, ctypes.c_int]
    L.poisson_plan_reset_timing.argtypes = [P]
    L.poisson_plan_get_timing.argtypes = [P, ctypes.POINTER(PassStat), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]
    L.poisson_plan_set_graph.argtypes = [P, ctypes.c_int]
    L.poisson_plan_autotune.argtypes = [P, ctypes.c_int]
    L.poisson_plan_describe.argtypes = [P, ctypes.c_char_p, ctypes.c_int]
    L.poisson_project.argtypes = [P, P, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(Stats)]
    L.poisson_solve_noalloc.argtypes = [dp, P, P, P, ctypes.POINTER(Stats)]
    for name in SYMBOLS:
        if name != "poisson_workspace_bytes" and name != "poisson_error_string":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def error_string(code: int) -> str:
    return lib().poisson_error_string(int(code)).decode()


def make_desc(nx, ny, nz, dx=1.0, dy=1.0, dz=1.0, bc_z=BC_NEUMANN, precision="fp64",
              rtol=1e-10, max_refine=8, bc_x=BC_PERIODIC, bc_y=BC_PERIODIC,
              dz_cells=None) -> Desc:
    """A descriptor; dz_cells: nz cell thicknesses of a z-stretched grid (the
    array is kept alive with the descriptor, the library copies it)."""
    d = Desc()
    lib().poisson_desc_init(ctypes.byref(d))
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.dx, d.dy, d.dz = float(dx), float(dy), float(dz)
    d.bc_x, d.bc_y, d.bc_z = int(bc_x), int(bc_y), int(bc_z)
    d.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    d.rtol = float(rtol)
    d.max_refine = int(max_refine)
    if dz_cells is not None:
        import numpy as np
        h = np.ascontiguousarray(dz_cells, dtype=np.float64)
        d._h = h  # keeps the buffer alive while the descriptor is used
        d.dz_cells = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d


def validate(desc: Desc) -> int:
    return lib().poisson_desc_validate(ctypes.byref(desc))


def workspace_bytes(desc: Desc) -> int:
    return int(lib().poisson_workspace_bytes(ctypes.byref(desc)))


def _check_field(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def solve_noalloc(rhs, out, dx=1.0, dy=1.0, dz=1.0, bc_z=BC_NEUMANN, precision="fp64",
                  rtol=1e-10, max_refine=8, bc_x=BC_PERIODIC, bc_y=BC_PERIODIC, stream=None,
                  check=True, dz_cells=None):
    """poisson_solve_noalloc: one solve without a plan and without device
    allocation (the library's fixed per-GPU scratch).  rhs, out: float64 GPU
    tensors of shape (nz, ny, nx).  Returns the stats dict."""
    nz, ny, nx = rhs.shape
    _check_field(rhs, (nz, ny, nx), "rhs")
    _check_field(out, (nz, ny, nx), "out")
    d = make_desc(nx, ny, nz, dx, dy, dz, bc_z, precision, rtol, max_refine, bc_x, bc_y,
                  dz_cells)
    st = Stats()
    rc = lib().poisson_solve_noalloc(ctypes.byref(d), _stream_handle(stream),
                                     ctypes.c_void_p(rhs.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
    if check and rc != OK:
        raise PoissonError(rc, "poisson_solve_noalloc")
    r = st.as_dict()
    r["status"] = rc
    return r


class Plan:
    """One Poisson problem (grid, spacings, z boundary, precision) on one stream."""

    def __init__(self, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0, bc_z=BC_NEUMANN, precision="fp64",
                 rtol=1e-10, max_refine=8, stream=None, bc_x=BC_PERIODIC, bc_y=BC_PERIODIC,
                 dz_cells=None):
        self.desc = make_desc(nx, ny, nz, dx, dy, dz, bc_z, precision, rtol, max_refine,
                              bc_x, bc_y, dz_cells)
        self.shape = (nz, ny, nx)
        self._stream = stream
        h = ctypes.c_void_p()
        rc = lib().poisson_plan_create(ctypes.byref(self.desc), _stream_handle(stream),
                                       ctypes.byref(h))
        if rc != OK:
            raise PoissonError(rc, "poisson_plan_create")
        self._h = h

    def solve(self, rhs, out=None, check=True):
        """Solve L p = rhs - mean(rhs); returns (p, stats dict)."""
        import torch
        _check_field(rhs, self.shape, "rhs")
        if out is None:
            out = torch.empty_like(rhs)
        _check_field(out, self.shape, "out")
        st = Stats()
        rc = lib().poisson_solve(self._h, ctypes.c_void_p(rhs.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.byref(st))
        if check and rc not in (OK,):
            raise PoissonError(rc, "poisson_solve")
        d = st.as_dict()
        d["status"] = rc
        return out, d

    def solve_async(self, rhs, out):
        """Enqueue a solve without reading statistics (no host synchronisation
        except the once-per-iteration residual read of FP32_REFINE)."""
        _check_field(rhs, self.shape, "rhs")
        _check_field(out, self.shape, "out")
        rc = lib().poisson_solve(self._h, ctypes.c_void_p(rhs.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), None)
        if rc != OK:
            raise PoissonError(rc, "poisson_solve")
        return rc

    def project(self, u, v, w, p=None, psi=None, alpha=1.0, beta=1.0, check=True,
                stats=True):
        """Projection step (poisson_project): solve L psi = alpha D(u, v, w),
        then u -= beta G psi (in place, likewise v and w) and p += psi when p
        is given.  Returns (psi, stats dict or None)."""
        import torch
        for t, name in ((u, "u"), (v, "v"), (w, "w")):
            _check_field(t, self.shape, name)
        if p is not None:
            _check_field(p, self.shape, "p")
        if psi is None:
            psi = torch.empty_like(u)
        _check_field(psi, self.shape, "psi")
        st = Stats()
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        rc = lib().poisson_project(self._h, ptr(u), ptr(v), ptr(w), ptr(p), ptr(psi),
                                   float(alpha), float(beta), ctypes.byref(st) if stats else None)
        if check and rc != OK:
            raise PoissonError(rc, "poisson_project")
        if not stats:
            return psi, None
        d = st.as_dict()
        d["status"] = rc
        return psi, d

    def set_timing(self, enable=True):
        lib().poisson_plan_set_timing(self._h, 1 if enable else 0)

    def reset_timing(self):
        lib().poisson_plan_reset_timing(self._h)

    def timing(self):
        return _get_timing(self._h)

    def set_graph(self, mode="graph"):
        _set_graph(self._h, mode)

    def autotune(self, force=False):
        _autotune(self._h, force)

    def describe(self):
        return _describe(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


TUNE_FORCE = 1


def _autotune(h, force=False):
    rc = lib().poisson_plan_autotune(h, TUNE_FORCE if force else 0)
    if rc != OK:
        raise PoissonError(rc, "poisson_plan_autotune")


def _describe(h):
    buf = ctypes.create_string_buffer(1 << 16)
    rc = lib().poisson_plan_describe(h, buf, len(buf))
    if rc != OK:
        raise PoissonError(rc, "poisson_plan_describe")
    return buf.value.decode()


def _set_graph(h, mode):
    m = GRAPH_MODES[mode] if isinstance(mode, str) else int(mode)
    rc = lib().poisson_plan_set_graph(h, m)
    if rc != OK:
        raise PoissonError(rc, "poisson_plan_set_graph")


def _get_timing(h):
    n = ctypes.c_int(0)
    lib().poisson_plan_get_timing(h, None, 0, ctypes.byref(n))
    arr = (PassStat * max(1, n.value))()
    lib().poisson_plan_get_timing(h, arr, n.value, ctypes.byref(n))
    return {a.name.decode(): {"launches": a.launches, "total_ms": a.total_ms,
                              "bytes_per_launch": a.bytes_per_launch}
            for a in arr[: n.value]}


class BatchPlan:
    """Several independent problems (possibly different shapes) on one stream."""

    def __init__(self, problems, precision="fp64", rtol=1e-10, max_refine=8, stream=None):
        """problems: list of dicts with nx, ny, nz, dx, dy, dz, bc_z (and
        optionally bc_x, bc_y)."""
        n = len(problems)
        arr = (Desc * n)()
        keep = []  # descriptors whose thickness arrays arr's copies point to
        for i, p in enumerate(problems):
            d = make_desc(p["nx"], p["ny"], p["nz"], p["dx"], p["dy"], p["dz"],
                          p["bc_z"], precision, rtol, max_refine,
                          p.get("bc_x", BC_PERIODIC), p.get("bc_y", BC_PERIODIC),
                          p.get("dz_cells"))
            keep.append(d)
            arr[i] = d
        self.shapes = [(p["nz"], p["ny"], p["nx"]) for p in problems]
        h = ctypes.c_void_p()
        rc = lib().poisson_batch_plan_create(arr, n, _stream_handle(stream), ctypes.byref(h))
        if rc != OK:
            raise PoissonError(rc, "poisson_batch_plan_create")
        self._h = h
        self.count = n
        self._validated = None

    def _pointers(self, rhs_list, out_list):
        """Device pointers of the right-hand sides and outputs, after the
        checks of every tensor (float64, GPU, contiguous, the problem's
        shape).  A call with the same tensor objects as the previous one,
        unchanged in place (data pointers, shapes, contiguity, dtypes and
        devices), skips the per-tensor checks, which otherwise cost more
        than the launches of a small batch."""
        n = self.count
        if len(rhs_list) != n or len(out_list) != n:
            raise ValueError("one rhs and one output per problem")
        ts = [*rhs_list, *out_list]
        try:
            sig = [(t.data_ptr(), t.shape, t.is_contiguous(), t.dtype, t.is_cuda) for t in ts]
        except (AttributeError, TypeError):
            sig = None
        last = self._validated
        if (sig is None or last is None or sig != last[1]
                or not all(r() is t for r, t in zip(last[0], ts))):
            self._validated = None
            for i, (r, o) in enumerate(zip(rhs_list, out_list)):
                _check_field(r, self.shapes[i], f"rhs[{i}]")
                _check_field(o, self.shapes[i], f"out[{i}]")
            self._validated = ([weakref.ref(t) for t in ts], sig)
        ptrs = [x[0] for x in sig]
        return (ctypes.c_void_p * n)(*ptrs[:n]), (ctypes.c_void_p * n)(*ptrs[n:])

    def solve(self, rhs_list, out_list, check=True):
        R, O = self._pointers(rhs_list, out_list)
        st = (Stats * self.count)()
        rc = lib().poisson_batch_solve(self._h, R, O, st)
        if check and rc != OK:
            raise PoissonError(rc, "poisson_batch_solve")
        return rc, [s.as_dict() for s in st]

    def set_timing(self, enable=True):
        lib().poisson_plan_set_timing(self._h, 1 if enable else 0)

    def reset_timing(self):
        lib().poisson_plan_reset_timing(self._h)

    def timing(self):
        return _get_timing(self._h)

    def set_graph(self, mode="graph"):
        _set_graph(self._h, mode)

    def autotune(self, force=False):
        _autotune(self._h, force)

    def describe(self):
        return _describe(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
