"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/poisson.h, and validates descriptors before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2204_08834_amd import poisson as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "poisson.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(poisson_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(P.SYMBOLS) == names


def test_error_strings():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = P.error_string(code)
        assert s and "unknown" not in s
    assert "unknown" in P.error_string(-99)


def test_desc_init_defaults():
    d = P.Desc()
    assert P.lib().poisson_desc_init(ctypes.byref(d)) == 0
    assert (d.bc_x, d.bc_y, d.bc_z, d.precision) == (0, 0, 0, 0)
    assert d.rtol == 1e-10 and d.max_refine == 8 and d.dx == 1.0
    assert P.lib().poisson_desc_init(None) == P.ERR_INVALID_ARG


@pytest.mark.parametrize("shape,bc", [((512, 512, 256), 1), ((256, 256, 256), 0),
                                      ((1024, 1024, 512), 1), ((96, 96, 48), 1),
                                      ((64, 64, 64), 0), ((2, 1, 1), 0), ((32, 32, 33), 1),
                                      ((2048, 2048, 1), 1), ((6, 3, 12), 0), ((64, 32, 33), 2),
                                      ((8, 8, 4096), 2)])
def test_valid_descriptors(shape, bc):
    d = P.make_desc(*shape, 0.1, 0.2, 0.3, bc, "fp32_refine")
    assert P.validate(d) == P.OK


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), P.ERR_INVALID_ARG),
    (dict(ny=0), P.ERR_INVALID_ARG),
    (dict(nz=0), P.ERR_INVALID_ARG),
    (dict(nx=7), P.ERR_UNSUPPORTED),            # odd nx
    (dict(nx=20), P.ERR_UNSUPPORTED),           # nx/2 = 10 has a factor 5
    (dict(nx=4096), P.ERR_UNSUPPORTED),         # nx/2 above 1024
    (dict(ny=10), P.ERR_UNSUPPORTED),
    (dict(ny=18), P.ERR_UNSUPPORTED),           # 2*3^2 is not instantiated
    (dict(nz=10, bc_z=0), P.ERR_UNSUPPORTED),   # periodic z needs an FFT length
    (dict(nz=10000, bc_z=1), P.ERR_UNSUPPORTED),
    (dict(dx=0.0), P.ERR_INVALID_ARG),
    (dict(dy=-1.0), P.ERR_INVALID_ARG),
    (dict(dz=float("nan")), P.ERR_INVALID_ARG),
    (dict(dz=float("inf")), P.ERR_INVALID_ARG),
    (dict(bc_z=3), P.ERR_INVALID_ARG),
    (dict(bc_x=3), P.ERR_INVALID_ARG),
    (dict(bc_y=3), P.ERR_INVALID_ARG),
    (dict(bc_x=5), P.ERR_INVALID_ARG),
    (dict(precision=3), P.ERR_INVALID_ARG),
    (dict(precision="fp32_refine", rtol=0.0), P.ERR_INVALID_ARG),
    (dict(precision="fp32_refine", rtol=float("nan")), P.ERR_INVALID_ARG),
    (dict(precision="fp32_refine", max_refine=0), P.ERR_INVALID_ARG),
])
def test_invalid_descriptors(kw, code):
    base = dict(nx=64, ny=64, nz=32, dx=0.1, dy=0.1, dz=0.1, bc_z=1, precision="fp64",
                rtol=1e-10, max_refine=8, bc_x=0, bc_y=0)
    base.update(kw)
    d = P.make_desc(**base)
    assert P.validate(d) == code
    assert P.workspace_bytes(d) == 0


def test_validate_null_and_plan_null_args():
    L = P.lib()
    assert L.poisson_desc_validate(None) == P.ERR_INVALID_ARG
    assert L.poisson_plan_create(None, None, None) == P.ERR_INVALID_ARG
    assert L.poisson_batch_plan_create(None, 0, None, None) == P.ERR_INVALID_ARG
    assert L.poisson_solve(None, None, None, None) == P.ERR_INVALID_ARG
    assert L.poisson_batch_solve(None, None, None, None) == P.ERR_INVALID_ARG
    assert L.poisson_destroy(None) == P.OK
    assert L.poisson_plan_set_timing(None, 1) == P.ERR_INVALID_ARG
    n = ctypes.c_int()
    assert L.poisson_plan_get_timing(None, None, 0, ctypes.byref(n)) == P.ERR_INVALID_ARG


def test_invalid_descriptor_rejected_before_any_hip_call():
    # plan creation with a bad descriptor returns before touching the device,
    # so it behaves the same on a machine without a GPU
    d = P.make_desc(10, 64, 32)
    h = ctypes.c_void_p()
    assert P.lib().poisson_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == \
        P.ERR_UNSUPPORTED
    assert h.value is None


def test_workspace_bytes():
    d64 = P.make_desc(512, 512, 256, precision="fp64")
    d32 = P.make_desc(512, 512, 256, precision="fp32_refine")
    n = 512 * 512 * 256
    # FP64 works in place in the solution array; FP32 needs a 4 B/point
    # spectrum, and the refinement a 4 B/point copy of its first iterate
    d32p = P.make_desc(512, 512, 256, precision="fp32")
    assert P.workspace_bytes(d64) < 1 << 20
    assert n * 4 <= P.workspace_bytes(d32p) < n * 4.1
    assert n * 8 <= P.workspace_bytes(d32) < n * 8.1


def test_set_graph_rejects_null_plan():
    L = P.lib()
    assert L.poisson_plan_set_graph(None, 1) == P.ERR_INVALID_ARG
    assert P.GRAPH_MODES == {"host": 0, "graph": 1, "device": 2}


def test_autotune_and_describe_reject_null_plan():
    L = P.lib()
    assert L.poisson_plan_autotune(None, 0) == P.ERR_INVALID_ARG
    buf = ctypes.create_string_buffer(64)
    assert L.poisson_plan_describe(None, buf, 64) == P.ERR_INVALID_ARG


def test_project_rejects_null_plan_and_fields():
    L = P.lib()
    st = P.Stats()
    fake = ctypes.c_void_p(0x1000)
    assert L.poisson_project(None, fake, fake, fake, None, fake, 1.0, 1.0,
                             ctypes.byref(st)) == P.ERR_INVALID_ARG


def test_batch_argument_checks_are_not_cached_on_failure():
    """The batch binding caches a successful check of its tensors only: a
    rejected call is rejected again, whatever came before it."""
    torch = pytest.importorskip("torch")
    bp = P.BatchPlan.__new__(P.BatchPlan)
    bp._h, bp.count, bp._validated = None, 2, None
    bp.shapes = [(4, 4, 4), (2, 4, 6)]
    cpu = [torch.zeros(s, dtype=torch.float64) for s in bp.shapes]
    for _ in range(2):
        with pytest.raises(ValueError, match="GPU"):
            bp._pointers(cpu, cpu)
        assert bp._validated is None
    with pytest.raises(TypeError):
        bp._pointers(["not a tensor", cpu[1]], cpu)
    with pytest.raises(ValueError, match="one rhs"):
        bp._pointers(cpu[:1], cpu)
