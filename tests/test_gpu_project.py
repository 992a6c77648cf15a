"""GPU parity of the projection step (poisson_project) against the oracle.

The HIP path evaluates f = alpha D(u, v, w) inside its first transform pass,
solves L psi = f, and applies u -= beta G psi, p += psi in one march.  Checks:
  * psi against the oracle's solve of the oracle's divergence (FP64: 1e-12,
    or the conditioning bound; FP32 + refinement: the oracle's residual of
    psi <= 1e-10; FP32: 1e-4);
  * u, v, w against the oracle's correction applied to the GPU's own psi
    (isolates the correction kernel: rounding level), p == p0 + psi
    bitwise, the top-wall w untouched bitwise;
  * the corrected velocity is divergence-free (oracle divergence, host);
  * the device-side loop (graph / eager) gives the host loop's bits;
  * error paths leave u, v, w, p as they were.
Grids span several march tiles with ragged tails in y and z, the shortest
rows (nx = 2) and the longest (nx = 2048).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2204_08834_amd import inputs  # noqa: E402

NEU, PER = 1, 0

CASES = [
    (16, 12, 10, NEU), (64, 48, 20, NEU), (32, 32, 32, PER), (6, 3, 5, NEU),
    (2, 1, 1, NEU), (2, 4, 3, NEU), (24, 12, 6, PER), (512, 6, 9, NEU), (128, 24, 9, NEU),
    (96, 12, 6, PER), (2048, 2, 3, NEU), (8, 2, 1, PER),
]
IDS = [f"{c[0]}x{c[1]}x{c[2]}_{'w' if c[3] else 'p'}" for c in CASES]
BOX = (2.0, 1.5, 1.0)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_08834_amd import poisson
    poisson.lib()  # raises if the HIP library is missing: no fallback
    return poisson


def _fields(nx, ny, nz, bc, seed):
    u, v, w = inputs.uniform_velocity(nx, ny, nz, bc, seed)
    if bc == NEU:
        w[-1] = 0.25  # the wall value is neither read nor changed
    rng = np.random.default_rng(seed + 1000)
    p0 = rng.uniform(-1, 1, (nz, ny, nx))
    return u, v, w, p0


def _kappa(nx, ny, nz, dx, dy, dz, bc):
    def lam(n, h, j, walls=False):
        return 4 / h ** 2 * math.sin(math.pi * j / ((2 * n) if walls else n)) ** 2
    lmax = (lam(nx, dx, nx // 2) + lam(ny, dy, ny // 2)
            + (lam(nz, dz, nz - 1, True) if bc == NEU else lam(nz, dz, nz // 2)))
    c = [lam(nx, dx, 1) if nx > 1 else math.inf, lam(ny, dy, 1) if ny > 1 else math.inf,
         (lam(nz, dz, 1, True) if bc == NEU else lam(nz, dz, 1)) if nz > 1 else math.inf]
    return lmax / min(c)


def _run(P, case, prec, mode="host", alpha=3.0, beta=1.0 / 3.0, with_p=True, seed=5):
    nx, ny, nz, bc = case
    sp = (BOX[0] / nx, BOX[1] / ny, BOX[2] / nz)
    u, v, w, p0 = _fields(nx, ny, nz, bc, seed)
    du, dv, dw = (torch.from_numpy(a.copy()).cuda() for a in (u, v, w))
    dp = torch.from_numpy(p0.copy()).cuda() if with_p else None
    print(f"[project] {nx}x{ny}x{nz} bc={bc} {prec} {mode}", flush=True)
    with P.Plan(nx, ny, nz, *sp, bc, prec) as plan:
        plan.set_graph(mode)
        psi, st = plan.project(du, dv, dw, dp, alpha=alpha, beta=beta)
        torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in (du, dv, dw, psi)]
    return (u, v, w, p0), out, (dp.cpu().numpy() if with_p else None), st, sp


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_project_matches_oracle(orc, case, prec):
    P = _gpu()
    nx, ny, nz, bc = case
    alpha, beta = 3.0, 1.0 / 3.0
    (u, v, w, p0), (u1, v1, w1, psi), p1, st, sp = _run(P, case, prec, alpha=alpha, beta=beta)
    assert st["status"] == 0
    f = orc.divergence(u, v, w, *sp, bc, alpha=alpha)
    fmax = max(np.abs(f).max(), 1e-300)
    # the divergence of a periodic / walled field sums to zero
    assert abs(st["rhs_mean"]) <= 1e-12 * fmax
    psi_ref = orc.solve(f, *sp, bc)
    nref = max(np.linalg.norm(psi_ref), 1e-300)
    err = np.linalg.norm(psi - psi_ref) / nref if np.linalg.norm(f) > 0 else np.abs(psi).max()
    if prec == "fp64":
        tol = max(1e-12, 4 * _kappa(nx, ny, nz, *sp, bc) * 2.2e-16)
        print(f"[fp64-error] project {nx}x{ny}x{nz} bc={bc}: {err:.2e} (bound {tol:.2e})",
              flush=True)
        assert err <= tol, err
    elif prec == "fp32_refine":
        res, _ = orc.residual(f, psi, *sp, bc)
        assert res <= 1e-10, res
    else:
        assert err <= max(1e-4, 8 * _kappa(nx, ny, nz, *sp, bc) * 6e-8), err
    # correction kernel against the oracle's, on the GPU's own psi
    ur, vr, wr = orc.correct(u, v, w, psi, *sp, bc, beta=beta)
    for a, b, name in ((u1, ur, "u"), (v1, vr, "v"), (w1, wr, "w")):
        scale = max(np.abs(b).max(), 1.0)
        assert np.abs(a - b).max() <= 1e-14 * scale, name
    if bc == NEU:
        assert np.array_equal(w1[-1], w[-1])
    assert np.array_equal(p1, p0 + psi)
    # the corrected velocity is divergence-free up to the solve's accuracy
    d1 = orc.divergence(u1, v1, w1, *sp, bc)
    d0 = orc.divergence(u, v, w, *sp, bc)
    lim = {"fp64": 1e-11, "fp32_refine": 1e-9, "fp32": 1e-4}[prec]
    assert np.abs(d1).max() <= lim * max(np.abs(d0).max(), 1e-300), np.abs(d1).max()


@pytest.mark.parametrize("mode", ["graph", "device"])
@pytest.mark.parametrize("prec", ["fp32_refine", "fp64"])
def test_project_device_loop_matches_host_loop(prec, mode):
    P = _gpu()
    case = (64, 48, 20, NEU)
    _, a, pa, sa, _ = _run(P, case, prec, "host", seed=9)
    _, b, pb, sb, _ = _run(P, case, prec, mode, seed=9)
    assert sa == sb
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.array_equal(pa, pb)


def test_project_repeated_calls_and_without_p(orc):
    """A plan projects several fields in a row (graph mode: the segment graph
    is reused), with and without a pressure to update."""
    P = _gpu()
    nx, ny, nz, bc = 32, 24, 16, NEU
    sp = (BOX[0] / nx, BOX[1] / ny, BOX[2] / nz)
    with P.Plan(nx, ny, nz, *sp, bc, "fp32_refine") as plan:
        plan.set_graph("graph")
        for it, seed in enumerate((1, 2, 1)):
            u, v, w, _ = _fields(nx, ny, nz, bc, seed)
            du, dv, dw = (torch.from_numpy(x.copy()).cuda() for x in (u, v, w))
            psi, st = plan.project(du, dv, dw, None, alpha=2.0, beta=0.5)
            torch.cuda.synchronize()
            assert st["status"] == 0 and st["rel_residual"] <= 1e-10
            d1 = orc.divergence(du.cpu().numpy(), dv.cpu().numpy(), dw.cpu().numpy(), *sp, bc)
            d0 = orc.divergence(u, v, w, *sp, bc)
            print(f"[project] call {it}: max div {np.abs(d1).max():.2e}", flush=True)
            assert np.abs(d1).max() <= 1e-9 * np.abs(d0).max()


def test_project_nonfinite_leaves_fields(orc):
    P = _gpu()
    nx, ny, nz, bc = 32, 24, 16, NEU
    sp = (BOX[0] / nx, BOX[1] / ny, BOX[2] / nz)
    u, v, w, p0 = _fields(nx, ny, nz, bc, 3)
    u[3, 4, 5] = np.nan
    du, dv, dw, dp = (torch.from_numpy(x.copy()).cuda() for x in (u, v, w, p0))
    with P.Plan(nx, ny, nz, *sp, bc, "fp32_refine") as plan:
        psi, st = plan.project(du, dv, dw, dp, check=False)
        torch.cuda.synchronize()
    assert st["status"] == P.ERR_NONFINITE
    for a, b in ((du, u), (dv, v), (dw, w), (dp, p0)):
        assert np.array_equal(a.cpu().numpy(), b, equal_nan=True)


def test_project_argument_errors():
    P = _gpu()
    nx, ny, nz = 16, 8, 4
    with P.Plan(nx, ny, nz, 0.1, 0.1, 0.1, NEU, "fp64") as plan:
        u = torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda")
        v, w = torch.zeros_like(u), torch.zeros_like(u)
        # psi aliasing a velocity component: refused before any launch
        with pytest.raises(P.PoissonError) as e:
            plan.project(u, v, w, None, psi=u)
        assert e.value.code == P.ERR_INVALID_ARG
        with pytest.raises(P.PoissonError):
            plan.project(u, v, w, None, alpha=float("inf"))
    specs = [dict(nx=nx, ny=ny, nz=nz, dx=0.1, dy=0.1, dz=0.1, bc_z=NEU)]
    bp = P.BatchPlan(specs, "fp64")
    import ctypes
    rc = P.lib().poisson_project(bp._h, ctypes.c_void_p(u.data_ptr()),
                                 ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                 None, ctypes.c_void_p(torch.empty_like(u).data_ptr()), 1.0,
                                 1.0, None)
    bp.close()
    assert rc == P.ERR_INVALID_ARG


@pytest.mark.parametrize("prec", ["fp32_refine", "fp64"])
def test_project_rb512_full_size(orc, prec):
    """512 x 512 x 256 walls (box 2:2:1), the benchmark's launch
    configuration: the oracle's residual of psi and the divergence of the
    corrected velocity, on the host over the whole grid."""
    P = _gpu()
    nx, ny, nz, bc = 512, 512, 256, NEU
    sp = (2.0 / nx, 2.0 / ny, 1.0 / nz)
    print(f"[project] rb512 {prec}: generating velocities", flush=True)
    u, v, w = inputs.uniform_velocity(nx, ny, nz, bc, 3)
    du, dv, dw = (torch.from_numpy(x).cuda() for x in (u, v, w))
    with P.Plan(nx, ny, nz, *sp, bc, prec) as plan:
        psi, st = plan.project(du, dv, dw, None, alpha=1.0, beta=1.0)
        torch.cuda.synchronize()
    print(f"[project] rb512 {prec}: {st}", flush=True)
    assert st["status"] == 0
    f = orc.divergence(u, v, w, *sp, bc)
    psi_h = psi.cpu().numpy()
    del psi
    res, _ = orc.residual(f, psi_h, *sp, bc)
    print(f"[project] rb512 {prec}: oracle residual {res:.2e}", flush=True)
    assert res <= (1e-12 if prec == "fp64" else 1e-10)
    d1 = orc.divergence(du.cpu().numpy(), dv.cpu().numpy(), dw.cpu().numpy(), *sp, bc)
    assert np.abs(d1).max() <= (1e-11 if prec == "fp64" else 1e-9) * np.abs(f).max()
    del du, dv, dw
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# solid walls along x and y
# --------------------------------------------------------------------------
WALL_CASES = [((16, 12, 10), (NEU, NEU, NEU)), ((64, 48, 20), (PER, NEU, NEU)),
              ((24, 12, 8), (NEU, PER, PER)), ((6, 3, 5), (NEU, NEU, NEU)),
              ((512, 6, 9), (NEU, NEU, NEU)), ((2, 4, 3), (NEU, NEU, PER))]


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("case", WALL_CASES, ids=[f"{c[0][0]}x{c[0][1]}x{c[0][2]}_"
                                                  + "".join("PND"[b] for b in c[1])
                                                  for c in WALL_CASES])
def test_project_walls_match_oracle(orc, case, prec):
    P = _gpu()
    (nx, ny, nz), bcs = case
    sp = (BOX[0] / nx, BOX[1] / ny, BOX[2] / nz)
    kw = dict(bc_x=bcs[0], bc_y=bcs[1])
    u, v, w, p0 = _fields(nx, ny, nz, bcs[2], 21)
    u[:, :, -1] = 0.5  # wall faces (when there are walls): neither read nor changed
    v[:, -1, :] = -0.5
    du, dv, dw, dp = (torch.from_numpy(a.copy()).cuda() for a in (u, v, w, p0))
    alpha, beta = 2.0, 0.5
    print(f"[project] walls {nx}x{ny}x{nz} {bcs} {prec}", flush=True)
    with P.Plan(nx, ny, nz, *sp, bcs[2], prec, **kw) as plan:
        psi, st = plan.project(du, dv, dw, dp, alpha=alpha, beta=beta)
        torch.cuda.synchronize()
    assert st["status"] == 0
    u1, v1, w1, psi = (t.cpu().numpy() for t in (du, dv, dw, psi))
    f = orc.divergence(u, v, w, *sp, bcs[2], alpha=alpha, **kw)
    res, _ = orc.residual(f, psi, *sp, bcs[2], **kw)
    assert res <= (1e-12 if prec == "fp64" else 1e-10), res
    ur, vr, wr = orc.correct(u, v, w, psi, *sp, bcs[2], beta=beta, **kw)
    for a, b, name in ((u1, ur, "u"), (v1, vr, "v"), (w1, wr, "w")):
        assert np.abs(a - b).max() <= 1e-14 * max(np.abs(b).max(), 1.0), name
    if bcs[0] == NEU:
        assert np.array_equal(u1[:, :, -1], u[:, :, -1])
    if bcs[1] == NEU:
        assert np.array_equal(v1[:, -1, :], v[:, -1, :])
    assert np.array_equal(dp.cpu().numpy(), p0 + psi)
    d1 = orc.divergence(u1, v1, w1, *sp, bcs[2], **kw)
    d0 = orc.divergence(u, v, w, *sp, bcs[2], **kw)
    assert np.abs(d1).max() <= (1e-11 if prec == "fp64" else 1e-9) * np.abs(d0).max()


def test_project_cavity_full_size(orc):
    """512 x 512 x 256 cavity (solid walls on every axis): the oracle's
    residual of psi and the divergence of the corrected field, FP32 +
    refinement."""
    P = _gpu()
    nx, ny, nz = 512, 512, 256
    sp = (2.0 / nx, 2.0 / ny, 1.0 / nz)
    kw = dict(bc_x=NEU, bc_y=NEU)
    u, v, w = inputs.uniform_velocity(nx, ny, nz, NEU, 8)
    du, dv, dw = (torch.from_numpy(x).cuda() for x in (u, v, w))
    with P.Plan(nx, ny, nz, *sp, NEU, "fp32_refine", **kw) as plan:
        psi, st = plan.project(du, dv, dw, None)
        torch.cuda.synchronize()
    assert st["status"] == 0
    f = orc.divergence(u, v, w, *sp, NEU, **kw)
    res, _ = orc.residual(f, psi.cpu().numpy(), *sp, NEU, **kw)
    print(f"[project] cavity full size: residual {res:.2e} {st}", flush=True)
    assert res <= 1e-10
    d1 = orc.divergence(du.cpu().numpy(), dv.cpu().numpy(), dw.cpu().numpy(), *sp, NEU, **kw)
    assert np.abs(d1).max() <= 1e-9 * np.abs(f).max()


@pytest.mark.parametrize("first", ["project", "solve"])
def test_graph_plan_alternating_project_and_solve(first):
    """One graph-mode FP32 + refinement plan serves projections and plain
    solves in either order.  The projection takes its first solve eagerly
    and the segment-only graph, keeping the first iterate in FP64; a plain
    solve captures the first-round graph, which keeps it in its FP32 copy.
    Every call equals the host loop bitwise."""
    P = _gpu()
    nx, ny, nz, bc = 32, 24, 16, NEU
    sp = (BOX[0] / nx, BOX[1] / ny, BOX[2] / nz)
    u, v, w, _ = _fields(nx, ny, nz, bc, 21)
    f = torch.from_numpy(inputs.random_rhs(nx, ny, nz, seed=22)).cuda()
    print(f"[project] alternating, {first} first", flush=True)

    def calls(mode):
        res = []
        with P.Plan(nx, ny, nz, *sp, bc, "fp32_refine") as plan:
            plan.set_graph(mode)
            order = ["project", "solve"] if first == "project" else ["solve", "project"]
            for what in order * 2:
                if what == "project":
                    du, dv, dw = (torch.from_numpy(x.copy()).cuda() for x in (u, v, w))
                    psi, st = plan.project(du, dv, dw, None, alpha=2.0, beta=0.5)
                    out = [t.cpu().numpy() for t in (du, dv, dw, psi)]
                else:
                    p, st = plan.solve(f)
                    out = [p.cpu().numpy()]
                torch.cuda.synchronize()
                assert st["status"] == 0 and st["rel_residual"] <= 1e-10, (what, st)
                res.append((what, out, st))
        return res

    host, graph = calls("host"), calls("graph")
    for (w1, o1, s1), (w2, o2, s2) in zip(host, graph):
        assert w1 == w2 and s1 == s2, (w1, s1, s2)
        for a, b in zip(o1, o2):
            assert np.array_equal(a, b), w1


@pytest.mark.parametrize("mode", ["host", "device", "graph"])
def test_project_stopping_at_first_iterate(mode):
    """A projection whose refinement meets rtol at its first residual uses
    the first (FP32) iterate as psi, widened exactly: every field equals the
    plain FP32 projection bitwise, in every loop mode (the device loop widens
    inside its gated accumulating pass; under capture the projection keeps
    the iterate in FP64)."""
    P = _gpu()
    nx, ny, nz, bc = 32, 24, 16, NEU
    sp = (BOX[0] / nx, BOX[1] / ny, BOX[2] / nz)
    u, v, w, p0 = _fields(nx, ny, nz, bc, 31)
    print(f"[project] first iterate {mode}", flush=True)

    def run(prec, m, rtol):
        du, dv, dw, dp = (torch.from_numpy(x.copy()).cuda() for x in (u, v, w, p0))
        with P.Plan(nx, ny, nz, *sp, bc, prec, rtol=rtol) as plan:
            plan.set_graph(m)
            psi, st = plan.project(du, dv, dw, dp, alpha=2.0, beta=0.5)
            torch.cuda.synchronize()
        return [t.cpu().numpy() for t in (du, dv, dw, dp, psi)], st

    ref, _ = run("fp32", "host", 1e-10)
    out, st = run("fp32_refine", mode, 1e-3)
    assert st["status"] == 0 and st["iterations"] == 0, st
    for a, b in zip(ref, out):
        assert np.array_equal(a, b)
