"""GPU parity: the HIP solve (through the C ABI) against the FP64 CPU oracle.

Small grids (spanning several tiles, ragged tails, radix-3 lengths, length-1
axes) are compared element by element with the oracle, and so are the
full-size 512x512x256 and 256^3 workloads (the oracle solves them in seconds
to tens of seconds); full-size exact discrete eigenmodes, the relative
residual of the discrete equation (the oracle's FP64 stencil on the CPU) and
the zero-mean gauge are checked besides.

Tolerances (relative L2 unless stated):
  FP64          error vs oracle <= 1e-12
  FP32_REFINE   residual <= 1e-10 (the stopping rule) and error <= kappa(L) *
                residual; error <= 1e-10 when the residual is driven to 1e-12
  FP32          error vs oracle <= 2e-5 (single FP32 solve, no refinement)
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2204_08834_amd import inputs  # noqa: E402

NEU, PER = 1, 0


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_08834_amd import poisson
    poisson.lib()  # raises if the HIP library is missing: no fallback
    return poisson


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def gpu_solve(f, dx, dy, dz, bc, precision="fp64", rtol=1e-10, max_refine=8):
    P = _gpu()
    nz, ny, nx = f.shape
    print(f"[gpu_solve] {nx}x{ny}x{nz} bc={bc} {precision}", flush=True)
    rhs = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    with P.Plan(nx, ny, nz, dx, dy, dz, bc, precision, rtol, max_refine) as plan:
        out, st = plan.solve(rhs)
        torch.cuda.synchronize()
    return out.cpu().numpy(), st


SMALL = [
    # nx, ny, nz, Lx, Ly, Lz, bc
    (32, 32, 32, 1.0, 1.0, 1.0, NEU),      # the 32^3 workload's shape
    (16, 8, 12, 2.0, 1.0, 0.7, NEU),
    (64, 48, 20, 2.0, 2.0, 1.0, NEU),      # radix 3 in y, ragged z chunks
    (96, 96, 48, 2.0, 2.0, 1.0, NEU),      # radix 3 in x and y
    (24, 12, 33, 1.0, 1.0, 1.0, NEU),      # odd nz, last chunk ragged
    (8, 4, 300, 1.0, 1.0, 3.0, NEU),       # long z: many chunks
    (2, 1, 5, 1.0, 1.0, 1.0, NEU),         # nx=2, ny=1
    (4, 2, 1, 1.0, 1.0, 1.0, NEU),         # nz=1
    (32, 32, 32, 2 * math.pi, 2 * math.pi, 2 * math.pi, PER),
    (12, 6, 24, 1.0, 2.0, 3.0, PER),
    (64, 64, 64, 2 * math.pi, 2 * math.pi, 2 * math.pi, PER),
    (6, 3, 12, 1.0, 1.0, 1.0, PER),        # odd ny: unpaired ky columns
    (2, 1, 1, 1.0, 1.0, 1.0, PER),         # the smallest grid
    (128, 16, 8, 2.0, 1.0, 1.0, PER),
]


def _small_case(case, seed=5):
    nx, ny, nz, Lx, Ly, Lz, bc = case
    f = inputs.uniform_velocity_rhs(nx, ny, nz, Lx, Ly, Lz, bc, seed)
    return f, (Lx / nx, Ly / ny, Lz / nz), bc


@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}x{c[2]}_{'w' if c[6] else 'p'}"
                                             for c in SMALL])
def test_fp64_matches_oracle(orc, case):
    f, sp, bc = _small_case(case)
    p_ref = orc.solve(f, *sp, bc)
    p, st = gpu_solve(f, *sp, bc, "fp64")
    err = rel(p, p_ref)
    assert err <= 1e-12, err
    assert abs(p.mean()) <= 1e-13 * max(np.abs(p).max(), 1e-300)


def kappa(nx, ny, nz, dx, dy, dz, bc):
    """2-norm condition number of L on mean-free fields: |lam|max / |lam|min
    over the non-zero closed-form eigenvalues (L is symmetric)."""
    lo, hi = [], 0.0
    for n, h, per in ((nx, dx, True), (ny, dy, True), (nz, dz, bc == PER)):
        if n == 1:
            continue
        m = np.arange(n)
        ang = np.pi * m / n if per else np.pi * m / (2 * n)
        lam = 4 / h ** 2 * np.sin(ang) ** 2
        lo.append(lam[1] if per else lam[1])
        hi += lam.max()
    return hi / min(lo)


@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}x{c[2]}_{'w' if c[6] else 'p'}"
                                             for c in SMALL])
def test_fp32_refine_matches_oracle(orc, case):
    """Stopping rule: relative residual <= 1e-10.  The error against the oracle
    is then bounded by kappa(L) times the residual (checked, and printed)."""
    f, sp, bc = _small_case(case, seed=6)
    p_ref = orc.solve(f, *sp, bc)
    p, st = gpu_solve(f, *sp, bc, "fp32_refine", rtol=1e-10)
    res, _ = orc.residual(f, p, *sp, bc)
    err = rel(p, p_ref)
    k = kappa(case[0], case[1], case[2], *sp, bc)
    print(f"fp32+refine {case[:3]}: {st['iterations']} corrections, residual {res:.2e}, "
          f"error {err:.2e}, kappa {k:.1e}", flush=True)
    assert st["status"] == 0
    assert st["rel_residual"] <= 1e-10
    assert res <= 1e-10, res
    assert abs(res - st["rel_residual"]) <= 1e-12 + 0.05 * res
    assert err <= k * res * 1.01 + 1e-15, (err, k, res)


@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}x{c[2]}_{'w' if c[6] else 'p'}"
                                             for c in SMALL])
def test_fp32_refine_error_1e10(orc, case):
    """With the residual driven to 1e-12 the refined solution matches the
    FP64 oracle to 1e-10 relative error."""
    f, sp, bc = _small_case(case, seed=8)
    p_ref = orc.solve(f, *sp, bc)
    p, st = gpu_solve(f, *sp, bc, "fp32_refine", rtol=1e-12)
    err = rel(p, p_ref)
    assert st["status"] == 0, st
    assert err <= 1e-10, err


@pytest.mark.parametrize("case", SMALL[:4] + SMALL[8:11])
def test_fp32_single_solve(orc, case):
    f, sp, bc = _small_case(case, seed=7)
    p_ref = orc.solve(f, *sp, bc)
    p, st = gpu_solve(f, *sp, bc, "fp32")
    err = rel(p, p_ref)
    assert err <= 2e-5, err


@pytest.mark.parametrize("bc", [NEU, PER])
def test_mean_removed_and_reported(orc, bc):
    f, sp, _ = _small_case((16, 8, 12, 1.0, 1.0, 1.0, bc))
    for prec, tol in (("fp64", 1e-12), ("fp32_refine", 1e-9), ("fp32", 2e-5)):
        p0, _ = gpu_solve(f, *sp, bc, prec)
        p1, st = gpu_solve(f + 3.25, *sp, bc, prec)
        assert abs(st["rhs_mean"] - 3.25) <= 1e-9 * 3.25, (prec, st)
        assert rel(p1, p0) <= tol * 10, prec


def test_walls32_workload(orc):
    """The 32^3 walls workload: FP64 solve against the oracle at 1e-12."""
    prob = inputs.workload("walls32")
    p_ref = orc.solve(prob.f, *prob.spacings(), prob.bc_z)
    p, st = gpu_solve(prob.f, *prob.spacings(), prob.bc_z, "fp64")
    assert rel(p, p_ref) <= 1e-12
    res, _ = orc.residual(prob.f, p, *prob.spacings(), prob.bc_z)
    assert res <= 1e-13


def _eigen(nx, ny, nz, Lx, Ly, Lz, bc, a, b, c):
    dx, dy, dz = Lx / nx, Ly / ny, Lz / nz
    i = (np.arange(nx) + 0.5)[None, None, :]
    j = (np.arange(ny) + 0.5)[None, :, None]
    k = (np.arange(nz) + 0.5)[:, None, None]
    fx = np.cos(2 * np.pi * a * i / nx + 0.3)
    fy = np.cos(2 * np.pi * b * j / ny + 0.1)
    if bc == PER:
        fz = np.cos(2 * np.pi * c * k / nz + 0.2)
        lz = -4 / dz ** 2 * math.sin(math.pi * c / nz) ** 2
    else:
        fz = np.cos(np.pi * c * k / nz)
        lz = -4 / dz ** 2 * math.sin(math.pi * c / (2 * nz)) ** 2
    lam = -4 / dx ** 2 * math.sin(math.pi * a / nx) ** 2 - 4 / dy ** 2 * math.sin(
        math.pi * b / ny) ** 2 + lz
    return fx * fy * fz, lam, (dx, dy, dz)


@pytest.mark.parametrize("modes", [(1, 0, 0), (0, 0, 1), (3, 5, 7), (256, 256, 255), (0, 1, 0)])
def test_eigenmode_full_size_walls(modes):
    """512x512x256 walls: exact discrete eigenmodes (closed form) at full size."""
    a, b, c = modes
    f, lam, sp = _eigen(512, 512, 256, 2.0, 2.0, 1.0, NEU, a, b, c)
    for prec, tol in (("fp64", 1e-12), ("fp32_refine", 1e-10)):
        p, st = gpu_solve(f, *sp, NEU, prec)
        err = rel(p, f / lam)
        print(f"walls eigenmode {modes} {prec}: error {err:.2e} stats {st}", flush=True)
        assert err <= tol, (prec, err)


@pytest.mark.parametrize("modes", [(1, 0, 0), (0, 0, 1), (5, 9, 128), (128, 128, 128)])
def test_eigenmode_full_size_periodic(modes):
    a, b, c = modes
    f, lam, sp = _eigen(256, 256, 256, 2 * math.pi, 2 * math.pi, 2 * math.pi, PER, a, b, c)
    for prec, tol in (("fp64", 1e-12), ("fp32_refine", 1e-10)):
        p, st = gpu_solve(f, *sp, PER, prec)
        err = rel(p, f / lam)
        print(f"periodic eigenmode {modes} {prec}: error {err:.2e} stats {st}", flush=True)
        assert err <= tol, (prec, err)


@pytest.mark.parametrize("name", ["rb512", "hit256"])
def test_full_size_workload_matches_oracle(orc, name):
    """The full-size workloads in the benchmark's configuration (512x512x256
    walls with the two-layer right-hand side; 256^3 periodic with the
    spectral one), element by element against the oracle's solve of the
    whole grid: FP64 to 1e-12 relative L2 error, FP32 + refinement (stopping
    at a 1e-10 residual) to 1e-10; also the oracle residual of each field,
    the zero mean, and the largest pointwise error relative to max|p|."""
    prob = inputs.workload(name)
    sp = prob.spacings()
    print(f"[{name}] oracle solve of the whole grid", flush=True)
    ref = orc.solve(prob.f, *sp, prob.bc_z)
    scale = np.abs(ref).max()
    p64, st64 = gpu_solve(prob.f, *sp, prob.bc_z, "fp64")
    r64, _ = orc.residual(prob.f, p64, *sp, prob.bc_z)
    e64 = rel(p64, ref)
    m64 = float(np.abs(p64 - ref).max() / scale)
    print(f"{name}: fp64 residual {r64:.3e}, error vs oracle {e64:.3e} (max {m64:.3e})",
          flush=True)
    assert r64 <= 1e-12
    assert e64 <= 1e-12 and m64 <= 1e-12
    assert abs(p64.mean()) <= 1e-13 * np.abs(p64).max()
    del p64
    p32, st32 = gpu_solve(prob.f, *sp, prob.bc_z, "fp32_refine")
    r32, _ = orc.residual(prob.f, p32, *sp, prob.bc_z)
    e32 = rel(p32, ref)
    m32 = float(np.abs(p32 - ref).max() / scale)
    print(f"{name}: fp32+refine residual {r32:.3e} after {st32['iterations']} corrections, "
          f"error vs oracle {e32:.3e} (max {m32:.3e})", flush=True)
    assert st32["status"] == 0 and r32 <= 1e-10
    assert abs(r32 - st32["rel_residual"]) <= 1e-12 + 0.05 * r32
    assert e32 <= 1e-10 and m32 <= 1e-10
    assert abs(p32.mean()) <= 1e-13 * np.abs(p32).max()


def test_repeat_is_bitwise_deterministic():
    prob = inputs.scaled("rb512", 64, 64, 32)
    p1, _ = gpu_solve(prob.f, *prob.spacings(), prob.bc_z, "fp32_refine")
    p2, _ = gpu_solve(prob.f, *prob.spacings(), prob.bc_z, "fp32_refine")
    assert np.array_equal(p1, p2)


def test_nonfinite_rhs_reports_error():
    P = _gpu()
    f = inputs.random_rhs(16, 16, 16, 1)
    f[3, 4, 5] = np.nan
    rhs = torch.from_numpy(f).cuda()
    with P.Plan(16, 16, 16, 0.1, 0.1, 0.1, NEU, "fp32_refine") as plan:
        _, st = plan.solve(rhs, check=False)
    assert st["status"] == P.ERR_NONFINITE


def test_not_converged_reports_error():
    P = _gpu()
    prob = inputs.scaled("rb512", 32, 32, 16)
    rhs = torch.from_numpy(prob.f).cuda()
    with P.Plan(32, 32, 16, *prob.spacings(), NEU, "fp32_refine", rtol=1e-20,
                max_refine=1) as plan:
        out, st = plan.solve(rhs, check=False)
    assert st["status"] == P.ERR_NOT_CONVERGED
    assert st["iterations"] == 1
    assert np.isfinite(out.cpu().numpy()).all()


def test_stream_argument_and_aliasing_rejected():
    P = _gpu()
    f = torch.from_numpy(inputs.random_rhs(8, 8, 8, 2)).cuda()
    s = torch.cuda.Stream()
    with P.Plan(8, 8, 8, 1.0, 1.0, 1.0, NEU, "fp64", stream=s) as plan:
        with torch.cuda.stream(s):
            out, _ = plan.solve(f)
        s.synchronize()
        with pytest.raises(P.PoissonError):
            plan.solve(f, out=f)  # rhs and sol alias


def test_timing_reports_passes():
    P = _gpu()
    f = torch.from_numpy(inputs.random_rhs(64, 64, 32, 3)).cuda()
    with P.Plan(64, 64, 32, 1.0, 1.0, 1.0, NEU, "fp64") as plan:
        plan.set_timing(True)
        plan.solve(f)
        t = plan.timing()
    assert {"x_r2c_f64", "y_fwd_f64", "z_walls_f64", "y_inv_f64", "x_c2r_f64"} <= set(t)
    assert all(v["launches"] == 1 and v["total_ms"] > 0 for v in t.values())


# ---------------------------------------------------------------------------
# batched solves
# ---------------------------------------------------------------------------
def _batch_problems(probs, precision, rtol=1e-10):
    P = _gpu()
    specs = [dict(nx=p.nx, ny=p.ny, nz=p.nz, dx=p.dx, dy=p.dy, dz=p.dz, bc_z=p.bc_z)
             for p in probs]
    rhs = [torch.from_numpy(p.f).cuda() for p in probs]
    outs = [torch.empty_like(r) for r in rhs]
    bp = P.BatchPlan(specs, precision, rtol=rtol)
    rc, stats = bp.solve(rhs, outs, check=False)
    torch.cuda.synchronize()
    bp.close()
    return rc, stats, [o.cpu().numpy() for o in outs]


def _mixed_small():
    probs = [inputs.scaled("hit256", 32, 32, 32, seed=11), inputs.scaled("rb512", 48, 48, 24, seed=12),
             inputs.scaled("hit256", 32, 32, 32, seed=13), inputs.scaled("rb512", 64, 32, 20, seed=14),
             inputs.scaled("rb512", 48, 48, 24, seed=15)]
    return probs


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "fp32"])
def test_batch_equals_single_solves(precision):
    """A mixed-shape batch gives the fields of one plan per problem: bitwise
    for the plain solves; with refinement, the residual sums of a batched
    group are blocked by the group's size, so the mean of p (a constant
    removed from the field) may differ by rounding: within 1e-14 max|p|."""
    probs = _mixed_small()
    rc, stats, outs = _batch_problems(probs, precision)
    assert rc == 0, stats
    for prob, st, p in zip(probs, stats, outs):
        q, st1 = gpu_solve(prob.f, *prob.spacings(), prob.bc_z, precision)
        if precision == "fp32_refine":
            assert np.max(np.abs(p - q)) <= 1e-14 * np.max(np.abs(q)), (prob.name, rel(p, q))
        else:
            assert np.array_equal(p, q), (prob.name, rel(p, q))
        assert st["iterations"] == st1["iterations"]
        assert abs(st["rhs_mean"] - st1["rhs_mean"]) <= 1e-15


def test_batch_mixed64_workload(orc):
    """The 64-problem mixed batch (24 x 64^3 periodic, 24 x 96x96x48 walls,
    16 x 128x128x64 walls), FP32 + refinement to 1e-10: every problem converges;
    one problem of each shape is compared with the oracle."""
    probs = inputs.batch_mixed64()
    for p in probs:
        inputs.make_rhs(p)
    rc, stats, outs = _batch_problems(probs, "fp32_refine")
    assert rc == 0
    assert all(s["status"] == 0 and 0 <= s["rel_residual"] <= 1e-10 for s in stats)
    for idx in (0, 24, 48):
        prob = probs[idx]
        sp = prob.spacings()
        p_ref = orc.solve(prob.f, *sp, prob.bc_z)
        res, _ = orc.residual(prob.f, outs[idx], *sp, prob.bc_z)
        err = rel(outs[idx], p_ref)
        k = kappa(prob.nx, prob.ny, prob.nz, *sp, prob.bc_z)
        print(f"batch problem {idx} ({prob.name}): residual {res:.2e} error {err:.2e}", flush=True)
        assert res <= 1e-10 and err <= k * res * 1.01 + 1e-15


def test_batch_partial_convergence_and_errors():
    """Problems that stop early (converged or failing) leave the others running."""
    P = _gpu()
    probs = _mixed_small()
    probs[1].f = probs[1].f.copy()
    probs[1].f[0, 0, 0] = np.nan
    rc, stats, outs = _batch_problems(probs, "fp32_refine")
    assert rc == P.ERR_NONFINITE
    assert stats[1]["status"] == P.ERR_NONFINITE
    for i in (0, 2, 3, 4):
        assert stats[i]["status"] == 0 and stats[i]["rel_residual"] <= 1e-10


ZCASES = [(64, 48, 20), (24, 12, 33), (8, 4, 300), (32, 32, 130), (16, 8, 520)]


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_zwalls_tile_variants(orc, variant, monkeypatch):
    """Every tile variant of the wall-bounded z solve (the autotuner's
    choices) matches the oracle: FP64 to 1e-12, FP32 + refinement to a
    1e-10 residual."""
    monkeypatch.setenv("POISSON_ZWALLS_VARIANT", str(variant))
    for nx, ny, nz in ZCASES:
        f = inputs.uniform_velocity_rhs(nx, ny, nz, 2.0, 2.0, 1.0, NEU, 7)
        sp = (2.0 / nx, 2.0 / ny, 1.0 / nz)
        p_ref = orc.solve(f, *sp, NEU)
        p, _ = gpu_solve(f, *sp, NEU, "fp64")
        assert rel(p, p_ref) <= 1e-12, (variant, nx, ny, nz)
        q, st = gpu_solve(f, *sp, NEU, "fp32_refine")
        res, _ = orc.residual(f, q, *sp, NEU)
        assert st["status"] == 0 and res <= 1e-10, (variant, nx, ny, nz, res)


def test_batch_rejects_overlap_across_problems():
    """A batch refuses a solution that shares memory with another problem's
    solution or with any right-hand side, whatever the two problems' sizes:
    a small problem's output placed in the tail of a large problem's output,
    or on another problem's right-hand side.  The check runs before any
    launch; every pointer lies inside one allocation."""
    P = _gpu()
    import ctypes
    big, small = (32, 32, 32), (8, 8, 8)
    nb, ns = 32 * 32 * 32, 8 * 8 * 8
    specs = [dict(nx=big[0], ny=big[1], nz=big[2], dx=1.0, dy=1.0, dz=1.0, bc_z=NEU),
             dict(nx=small[0], ny=small[1], nz=small[2], dx=1.0, dy=1.0, dz=1.0, bc_z=NEU)]
    arena = torch.zeros(5 * nb, dtype=torch.float64, device="cuda")
    base, es = arena.data_ptr(), arena.element_size()
    r0, r1, s0 = base, base + nb * es, base + 2 * nb * es
    bp = P.BatchPlan(specs, "fp64")
    L = P.lib()
    V = ctypes.c_void_p * 2

    def call(rhs, sol):
        return L.poisson_batch_solve(bp._h, V(*rhs), V(*sol), None)

    tail = s0 + (nb - ns // 2) * es          # small output starts inside the big one's tail
    assert call([r0, r1], [s0, tail]) == P.ERR_INVALID_ARG
    s1 = s0 + nb * es                        # big output starts inside the small one
    assert call([r0, r1], [s1 + (ns // 2) * es, s1]) == P.ERR_INVALID_ARG
    assert call([r0, r1], [s0, r0 + 16 * es]) == P.ERR_INVALID_ARG   # sol[1] on rhs[0]
    assert call([r0, r1], [r1, s0]) == P.ERR_INVALID_ARG             # sol[0] on rhs[1]
    assert call([r0, r0], [s0, s0 + nb * es]) == P.OK                 # shared rhs is fine
    torch.cuda.synchronize()
    bp.close()
