"""GPU: launch variants and the plan-time autotuner.

Every variant the autotuner may pick (y tile width and radix order, block
order; the z-solve tiles are covered in test_gpu_parity.py) must solve to the
oracle's tolerance; the block order does not change the arithmetic at all
(bitwise equal fields).  The tuner records its choices, later plans of the
same shape reuse them, and POISSON_TUNE_CACHE persists them.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2204_08834_amd import inputs  # noqa: E402

NEU, PER = 1, 0
YCASES = [(64, 64, 16, NEU), (32, 96, 8, PER), (16, 128, 12, NEU), (8, 512, 6, PER)]


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_08834_amd import poisson
    poisson.lib()  # raises if the HIP library is missing: no fallback
    return poisson


def _solve(f, sp, bc, precision, tune=False):
    P = _gpu()
    nz, ny, nx = f.shape
    rhs = torch.from_numpy(f).cuda()
    with P.Plan(nx, ny, nz, *sp, bc, precision) as plan:
        if tune:
            plan.autotune()
        out, st = plan.solve(rhs)
        desc = plan.describe()
        torch.cuda.synchronize()
    return out.cpu().numpy(), st, desc


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_y_variants_match_oracle(orc, variant, monkeypatch):
    monkeypatch.setenv("POISSON_Y_VARIANT", str(variant))
    for nx, ny, nz, bc in YCASES:
        L = (2.0, 2.0, 1.0) if bc == NEU else (1.0, 3.0, 2.0)
        f = inputs.uniform_velocity_rhs(nx, ny, nz, *L, bc, 9)
        sp = (L[0] / nx, L[1] / ny, L[2] / nz)
        p_ref = orc.solve(f, *sp, bc)
        p, _, desc = _solve(f, sp, bc, "fp64")
        assert f"y_tile={variant}" in desc
        assert rel(p, p_ref) <= 1e-12, (variant, nx, ny, nz, bc)
        q, st, _ = _solve(f, sp, bc, "fp32_refine")
        assert st["status"] == 0 and st["rel_residual"] <= 1e-10


def test_block_order_is_bitwise_neutral(monkeypatch):
    prob = inputs.scaled("rb512", 128, 128, 64, seed=61)
    sp = prob.spacings()
    a, _, da = _solve(prob.f, sp, NEU, "fp32_refine")
    monkeypatch.setenv("POISSON_BLOCK_ORDER", "forward")
    b, _, db = _solve(prob.f, sp, NEU, "fp32_refine")
    assert "reverse=1" in da and "reverse=0" in db
    assert np.array_equal(a, b)


def test_autotune_choices_solve_and_are_reused(orc, tmp_path, monkeypatch):
    P = _gpu()
    monkeypatch.delenv("POISSON_ZWALLS_VARIANT", raising=False)
    monkeypatch.delenv("POISSON_Y_VARIANT", raising=False)
    monkeypatch.delenv("POISSON_BLOCK_ORDER", raising=False)
    monkeypatch.setenv("POISSON_TUNE_CACHE", str(tmp_path / "tune.txt"))
    for name, shape in (("rb512", (96, 96, 48)), ("hit256", (64, 64, 64))):
        prob = inputs.scaled(name, *shape, seed=62)
        sp = prob.spacings()
        p_ref = orc.solve(prob.f, *sp, prob.bc_z)
        p, st, desc = _solve(prob.f, sp, prob.bc_z, "fp64", tune=True)
        print(desc, flush=True)
        assert "tuned" in desc
        assert rel(p, p_ref) <= 1e-12
        # a later plan of the same shape starts from the cached choice
        _, _, desc2 = _solve(prob.f, sp, prob.bc_z, "fp64")
        assert desc2 == desc
        q, st, desc3 = _solve(prob.f, sp, prob.bc_z, "fp32_refine", tune=True)
        assert "tuned" in desc3 and st["rel_residual"] <= 1e-10
    text = (tmp_path / "tune.txt").read_text()
    assert "f64 96 96 48 001" in text and "f32 64 64 64 000" in text


def test_stretched_grids_tune_apart(orc, tmp_path, monkeypatch):
    """A stretched-z grid runs other z-solve kernels than the uniform grid of
    the same shape: the tuner keeps a separate entry for it (and both solve
    to the oracle)."""
    P = _gpu()
    monkeypatch.setenv("POISSON_TUNE_CACHE", str(tmp_path / "tune.txt"))
    for v in ("POISSON_ZWALLS_VARIANT", "POISSON_Y_VARIANT", "POISSON_BLOCK_ORDER"):
        monkeypatch.delenv(v, raising=False)
    nx, ny, nz = 48, 48, 40
    sp = (2.0 / nx, 1.5 / ny)
    f = inputs.random_rhs(nx, ny, nz, seed=91, zero_mean=False)
    h = inputs.tanh_cells(nz, 1.0, 2.0)
    for cells in (None, h):
        ref = orc.solve(f, *sp, 1.0 / nz, NEU, dz_cells=cells)
        with P.Plan(nx, ny, nz, *sp, 1.0 / nz, NEU, "fp64", dz_cells=cells) as plan:
            plan.autotune()
            out, st = plan.solve(torch.from_numpy(f).cuda())
            assert "tuned" in plan.describe()
        # (the stretched operator's conditioning is tested in test_gpu_stretched.py)
        assert st["status"] == 0 and rel(out.cpu().numpy(), ref) <= (1e-12 if cells is None else 1e-10)
    text = (tmp_path / "tune.txt").read_text()
    assert "f64 48 48 40 001 " in text and "f64 48 48 40 001s " in text


def test_batch_autotune_and_describe():
    P = _gpu()
    probs = [inputs.scaled("hit256", 32, 32, 32, seed=71), inputs.scaled("rb512", 64, 64, 32, seed=72),
             inputs.scaled("hit256", 32, 32, 32, seed=73)]
    specs = [dict(nx=p.nx, ny=p.ny, nz=p.nz, dx=p.dx, dy=p.dy, dz=p.dz, bc_z=p.bc_z) for p in probs]
    rhs = [torch.from_numpy(p.f).cuda() for p in probs]
    outs = [torch.empty_like(r) for r in rhs]
    bp = P.BatchPlan(specs, "fp32_refine")
    bp.autotune()
    d = bp.describe()
    print(d, flush=True)
    assert d.count("\n") == 3 and "problems=2" in d and "problems=1" in d
    # the autotuner also chose the batch schedule of each loop driver
    assert d.startswith("schedule=") and "host loop:" in d and "device loops:" in d
    rc, stats = bp.solve(rhs, outs)
    assert rc == 0 and all(s["rel_residual"] <= 1e-10 for s in stats)
    bp.close()


@pytest.mark.parametrize("planes,check", [(4, 4), (8, 8), (16, 16), (5, 3), (43, 22), (7, 40)])
def test_march_depths(planes, check, monkeypatch):
    """Every plane-range depth of the residual passes (4, 8, 16: halved for
    small grids; others exact, uneven last range included): converged solves,
    and the device-side loop (whose sum counts the march grid) equal to the
    host loop bitwise."""
    P = _gpu()
    monkeypatch.setenv("POISSON_MARCH_PLANES", str(planes))
    monkeypatch.setenv("POISSON_CHECK_PLANES", str(check))
    for name, shape in (("rb512", (128, 128, 96)), ("hit256", (64, 64, 64)), ("rb512", (96, 48, 36))):
        prob = inputs.scaled(name, *shape, seed=81)
        sp = prob.spacings()
        rhs = torch.from_numpy(prob.f).cuda()
        res = {}
        for mode in ("host", "graph"):
            with P.Plan(prob.nx, prob.ny, prob.nz, *sp, prob.bc_z, "fp32_refine") as plan:
                plan.set_graph(mode)
                out, st = plan.solve(rhs)
                # the plan's depth settings (an exact depth beyond the grid
                # runs as one range of all planes)
                assert f"march_planes={planes} check_planes={check} " in plan.describe()
                torch.cuda.synchronize()
            res[mode] = (out.cpu().numpy(), st)
        assert res["host"][1]["status"] == 0 and res["host"][1]["rel_residual"] <= 1e-10
        assert np.array_equal(res["host"][0], res["graph"][0])
        assert res["host"][1] == res["graph"][1]
