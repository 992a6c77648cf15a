"""Work-list schedule of batched solves: one launch per pass serves the
problems of every shape of a batch (the default for batches of several
shapes).  Checked against the per-group schedule (one launch per shape group
and pass, POISSON_BATCH_SCHEDULE=groups) and against single-problem plans:
bitwise for the plain FP64 and FP32 solves; with refinement the sum of f is
blocked differently by the list's forward x pass, so the fields agree to the
rounding of the removed mean (1e-14 of max|p|).  The device-side loops
(eager and captured graph) equal the host loop.  One problem of each shape
is compared with the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2204_08834_amd import inputs  # noqa: E402

PER, NEU, DIR = 0, 1, 2


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_08834_amd import poisson
    poisson.lib()  # raises if the HIP library is missing: no fallback
    return poisson


def _mixed():
    # three shapes, periodic and wall-bounded z, several problems each,
    # lengths inside and outside the list kernels' classes (nx = 384 has
    # M = 192: its own launch inside the list schedule)
    probs = []
    for sd in range(3):
        probs.append(inputs.scaled("hit256", 32, 32, 32, seed=100 + sd))
    for sd in range(2):
        probs.append(inputs.scaled("rb512", 48, 48, 24, seed=110 + sd))
    for sd in range(2):
        probs.append(inputs.scaled("rb512", 64, 32, 100, seed=120 + sd))
    probs.append(inputs.scaled("rb512", 384, 8, 6, seed=130))
    return probs


def _solve_batch(P, probs, precision, mode="host", schedule=None, monkeypatch=None,
                 timing=False):
    if schedule is not None:
        monkeypatch.setenv("POISSON_BATCH_SCHEDULE", schedule)
    specs = [dict(nx=p.nx, ny=p.ny, nz=p.nz, dx=p.dx, dy=p.dy, dz=p.dz, bc_z=p.bc_z)
             for p in probs]
    rhs = [torch.from_numpy(p.f).cuda() for p in probs]
    outs = [torch.full_like(r, float("nan")) for r in rhs]
    bp = P.BatchPlan(specs, precision)
    if schedule is not None:
        monkeypatch.delenv("POISSON_BATCH_SCHEDULE")
    bp.set_graph(mode)
    if timing:
        bp.set_timing(True)
    rc, st = bp.solve(rhs, outs, check=False)
    torch.cuda.synchronize()
    t = bp.timing() if timing else None
    desc = bp.describe()
    bp.close()
    return rc, st, [o.cpu().numpy() for o in outs], t, desc


def _same(a, b, precision):
    if precision == "fp32_refine":
        return np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))
    return np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "fp32"])
def test_list_equals_group_schedule(precision, monkeypatch):
    P = _gpu()
    probs = _mixed()
    print(f"[batchlist] {precision}", flush=True)
    rc1, st1, o1, _, d1 = _solve_batch(P, probs, precision)
    rc2, st2, o2, _, d2 = _solve_batch(P, probs, precision, schedule="groups",
                                       monkeypatch=monkeypatch)
    assert "schedule=list" in d1 and "schedule=groups" in d2
    assert rc1 == 0 and rc2 == 0, (st1, st2)
    for i, (a, b) in enumerate(zip(o1, o2)):
        assert np.isfinite(a).all(), i
        assert _same(a, b, precision), (i, probs[i].name)
        assert st1[i]["iterations"] == st2[i]["iterations"]
        assert abs(st1[i]["rhs_mean"] - st2[i]["rhs_mean"]) <= 1e-15


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_list_equals_single_solves(orc, precision):
    P = _gpu()
    probs = _mixed()
    rc, st, outs, _, _ = _solve_batch(P, probs, precision)
    assert rc == 0, st
    seen = set()
    for prob, s, p in zip(probs, st, outs):
        with P.Plan(prob.nx, prob.ny, prob.nz, *prob.spacings(), prob.bc_z, precision) as plan:
            q, s1 = plan.solve(torch.from_numpy(prob.f).cuda())
            torch.cuda.synchronize()
        q = q.cpu().numpy()
        assert _same(p, q, precision), prob.name
        assert s["iterations"] == s1["iterations"]
        shape = (prob.nx, prob.ny, prob.nz)
        if shape not in seen:
            seen.add(shape)
            ref = orc.solve(prob.f, *prob.spacings(), prob.bc_z)
            err = np.linalg.norm(p - ref) / np.linalg.norm(ref)
            if precision == "fp64":
                assert err <= 1e-12, (prob.name, err)
            else:
                res, _ = orc.residual(prob.f, p, *prob.spacings(), prob.bc_z)
                assert s["status"] == 0 and res <= 1e-10, (prob.name, res)


@pytest.mark.parametrize("mode", ["device", "graph"])
def test_list_device_loop_equals_host_loop(mode):
    P = _gpu()
    probs = _mixed()
    rc1, st1, o1, _, _ = _solve_batch(P, probs, "fp32_refine", mode="host")
    rc2, st2, o2, _, _ = _solve_batch(P, probs, "fp32_refine", mode=mode)
    assert rc1 == 0 and rc2 == 0
    for i, (a, b) in enumerate(zip(o1, o2)):
        assert np.array_equal(a, b), i
        assert st1[i]["iterations"] == st2[i]["iterations"]
        assert st1[i]["rel_residual"] == st2[i]["rel_residual"]


def test_list_failing_problem_leaves_others_running():
    P = _gpu()
    probs = _mixed()
    probs[3].f = probs[3].f.copy()
    probs[3].f[1, 2, 3] = np.inf
    for mode in ("host", "device"):
        rc, st, outs, _, _ = _solve_batch(P, probs, "fp32_refine", mode=mode)
        assert rc == P.ERR_NONFINITE
        assert st[3]["status"] == P.ERR_NONFINITE
        for i in range(len(probs)):
            if i != 3:
                assert st[i]["status"] == 0 and st[i]["rel_residual"] <= 1e-10, (mode, i)


def test_list_one_launch_per_pass():
    """In the list schedule every transform pass of a solve is one launch for
    all shapes whose lengths have list classes (here: every shape but the
    one with nx = 384, which gets its own launches besides)."""
    P = _gpu()
    probs = [p for p in _mixed() if p.nx != 384]
    rc, st, _, t, _ = _solve_batch(P, probs, "fp64", timing=True)
    assert rc == 0
    for name in ("x_r2c_f64", "y_fwd_f64", "z_f64", "y_inv_f64", "x_c2r_f64"):
        assert t[name]["launches"] == 1, (name, t)


def test_autotuned_schedule_gives_the_same_fields():
    """The autotuner picks the schedule per loop driver; whatever it picks,
    the fields equal the per-group schedule's (within the refinement's
    rounding of the removed mean)."""
    P = _gpu()
    probs = _mixed()
    specs = [dict(nx=p.nx, ny=p.ny, nz=p.nz, dx=p.dx, dy=p.dy, dz=p.dz, bc_z=p.bc_z)
             for p in probs]
    rhs = [torch.from_numpy(p.f).cuda() for p in probs]
    ref = _solve_batch(P, probs, "fp32_refine")[2]
    bp = P.BatchPlan(specs, "fp32_refine")
    bp.autotune()
    d = bp.describe()
    assert "host loop:" in d and "device loops:" in d
    for mode in ("host", "device", "graph"):
        outs = [torch.empty_like(r) for r in rhs]
        bp.set_graph(mode)
        rc, st = bp.solve(rhs, outs)
        torch.cuda.synchronize()
        assert rc == 0
        for i, o in enumerate(outs):
            assert _same(o.cpu().numpy(), ref[i], "fp32_refine"), (mode, i)
    bp.close()
