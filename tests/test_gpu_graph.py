"""GPU: the device-side refinement loop of poisson_plan_set_graph (captured
hipGraph, mode "graph"; the same launch sequence issued eagerly, mode
"device") against the host-driven loop (mode "host").

For one problem the device loop takes exactly the host loop's decisions
(same kernels, same reduction order), so fields and statistics agree
bitwise; a batch agrees as well, since every per-problem decision depends
on that problem's residual only.  Graph replays are checked one by one,
with the program's own eager work and synchronisations in between, against
the eager result.
"""
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


def _solve(prob, precision, mode, rtol=1e-10, max_refine=8):
    P = _gpu()
    print(f"[graph] {prob.nx}x{prob.ny}x{prob.nz} bc={prob.bc_z} {precision} {mode}", flush=True)
    rhs = torch.from_numpy(prob.f).cuda()
    with P.Plan(prob.nx, prob.ny, prob.nz, *prob.spacings(), prob.bc_z, precision, rtol,
                max_refine) as plan:
        plan.set_graph(mode)
        out, st = plan.solve(rhs, check=False)
        torch.cuda.synchronize()
    return out.cpu().numpy(), st


CASES = [("rb512", 64, 64, 32, NEU), ("hit256", 32, 32, 32, PER), ("rb512", 48, 24, 20, NEU)]


@pytest.mark.parametrize("mode", ["device", "graph"])
@pytest.mark.parametrize("precision", ["fp32_refine", "fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}_{c[1]}x{c[2]}x{c[3]}" for c in CASES])
def test_single_problem_matches_host_loop(case, precision, mode):
    name, nx, ny, nz, _ = case
    prob = inputs.scaled(name, nx, ny, nz)
    p_host, st_host = _solve(prob, precision, "host")
    p_dev, st_dev = _solve(prob, precision, mode)
    assert st_dev["status"] == st_host["status"] == 0
    assert np.array_equal(p_dev, p_host)
    assert st_dev["iterations"] == st_host["iterations"]
    assert st_dev["rel_residual"] == st_host["rel_residual"]
    assert st_dev["rhs_mean"] == st_host["rhs_mean"]


@pytest.mark.parametrize("rtol,max_refine", [(1e-20, 3), (1e-14, 8), (1e-13, 1)])
def test_stopping_rules_match_host_loop(rtol, max_refine):
    """Not converged (max_refine or stall) and several corrections: the
    segment-only graph is relaunched while a problem runs."""
    prob = inputs.scaled("rb512", 64, 64, 32, seed=21)
    p_host, st_host = _solve(prob, "fp32_refine", "host", rtol, max_refine)
    p_dev, st_dev = _solve(prob, "fp32_refine", "graph", rtol, max_refine)
    print(f"host {st_host} graph {st_dev}", flush=True)
    assert st_dev["status"] == st_host["status"]
    assert st_dev["iterations"] == st_host["iterations"]
    assert st_dev["rel_residual"] == st_host["rel_residual"]
    assert np.array_equal(p_dev, p_host)


def test_graph_replays_with_new_arguments():
    """One captured plan solving several right-hand sides into different
    output tensors, with eager work and synchronisations in between: every
    replay equals the host-driven solve of the same input."""
    P = _gpu()
    shape = (32, 48, 64)
    probs = [inputs.scaled("rb512", 64, 48, 32, seed=s) for s in (31, 32, 33)]
    refs = [_solve(p, "fp32_refine", "host")[0] for p in probs]
    dx, dy, dz = probs[0].spacings()
    with P.Plan(64, 48, 32, dx, dy, dz, NEU, "fp32_refine") as plan:
        plan.set_graph("graph")
        for it, k in enumerate([0, 1, 2, 1, 0]):
            rhs = torch.from_numpy(probs[k].f).cuda()
            out = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()  # eager work
            _, st = plan.solve(rhs, out)
            torch.cuda.synchronize()
            print(f"replay {it} problem {k}: {st}", flush=True)
            assert np.isfinite(junk.item())
            assert st["status"] == 0 and st["rel_residual"] <= 1e-10
            assert np.array_equal(out.cpu().numpy(), refs[k]), it


def _batch(probs, precision, mode):
    P = _gpu()
    specs = [dict(nx=p.nx, ny=p.ny, nz=p.nz, dx=p.dx, dy=p.dy, dz=p.dz, bc_z=p.bc_z)
             for p in probs]
    rhs = [torch.from_numpy(p.f).cuda() for p in probs]
    outs = [torch.empty_like(r) for r in rhs]
    bp = P.BatchPlan(specs, precision)
    bp.set_graph(mode)
    rc, stats = bp.solve(rhs, outs, check=False)
    torch.cuda.synchronize()
    bp.close()
    return rc, stats, [o.cpu().numpy() for o in outs]


def _mixed():
    return [inputs.scaled("hit256", 32, 32, 32, seed=41), inputs.scaled("rb512", 48, 48, 24, seed=42),
            inputs.scaled("hit256", 32, 32, 32, seed=43), inputs.scaled("rb512", 64, 32, 20, seed=44),
            inputs.scaled("rb512", 48, 48, 24, seed=45)]


@pytest.mark.parametrize("mode", ["device", "graph"])
def test_batch_matches_host_loop(mode):
    probs = _mixed()
    rc_h, st_h, p_h = _batch(probs, "fp32_refine", "host")
    rc_d, st_d, p_d = _batch(probs, "fp32_refine", mode)
    assert rc_h == rc_d == 0
    for a, b, sa, sb in zip(p_h, p_d, st_h, st_d):
        assert np.array_equal(a, b)
        assert sa == sb


def test_graph_batch_with_failing_problem():
    P = _gpu()
    probs = _mixed()
    probs[2].f = probs[2].f.copy()
    probs[2].f[1, 2, 3] = np.inf
    rc, stats, outs = _batch(probs, "fp32_refine", "graph")
    assert rc == P.ERR_NONFINITE
    assert stats[2]["status"] == P.ERR_NONFINITE
    rc_h, st_h, p_h = _batch(probs, "fp32_refine", "host")
    for i in (0, 1, 3, 4):
        assert stats[i]["status"] == 0 and stats[i]["rel_residual"] <= 1e-10
        assert np.array_equal(outs[i], p_h[i])


def test_mode_switch_and_invalid_mode():
    P = _gpu()
    prob = inputs.scaled("rb512", 32, 32, 16, seed=51)
    rhs = torch.from_numpy(prob.f).cuda()
    with P.Plan(32, 32, 16, *prob.spacings(), NEU, "fp32_refine") as plan:
        a, _ = plan.solve(rhs)
        plan.set_graph("graph")
        b, _ = plan.solve(rhs)
        plan.set_graph("host")
        c, _ = plan.solve(rhs)
        with pytest.raises(P.PoissonError):
            plan.set_graph(3)
        torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_batch_rechecks_changed_arguments():
    """Calls with the same tensors as the previous call skip the per-tensor
    checks; a tensor replaced in the list, or changed in place, is checked
    again, and the results of the repeated calls agree."""
    P = _gpu()
    probs = _mixed()[:2]
    specs = [dict(nx=p.nx, ny=p.ny, nz=p.nz, dx=p.dx, dy=p.dy, dz=p.dz, bc_z=p.bc_z)
             for p in probs]
    rhs = [torch.from_numpy(p.f).cuda() for p in probs]
    outs = [torch.empty_like(r) for r in rhs]
    bp = P.BatchPlan(specs, "fp64")
    try:
        bp.solve(rhs, outs)
        first = [o.clone() for o in outs]
        bp.solve(rhs, outs)
        assert all(torch.equal(a, b) for a, b in zip(first, outs))
        good = outs[1]
        bad = [torch.empty(3, 3, 3, dtype=torch.float64, device="cuda"),  # shape
               torch.empty_like(good, dtype=torch.float32),  # dtype
               torch.empty_like(good).transpose(0, 2),  # not contiguous
               torch.empty_like(good, device="cpu")]  # not on the GPU
        for t in bad:
            with pytest.raises((ValueError, TypeError)):
                bp.solve(rhs, [outs[0], t])
        # the same tensor object, changed in place: shape, then dtype alone
        keep = good.data
        good.data = torch.empty(3, 3, 3, dtype=torch.float64, device="cuda")
        with pytest.raises(ValueError):
            bp.solve(rhs, outs)
        good.data = keep.view(torch.int64)
        with pytest.raises(ValueError):
            bp.solve(rhs, outs)
        good.data = keep
        bp.solve(rhs, outs)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(first, outs))
    finally:
        bp.close()


@pytest.mark.parametrize("mode", ["host", "device", "graph"])
@pytest.mark.parametrize("bcs", [(PER, PER, NEU), (NEU, NEU, NEU)])
def test_stop_before_any_correction_returns_first_iterate(mode, bcs):
    """The refinement keeps its first iterate in an exact FP32 copy.  A
    problem whose first residual already meets rtol stops there: the
    solution is that iterate, widened exactly, i.e. bitwise the plain FP32
    solve (same kernels, same tuned variants), whatever the output array
    held before."""
    P = _gpu()
    prob = inputs.scaled("rb512", 48, 24, 20, seed=61)
    sp = prob.spacings()
    rhs = torch.from_numpy(prob.f).cuda()
    print(f"[graph] first iterate {mode} {bcs}", flush=True)
    with P.Plan(48, 24, 20, *sp, bcs[2], "fp32", bc_x=bcs[0], bc_y=bcs[1]) as plan:
        ref, _ = plan.solve(rhs)
    with P.Plan(48, 24, 20, *sp, bcs[2], "fp32_refine", rtol=1e-3, bc_x=bcs[0],
                bc_y=bcs[1]) as plan:
        plan.set_graph(mode)
        for _ in range(2):
            out = torch.full_like(rhs, float("nan"))
            out, st = plan.solve(rhs, out)
            torch.cuda.synchronize()
            assert st["status"] == 0 and st["iterations"] == 0, st
            assert 0 < st["rel_residual"] <= 1e-3
            assert torch.equal(out, ref)


@pytest.mark.parametrize("mode", ["host", "device", "graph"])
def test_batch_with_a_zero_problem(mode):
    """A zero right-hand side converges at its first residual (the zero
    iterate) while the others of its group go on: its solution is zero and
    the others equal the host loop's bitwise."""
    probs = _mixed()
    probs[1].f = np.zeros_like(probs[1].f)
    rc_h, st_h, p_h = _batch(probs, "fp32_refine", "host")
    rc, st, outs = _batch(probs, "fp32_refine", mode)
    assert rc == rc_h == 0
    assert st[1]["iterations"] == 0 and st[1]["status"] == 0
    assert not np.any(outs[1])
    for a, b, sa, sb in zip(p_h, outs, st_h, st):
        assert np.array_equal(a, b)
        assert sa == sb


@pytest.mark.parametrize("mode", ["device", "graph"])
def test_loops_on_a_caller_stream(mode):
    """The device-side loops issue to the plan's stream (eager launches and
    graph launches alike; graphs are captured on a stream of the plan's
    own): on a non-default caller stream, repeated solves with a right-hand
    side rewritten on that stream in between equal the host loop's
    bitwise."""
    P = _gpu()
    prob = inputs.scaled("rb512", 64, 48, 40, seed=141)
    base = torch.from_numpy(prob.f).cuda()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    res = {}
    for m in ("host", mode):
        with torch.cuda.stream(s):
            rhs = torch.empty_like(base)
            out = torch.empty_like(base)
            got = []
            with P.Plan(prob.nx, prob.ny, prob.nz, *prob.spacings(), prob.bc_z, "fp32_refine",
                        stream=s) as plan:
                plan.set_graph(m)
                for scale in (1.0, -2.0, 0.5):
                    rhs.copy_(base).mul_(scale)  # queued on s before the solve
                    _, st = plan.solve(rhs, out)
                    got.append((out.clone(), st))
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        res[m] = [(o.cpu().numpy(), st) for o, st in got]
    for (a, sa), (b, sb) in zip(res["host"], res[mode]):
        assert sa["status"] == 0 and sa["rel_residual"] <= 1e-10
        assert np.array_equal(a, b) and sa == sb
