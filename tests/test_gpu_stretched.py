"""GPU parity of the z-stretched solve (walls in z, cells of thickness h_k)
against the oracle's stretched solve (pinned in test_oracle_stretched.py):
FP64 to 1e-12 (or the conditioning bound) with the residual at the
oracle's own level, FP32 + refinement to an oracle residual of 1e-10 (or ten
times what FP64 reaches) with the error bounded by kappa times the two
residuals, single FP32 solves by conditioning; the volume-weighted mean
reported; equal thicknesses equal to
the uniform path; batches and the allocation-free entry point equal the
plan's solve."""
import ctypes
import math

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


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def kappa(nx, ny, dx, dy, h, bcs):
    """Rough condition number: largest over smallest operator scale."""
    hmin = h.min()
    top = 4 / dx ** 2 + 4 / dy ** 2 + 4 / hmin ** 2
    L = h.sum()
    low = (math.pi / L) ** 2
    if bcs[0] != PER:
        low = min(low, (math.pi / (2 * nx * dx)) ** 2)
    return top / low


def gpu_solve(P, f, sp, h, bcs, prec, rtol=1e-10):
    nz, ny, nx = f.shape
    with P.Plan(nx, ny, nz, sp[0], sp[1], 1.0 / nz, bcs[2], prec, rtol=rtol, bc_x=bcs[0],
                bc_y=bcs[1], dz_cells=h) as plan:
        out, st = plan.solve(torch.from_numpy(f).cuda(), check=False)
        torch.cuda.synchronize()
    return out.cpu().numpy(), st


CASES = [((32, 32, 32), 2.0), ((64, 48, 20), 1.5), ((16, 8, 300), 2.5), ((8, 4, 1), 0.0),
         ((24, 12, 33), 3.0), ((2, 1, 70), 2.0), ((96, 64, 130), 2.2), ((4, 6, 1500), 1.8)]
BCS = [(PER, PER, NEU), (PER, PER, DIR), (NEU, PER, NEU), (PER, DIR, NEU), (NEU, NEU, NEU),
       (DIR, NEU, DIR)]


@pytest.mark.parametrize("bcs", BCS, ids=["".join("PND"[b] for b in c) for c in BCS])
def test_stretched_matches_oracle(orc, bcs):
    P = _gpu()
    for (nx, ny, nz), beta in CASES:
        h = inputs.tanh_cells(nz, 1.0, beta)
        sp = (2.0 / nx, 1.5 / ny)
        f = inputs.random_rhs(nx, ny, nz, seed=nx + 3 * nz, zero_mean=False) + 0.2
        ref, info = orc.solve(f, *sp, None, bcs[2], bc_x=bcs[0], bc_y=bcs[1], dz_cells=h,
                              return_info=True)
        res_ref, _ = orc.residual(f, ref, *sp, None, bcs[2], bc_x=bcs[0], bc_y=bcs[1], dz_cells=h)
        k = kappa(nx, ny, *sp, h, bcs)
        # the refinement is asked for what FP64 can deliver on this operator
        rtol = max(1e-10, 10 * res_ref)
        for prec in ("fp64", "fp32_refine", "fp32"):
            print(f"[stretched] {nx}x{ny}x{nz} beta {beta} {bcs} {prec}", flush=True)
            p, st = gpu_solve(P, f, sp, h, bcs, prec, rtol=rtol)
            assert st["status"] == 0, st
            err = rel(p, ref)
            res, _ = orc.residual(f, p, *sp, None, bcs[2], bc_x=bcs[0], bc_y=bcs[1], dz_cells=h)
            print(f"[stretched]   error {err:.2e} residual {res:.1e} (oracle {res_ref:.1e}) "
                  f"kappa {k:.1e}", flush=True)
            if prec == "fp64":
                assert err <= max(1e-12, 4 * k * 2.2e-16), (err, k)
                # backward stable: the residual at the oracle's own level
                assert res <= max(1e-12, 4 * res_ref), (res, res_ref)
            elif prec == "fp32_refine":
                assert res <= rtol, (res, rtol, st)
                assert abs(res - st["rel_residual"]) <= 1e-12 + 0.05 * res
                assert err <= k * (res + res_ref) * 1.01 + 1e-15, (err, k, res)
            else:
                assert err <= max(2e-5, 8 * k * 6e-8), (err, k)
            if DIR in bcs:
                assert st["rhs_mean"] == 0.0
            else:
                assert abs(st["rhs_mean"] - info["rhs_mean"]) <= 1e-13


def test_equal_thicknesses_equal_uniform():
    P = _gpu()
    nx, ny, nz = 64, 32, 40
    sp = (2.0 / nx, 1.0 / ny, 1.0 / nz)
    f = inputs.random_rhs(nx, ny, nz, seed=4)
    rhs = torch.from_numpy(f).cuda()
    for prec in ("fp64", "fp32"):
        with P.Plan(nx, ny, nz, *sp, NEU, prec) as plan:
            u, _ = plan.solve(rhs)
        with P.Plan(nx, ny, nz, *sp, NEU, prec, dz_cells=np.full(nz, sp[2])) as plan:
            s_, _ = plan.solve(rhs)
        torch.cuda.synchronize()
        a, b = s_.cpu().numpy(), u.cpu().numpy()
        assert rel(a, b) <= (1e-13 if prec == "fp64" else 1e-6), (prec, rel(a, b))


def test_stretched_full_size(orc):
    """512 x 512 x 256 walls (box 2 x 2 x 1) on a tanh grid (beta = 2): the
    oracle's residual of the FP64 and refined solutions over the whole grid
    and their error against the oracle's solve."""
    P = _gpu()
    nx, ny, nz = 512, 512, 256
    h = inputs.tanh_cells(nz, 1.0, 2.0)
    sp = (2.0 / nx, 2.0 / ny)
    f = inputs.random_rhs(nx, ny, nz, seed=3, zero_mean=False)
    print("[stretched] full size: oracle solve", flush=True)
    ref = orc.solve(f, *sp, None, NEU, dz_cells=h)
    for prec, tol in (("fp64", 1e-12), ("fp32_refine", 1e-10)):
        p, st = gpu_solve(P, f, sp, h, (PER, PER, NEU), prec)
        res, _ = orc.residual(f, p, *sp, None, NEU, dz_cells=h)
        err = rel(p, ref)
        print(f"[stretched] full size {prec}: residual {res:.2e} error {err:.2e} {st}",
              flush=True)
        assert st["status"] == 0 and res <= tol and err <= tol, (prec, res, err)


def test_stretched_batch_and_noalloc_equal_plan():
    P = _gpu()
    shapes = [((32, 16, 24), 2.0, NEU), ((32, 16, 24), 1.0, NEU), ((48, 24, 20), 0.0, DIR),
              ((32, 16, 24), 2.0, NEU)]
    probs, rhs = [], []
    for (nx, ny, nz), beta, bz in shapes:
        h = inputs.tanh_cells(nz, 1.0, beta) if beta else None
        f = torch.from_numpy(inputs.random_rhs(nx, ny, nz, seed=nz + int(10 * beta))).cuda()
        probs.append(dict(nx=nx, ny=ny, nz=nz, dx=1.0 / nx, dy=1.0 / ny, dz=1.0 / nz, bc_z=bz,
                          dz_cells=h))
        rhs.append(f)

    for prec in ("fp64", "fp32_refine"):
        singles = []
        for pr, f in zip(probs, rhs):
            nx, ny, nz, bz, h = pr["nx"], pr["ny"], pr["nz"], pr["bc_z"], pr["dz_cells"]
            with P.Plan(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, bz, prec, dz_cells=h) as plan:
                q, _ = plan.solve(f)
                torch.cuda.synchronize()
                singles.append(q.cpu().numpy())
            outs_na = torch.empty_like(f)
            st = P.solve_noalloc(f, outs_na, 1.0 / nx, 1.0 / ny, 1.0 / nz, bz, prec,
                                 dz_cells=h)
            torch.cuda.synchronize()
            assert np.array_equal(outs_na.cpu().numpy(), singles[-1]), prec
        for mode in ("host", "device"):
            bp = P.BatchPlan(probs, prec)
            bp.set_graph(mode)
            outs = [torch.empty_like(r) for r in rhs]
            rc, _ = bp.solve(rhs, outs)
            torch.cuda.synchronize()
            bp.close()
            assert rc == 0
            for o, q in zip(outs, singles):
                o = o.cpu().numpy()
                if prec == "fp64":
                    assert np.array_equal(o, q), mode
                else:  # the batch's sums are blocked by the group's size
                    assert np.max(np.abs(o - q)) <= 1e-14 * np.max(np.abs(q)), mode


def test_stretched_rejections():
    P = _gpu()
    h = inputs.tanh_cells(8, 1.0, 2.0)
    assert P.validate(P.make_desc(8, 8, 8, bc_z=PER, dz_cells=h)) == P.ERR_UNSUPPORTED
    bad = h.copy()
    bad[3] = -1.0
    assert P.validate(P.make_desc(8, 8, 8, bc_z=NEU, dz_cells=bad)) == P.ERR_INVALID_ARG
    bad[3] = float("nan")
    assert P.validate(P.make_desc(8, 8, 8, bc_z=NEU, dz_cells=bad)) == P.ERR_INVALID_ARG
    with P.Plan(8, 8, 8, 0.1, 0.1, 0.1, NEU, "fp64", dz_cells=h) as plan:
        u = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
        v, w = torch.zeros_like(u), torch.zeros_like(u)
        with pytest.raises(P.PoissonError) as e:
            plan.project(u, v, w)
        assert e.value.code == P.ERR_UNSUPPORTED
