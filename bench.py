"""Benchmark of the FFT-based Poisson solve (FluTAS Section 3.3.1) on one MI355X.

One step = one complete solve of the 512x512x256 wall-bounded workload
(2:2:1 box, walls in z, divergence of a seeded velocity over a two-layer
density): forward x, forward y, tridiagonal z solve, backward y, backward x,
and for FP32 + refinement the FP64 residual passes and corrections until the
relative residual is <= 1e-10.  Inputs are resident in HBM before timing.

Prints one JSON line.  `value` is the FP32+refinement throughput in Mpoints/s;
the plain FP64 solve of the same workload is timed beside it, and so is the
whole projection step on the same grid (divergence of the face velocities
fused into the first pass, the solve, the velocity correction and pressure
update), under "projection", and wall-bounded boxes of the same grid (a
cavity and a channel, cosine expansions along x and y), under "walls".  The
256^3 triply periodic workload (spectral right-hand side) is timed the same
way under "hit256", the 512x512x256 grid with tanh-stretched z cells under
"stretched", and the largest single-GPU configuration (1024x1024x512 walls,
spectral right-hand side synthesised on the GPU) under "rb1024".  The error of every returned field against the FP64
oracle is reported under "err_vs_oracle" (the oracle's solve of the whole
grid is also the CPU baseline).  The roofline
entry is for the kernel with the largest share of the FP32+refinement step,
timed live with HIP events on the plan's stream.

    python bench.py [--steps K] [--warmup W] [--workload rb512] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpoints/s Poisson solve, FP32+refine vs FP64 @1e-10 resid; HBM GB/s %peak"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published figure
COPY_BYTES = 1 << 30
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_rb512.txt")
KERNEL_SOURCES = ["api.cpp", "common.hpp", "fft_core.hpp", "lengths.hpp", "k_misc.hip",
                  "k_xpass.hip", "k_xlist.hip", "k_ypass.hip", "k_zperiodic.hip", "k_zwalls.hip",
                  "zper_body.hpp", "stencil.hpp"]

DESCRIPTIONS = {
    "rb512": "512x512x256 walls-in-z, box 2x2x1, RHS = div(u/rho_face) with a two-layer "
             "density and U(-1,1) velocities (seed 3), zero mean",
    "hit256": "256^3 triply periodic (2pi)^3, RHS = div of a k^-5/3 random-phase velocity "
              "(shells 1..85, seed 2)",
    "rb1024": "1024x1024x512 walls-in-z, box 2x2x1, RHS = div of a k^-5/3 random-phase "
              "velocity (shells 1..341, seed 5)",
    "walls32": "32^3 walls-in-z unit box, RHS = div of U(-1,1) velocities (seed 42)",
}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2204_08834_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(pass_name: str):
    """HBM bytes per launch of one pass from the committed rocprofv3 counter
    summary, or None when it is absent, lacks the pass, or the kernel sources
    changed since it was taken."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    kv = {}
    with open(PROFILE_TRAFFIC) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if "=" in line:
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_hash():
        return None
    try:
        return float(kv[f"hbm_bytes[{pass_name}]"])
    except (KeyError, ValueError):
        return None


def time_solves(plan, rhs, out, steps, sync_each):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        if sync_each:
            _, last = plan.solve(rhs, out)
        else:
            plan.solve_async(rhs, out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, last


def bench_batch(steps, warmup):
    """The 64-problem mixed batch (24 x 64^3 periodic, 24 x 96x96x48 walls,
    16 x 128x128x64 walls; U(-1,1) velocity divergences, seeds 1000+b),
    FP32 + refinement to 1e-10, through one batched plan: host-driven loop,
    captured-graph loop and eager device loop in the work-list schedule, and
    the two device loops in the per-group schedule for comparison."""
    import torch
    from paper_2204_08834_amd import inputs, poisson
    probs = inputs.batch_mixed64()
    for p in probs:
        inputs.make_rhs(p)
    specs = [dict(nx=p.nx, ny=p.ny, nz=p.nz, dx=p.dx, dy=p.dy, dz=p.dz, bc_z=p.bc_z)
             for p in probs]
    rhs = [torch.from_numpy(p.f).cuda() for p in probs]
    outs = [torch.empty_like(r) for r in rhs]
    npts = sum(p.npoints for p in probs)
    res = {"problems": len(probs), "points": npts,
           "schedules": "list: one work-list launch per pass for all shapes; groups: one "
                        "launch per shape group and pass on forked streams; tuned: the "
                        "autotuner's choice per loop driver (host / graph / device entries)"}
    runs = [("host", "tuned"), ("graph", "tuned"), ("device", "tuned"),
            ("host", "list"), ("device", "list"), ("graph", "list"),
            ("host", "groups"), ("device", "groups"), ("graph", "groups")]
    for mode, sched in runs:
        if sched != "tuned":
            os.environ["POISSON_BATCH_SCHEDULE"] = sched
        bp = poisson.BatchPlan(specs, "fp32_refine", rtol=1e-10, max_refine=8)
        os.environ.pop("POISSON_BATCH_SCHEDULE", None)
        bp.autotune()
        if sched == "tuned":
            res["schedule"] = bp.describe().strip()
        bp.set_graph(mode)
        for _ in range(warmup):
            bp.solve(rhs, outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = bp.solve(rhs, outs)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        bp.close()
        key = mode if sched == "tuned" else f"{mode}_{sched}"
        res[key] = {"ms_per_batch": ms, "mpoints_s": npts / (ms * 1e-3) / 1e6,
                    "max_rel_residual": max(x["rel_residual"] for x in st),
                    "max_iterations": max(x["iterations"] for x in st)}
    return res


def bench_project(prob, steps, warmup, tune):
    """The projection step (poisson_project) on the workload's grid: U(-1,1)
    face velocities (the workload's seed), alpha = beta = 1, with the pressure
    update.  Every step projects a fresh copy of the same provisional
    velocity; the copy is made before the step's timed region."""
    import torch
    from paper_2204_08834_amd import inputs, poisson
    u, v, w = inputs.uniform_velocity(prob.nx, prob.ny, prob.nz, prob.bc_z, prob.seed)
    src = [torch.from_numpy(x).cuda() for x in (u, v, w)]
    del u, v, w
    work = [torch.empty_like(x) for x in src]
    pres = torch.zeros_like(src[0])
    psi = torch.empty_like(src[0])
    npts = prob.npoints
    dx, dy, dz = prob.spacings()
    res = {"velocity": "U(-1,1) face velocities, alpha = beta = 1, p += psi"}

    def step(plan):
        for a, b in zip(work, src):
            a.copy_(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = plan.project(*work, pres, psi, 1.0, 1.0)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    for prec in ("fp32_refine", "fp64"):
        plan = poisson.Plan(prob.nx, prob.ny, prob.nz, dx, dy, dz, prob.bc_z, prec,
                            rtol=1e-10, max_refine=8)
        if tune:
            plan.autotune()
        for _ in range(warmup):
            step(plan)
        total, st = 0.0, None
        for _ in range(steps):
            t, st = step(plan)
            total += t
        ms = total / steps * 1e3
        plan.set_timing(True)
        plan.reset_timing()
        for _ in range(steps):
            step(plan)
        passes = plan.timing()
        plan.close()
        step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in passes.values()) / steps
        res[prec] = {
            "ms_per_step": ms, "mpoints_s": npts / (ms * 1e-3) / 1e6,
            "rel_residual": st["rel_residual"], "iterations": st["iterations"],
            "model_bytes_per_point": step_bytes / npts,
            "model_hbm_gbs": step_bytes / (ms * 1e-3) / 1e9,
            "passes": {k: {"avg_ms": v["total_ms"] / v["launches"],
                           "launches_per_step": v["launches"] / steps,
                           "gbs": v["bytes_per_launch"] / (v["total_ms"] / v["launches"]
                                                           * 1e-3) / 1e9}
                       for k, v in passes.items()}}
        print(f"[bench] projection {prec} {ms:.3f} ms/step", file=sys.stderr, flush=True)
    return res


def bench_walls(steps, warmup, tune):
    """Wall-bounded boxes on the rb512 grid (512x512x256, box 2x2x1): a
    cavity with Neumann walls on every axis and a channel (periodic x, walls
    in y and z), U(-1,1) right-hand side (seed 3); FP32 + refinement to 1e-10
    and FP64, per-pass event timing."""
    import torch
    from paper_2204_08834_amd import inputs, poisson
    nx, ny, nz = 512, 512, 256
    sp = (2.0 / nx, 2.0 / ny, 1.0 / nz)
    f = torch.from_numpy(inputs.random_rhs(nx, ny, nz, seed=3, zero_mean=False)).cuda()
    out = torch.empty_like(f)
    npts = nx * ny * nz
    res = {}
    for name, (bx, by, bz) in (("cavity_NNN", (1, 1, 1)), ("channel_PNN", (0, 1, 1))):
        entry = {}
        for prec in ("fp32_refine", "fp64"):
            plan = poisson.Plan(nx, ny, nz, *sp, bz, prec, rtol=1e-10, max_refine=8,
                                bc_x=bx, bc_y=by)
            if tune:
                plan.autotune()
            for _ in range(warmup):
                plan.solve(f, out)
            ms, st = time_solves(plan, f, out, steps, sync_each=True)
            plan.set_timing(True)
            plan.reset_timing()
            for _ in range(steps):
                plan.solve(f, out)
            passes = plan.timing()
            schedule = plan.describe().strip()
            plan.close()
            step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in passes.values()) / steps
            entry[prec] = {
                "ms_per_step": ms, "mpoints_s": npts / (ms * 1e-3) / 1e6,
                "rel_residual": st["rel_residual"], "iterations": st["iterations"],
                "model_hbm_gbs": step_bytes / (ms * 1e-3) / 1e9,
                "schedule": schedule,
                "passes": {k: {"avg_ms": v["total_ms"] / v["launches"],
                               "launches_per_step": v["launches"] / steps,
                               "gbs": v["bytes_per_launch"] / (v["total_ms"] / v["launches"]
                                                               * 1e-3) / 1e9}
                           for k, v in passes.items()}}
            print(f"[bench] walls {name} {prec} {ms:.3f} ms/solve", file=sys.stderr, flush=True)
        res[name] = entry
    return res


def host_cpu():
    """CPU model name and logical CPU counts of the host (Linux /proc)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_baseline(prob, nplanes):
    """The FP64 oracle timed on the host on the workload, or on a slab of it:
    the first `nplanes` z-planes (x and y lines keep their full length, so
    the per-point cost of the oracle's O(n) per-point DFTs is that of the
    full grid).  The default is the whole grid (about 13 s on 16 cores).
    Returns the record and the oracle's solution (None for a slab, which is
    a different problem)."""
    import numpy as np
    import oracle
    f = np.ascontiguousarray(prob.f[:nplanes])
    oracle.solve(f[:2], *prob.spacings(), prob.bc_z)  # load the library, warm up
    t0 = time.perf_counter()
    p = oracle.solve(f, *prob.spacings(), prob.bc_z)
    dt = time.perf_counter() - t0
    pts = f.size
    rec = {"value": pts / dt / 1e6, "unit": "Mpoints/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": (f"the whole {prob.nx}x{prob.ny}x{prob.nz} workload" if nplanes == prob.nz
                      else f"first {nplanes} of {prob.nz} z-planes of the workload "
                           f"({prob.nx}x{prob.ny}x{nplanes})")
                     + f", one FP64 oracle solve, {dt:.2f} s"}
    rec.update(host_cpu())
    return rec, (p if nplanes == prob.nz else None)


def error_vs_oracle(p, ref):
    """Relative L2 and max-norm error of a solution against the oracle's."""
    import numpy as np
    d = p - ref
    return {"rel_l2": float(np.linalg.norm(d.ravel()) / np.linalg.norm(ref.ravel())),
            "rel_max": float(np.abs(d).max() / np.abs(ref).max())}


def bench_extra_workload(name, steps, warmup, tune, with_oracle):
    """A second workload of the scope (hit256: 256^3 triply periodic,
    spectral right-hand side): FP32 + refinement to 1e-10 and plain FP64,
    each timed like the main workload, with the error of both results
    against the FP64 oracle."""
    import torch
    from paper_2204_08834_amd import inputs, poisson
    prob = inputs.workload(name)
    npts = prob.npoints
    sp = prob.spacings()
    rhs = torch.from_numpy(prob.f).cuda()
    out = torch.empty_like(rhs)
    res = {"workload": f"{name}: {DESCRIPTIONS[name]}", "grid": [prob.nx, prob.ny, prob.nz]}
    sols = {}
    for prec in ("fp32_refine", "fp64"):
        plan = poisson.Plan(prob.nx, prob.ny, prob.nz, *sp, prob.bc_z, prec, rtol=1e-10,
                            max_refine=8)
        if tune:
            plan.autotune()
        for _ in range(warmup):
            plan.solve(rhs, out)
        refine = prec == "fp32_refine"
        ms, st = time_solves(plan, rhs, out, steps, sync_each=refine)
        plan.set_timing(True)
        plan.reset_timing()
        for _ in range(steps):
            plan.solve(rhs, out)
        passes = plan.timing()
        plan.close()
        step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in passes.values()) / steps
        res[prec] = {"ms_per_step": ms, "mpoints_s": npts / (ms * 1e-3) / 1e6,
                     "model_hbm_gbs": step_bytes / (ms * 1e-3) / 1e9,
                     "model_bytes_per_point": step_bytes / npts}
        if refine:
            res[prec].update(rel_residual=st["rel_residual"], iterations=st["iterations"])
        sols[prec] = out.cpu().numpy()
        print(f"[bench] {name} {prec} {ms:.3f} ms/solve", file=sys.stderr, flush=True)
    res["fp32refine_over_fp64_speed"] = res["fp64"]["ms_per_step"] / res["fp32_refine"][
        "ms_per_step"]
    # the error against the oracle is taken in the CPU-baseline leg
    return res, (prob if with_oracle else None), sols


def bench_stretched(steps, warmup, tune):
    """The 512x512x256 walls grid (box 2x2x1) with tanh-stretched z cells
    (beta = 2, clustered at both walls), U(-1,1) right-hand side (seed 3):
    FP32 + refinement to 1e-10 and FP64."""
    import torch
    from paper_2204_08834_amd import inputs, poisson
    nx, ny, nz = 512, 512, 256
    h = inputs.tanh_cells(nz, 1.0, 2.0)
    f = torch.from_numpy(inputs.random_rhs(nx, ny, nz, seed=3, zero_mean=False)).cuda()
    out = torch.empty_like(f)
    npts = nx * ny * nz
    res = {"grid": [nx, ny, nz], "dz_cells": "tanh, beta 2 (min/max thickness "
           f"{h.min():.2e}/{h.max():.2e})"}
    for prec in ("fp32_refine", "fp64"):
        plan = poisson.Plan(nx, ny, nz, 2.0 / nx, 2.0 / ny, 1.0 / nz, 1, prec, rtol=1e-10,
                            dz_cells=h)
        if tune:
            plan.autotune()
        for _ in range(warmup):
            plan.solve(f, out)
        ms, st = time_solves(plan, f, out, steps, sync_each=True)
        plan.set_timing(True)
        plan.reset_timing()
        for _ in range(steps):
            plan.solve(f, out)
        passes = plan.timing()
        schedule = plan.describe().strip()
        plan.close()
        res[prec] = {"ms_per_step": ms, "mpoints_s": npts / (ms * 1e-3) / 1e6,
                     "rel_residual": st["rel_residual"], "iterations": st["iterations"],
                     "schedule": schedule,
                     "passes": {k: {"avg_ms": v["total_ms"] / v["launches"],
                                    "gbs": v["bytes_per_launch"] / (v["total_ms"] / v["launches"]
                                                                    * 1e-3) / 1e9}
                                for k, v in passes.items() if v["launches"]}}
        print(f"[bench] stretched {prec} {ms:.3f} ms/solve", file=sys.stderr, flush=True)
    return res


def bench_rb1024(steps, tune):
    """The largest single-GPU configuration, 1024x1024x512 walls in z (box
    2x2x1), right-hand side from the spectral recipe (shells 1..341, seed 5)
    synthesised on the GPU (the host synthesis takes minutes): FP32 +
    refinement to 1e-10 and FP64, with the refinement's relative residual
    (the oracle's O(n^2) transforms are out of reach at this size)."""
    import torch
    from paper_2204_08834_amd import inputs, poisson
    nx, ny, nz = 1024, 1024, 512
    t0 = time.perf_counter()
    rhs = inputs.spectral_velocity_rhs_torch(nx, ny, nz, 2.0, 2.0, 1.0, 1, 5, 341).contiguous()
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    torch.cuda.empty_cache()
    out = torch.empty_like(rhs)
    npts = nx * ny * nz
    res = {"workload": f"rb1024: {DESCRIPTIONS['rb1024']}; synthesised on the GPU "
                       f"(torch generator, {gen_s:.1f} s)", "grid": [nx, ny, nz]}
    for prec in ("fp32_refine", "fp64"):
        plan = poisson.Plan(nx, ny, nz, 2.0 / nx, 2.0 / ny, 1.0 / nz, 1, prec, rtol=1e-10)
        if tune:
            plan.autotune()
        plan.solve(rhs, out)
        ms, st = time_solves(plan, rhs, out, steps, sync_each=prec == "fp32_refine")
        plan.set_timing(True)
        plan.reset_timing()
        plan.solve(rhs, out)
        passes = plan.timing()
        plan.close()
        step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in passes.values())
        res[prec] = {"ms_per_step": ms, "mpoints_s": npts / (ms * 1e-3) / 1e6,
                     "model_hbm_gbs": step_bytes / (ms * 1e-3) / 1e9,
                     "model_bytes_per_point": step_bytes / npts,
                     "passes": {k: {"avg_ms": v["total_ms"] / v["launches"],
                                    "launches": v["launches"],
                                    "gbs": v["bytes_per_launch"] / (v["total_ms"] / v["launches"]
                                                                    * 1e-3) / 1e9}
                                for k, v in passes.items() if v["launches"]}}
        if st is not None:
            res[prec].update(rel_residual=st["rel_residual"], iterations=st["iterations"])
        print(f"[bench] rb1024 {prec} {ms:.3f} ms/solve", file=sys.stderr, flush=True)
    res["fp32refine_over_fp64_speed"] = res["fp64"]["ms_per_step"] / res["fp32_refine"][
        "ms_per_step"]
    del rhs, out
    torch.cuda.empty_cache()
    return res


def copy_calibration(steps, warmup):
    """Plain streaming kernels of known size: a device-to-device copy (the
    runtime's blit kernel) and an elementwise negation, 1 GiB read and 1 GiB
    written each.  The bandwidth they reach, and what the rocprofv3
    FETCH_SIZE / WRITE_SIZE counters read for them, calibrate the solver's
    counters."""
    import torch
    n = COPY_BYTES // 8
    src = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    out = {"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES}
    for label, fn in (("blit_copy", lambda: dst.copy_(src)),
                      ("elementwise_neg", lambda: torch.neg(src, out=dst))):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        gbs = 2 * COPY_BYTES / (ms * 1e-3) / 1e9
        out[label] = {"ms": ms, "gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}
    return out


# kernel-name patterns of the solver's passes (rocprofv3 reports demangled names)
PASS_PATTERNS = [
    ("x_r2c_residual_{p}", r"prec_{p}::k_x_res<\d+, false[,>]"),
    ("x_r2c_residual_walls_{p}", r"prec_{p}::k_x_res<\d+, true[,>]"),
    ("x_r2c_divergence_{p}", r"prec_{p}::k_x_div<"),
    ("x_r2c_{p}", r"prec_{p}::k_x_fwd<\d+, false>"),
    ("x_r2c_walls_{p}", r"prec_{p}::k_x_fwd<\d+, true>"),
    ("x_c2r_accumulate_{p}", r"prec_{p}::k_x_inv<\d+, true, false[,>]"),
    ("x_c2r_accumulate_walls_{p}", r"prec_{p}::k_x_inv<\d+, true, true[,>]"),
    ("x_c2r_{p}", r"prec_{p}::k_x_inv<\d+, false, false[,>]"),
    ("x_c2r_walls_{p}", r"prec_{p}::k_x_inv<\d+, false, true[,>]"),
    ("y_fwd_{p}", r"prec_{p}::k_y<\d+, false[,>]"),
    ("y_inv_{p}", r"prec_{p}::k_y<\d+, true[,>]"),
    ("y_fwd_walls_{p}", r"prec_{p}::k_yw<\d+, false>"),
    ("y_inv_walls_{p}", r"prec_{p}::k_yw<\d+, true>"),
    ("z_walls_{p}", r"prec_{p}::k_z_walls(_r)?<"),
    ("z_periodic_{p}", r"prec_{p}::k_z_per<"),
]


def pass_of_kernel(name):
    import re
    for p in ("f32", "f64"):
        for label, pat in PASS_PATTERNS:
            if re.search(pat.format(p=p), name):
                return label.format(p=p)
    if "k_residual_check" in name:
        return "residual_check_f64"
    if "k_sum_partials" in name:
        return "sum_partials"
    if "k_correct<" in name:
        return "correct_f64"
    return None


def read_counter_csv(path):
    """{(kernel name, counter): [value per dispatch]} from a rocprofv3
    counter_collection.csv."""
    import csv
    vals = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            key = (r["Kernel_Name"], r["Counter_Name"])
            vals.setdefault(key, []).append(float(r["Counter_Value"]))
    return vals


def summarize_counters(fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, out_path, commands):
    """Write the HBM traffic summary read by this script's roofline entry:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per pass, each scaled by
    what the same counter reads for the 1 GiB elementwise calibration
    kernel."""
    import statistics
    fetch, write = read_counter_csv(fetch_csv), read_counter_csv(write_csv)
    cfetch, cwrite = read_counter_csv(cal_fetch_csv), read_counter_csv(cal_write_csv)

    def cal(vals, counter):
        xs = [v for (k, c), vs in vals.items() if c == counter and "neg" in k for v in vs]
        return statistics.median(xs) * 1024.0
    f_scale = COPY_BYTES / cal(cfetch, "FETCH_SIZE")
    w_scale = COPY_BYTES / cal(cwrite, "WRITE_SIZE")
    def working(vs):
        # dispatches that did the pass's work: gated-off launches of the
        # device-side loop exit at once and read almost nothing
        top = max(vs)
        return [v for v in vs if v >= 0.1 * top]

    per_pass = {}
    for (k, c), vs in fetch.items():
        ps = pass_of_kernel(k)
        if ps and c == "FETCH_SIZE":
            per_pass.setdefault(ps, {})["fetch"] = statistics.median(working(vs)) * 1024.0
    for (k, c), vs in write.items():
        ps = pass_of_kernel(k)
        if ps and c == "WRITE_SIZE":
            per_pass.setdefault(ps, {})["write"] = statistics.median(working(vs)) * 1024.0
    lines = ["# HBM traffic per dispatch, rocprofv3 counters, 512x512x256 walls-in-z (rb512)",
             "# commands (from the repository root; rocprofv3 runs after "
             "`cd /tmp && export TMPDIR=/tmp`):"]
    lines += ["#   " + c for c in commands]
    lines += [f"# calibration: 1 GiB elementwise kernel reads FETCH_SIZE x {f_scale:.4f}, "
              f"WRITE_SIZE x {w_scale:.4f} of its true bytes",
              "# bytes below = counter KiB x 1024 x scale, median over the dispatches that did "
              "the pass's work (gated-off launches of the device-side loop excluded)",
              f"source_hash = {kernel_hash()}",
              f"fetch_scale = {f_scale:.6f}", f"write_scale = {w_scale:.6f}"]
    for ps in sorted(per_pass):
        fb = per_pass[ps].get("fetch", 0.0) * f_scale
        wb = per_pass[ps].get("write", 0.0) * w_scale
        lines.append(f"hbm_bytes[{ps}] = {fb + wb:.0f}   # read {fb:.0f} write {wb:.0f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_kernels(trace_csv, out_path, commands):
    """Write the per-kernel duration summary from a rocprofv3 kernel_trace.csv:
    dispatches, average / min / max duration of the dispatches that did the
    pass's work (gated-off launches of the device-side loop, which exit at
    once, are counted apart), share of the total, and the pass name."""
    import csv
    per = {}
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            per.setdefault(r["Kernel_Name"], []).append(d)
    total = sum(sum(v) for v in per.values())
    rows = []
    for name, ds in per.items():
        top = max(ds)
        work = [d for d in ds if d >= 0.1 * top]
        rows.append((sum(ds), name, len(ds), len(ds) - len(work), sum(work) / len(work), min(work),
                     max(work)))
    rows.sort(reverse=True)
    lines = ["# rocprofv3 kernel trace, 512x512x256 walls-in-z (rb512): every dispatch of the "
             "run (warmup, timed steps, per-pass timing, FP32+refine and FP64 plans)",
             "# commands (from the repository root; rocprofv3 runs after "
             "`cd /tmp && export TMPDIR=/tmp`):"]
    lines += ["#   " + c for c in commands]
    lines.append(f"# source_hash = {kernel_hash()}")
    lines.append("# avg/min/max over the dispatches that did the pass's work; 'gated' counts "
                 "launches of the device-side loop that exited at once")
    lines.append(f"{'pass':22s} {'calls':>5s} {'gated':>5s} {'avg_us':>9s} {'min_us':>9s} "
                 f"{'max_us':>9s} {'pct':>6s}  kernel")
    for tot, name, n, ng, avg, mn, mx in rows:
        lines.append(f"{pass_of_kernel(name) or '-':22s} {n:5d} {ng:5d} {avg:9.2f} {mn:9.2f} "
                     f"{mx:9.2f} {100.0 * tot / total:6.2f}  {name[:70]}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rb512", choices=sorted(DESCRIPTIONS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-project", action="store_true",
                    help="skip the projection step (divergence, solve, correction)")
    ap.add_argument("--no-walls", action="store_true",
                    help="skip the wall-bounded boxes (walls along x and y)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (hit256: 256^3 triply periodic; the "
                         "stretched-z 512x512x256 grid; rb1024: 1024x1024x512 walls)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the captured-graph loop timing (profiling runs: its gated-off "
                         "launches would mix into the per-kernel statistics)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default launch variants (no plan-time autotuning)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched workload (profiling runs)")
    ap.add_argument("--cpu-planes", type=int, default=0,
                    help="z-planes of the workload in the CPU oracle sample (0: all)")
    ap.add_argument("--only", choices=["fp32_refine", "fp64"], default=None,
                    help="time one precision only (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="time plain 1 GiB copy kernels instead (the HBM bandwidth a "
                         "streaming kernel attains, and the reference for scaling "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--summarize-counters", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV",
                    "CAL_FETCH_CSV", "CAL_WRITE_CSV", "OUT"),
                    help="write the HBM traffic summary from rocprofv3 --pmc FETCH_SIZE / "
                         "WRITE_SIZE counter_collection.csv files of a solve run and of a "
                         "--copy-calibration run")
    ap.add_argument("--summarize-kernels", nargs=2, metavar=("TRACE_CSV", "OUT"),
                    help="write the per-kernel duration summary from a rocprofv3 "
                         "kernel_trace.csv")
    ap.add_argument("--command", action="append", default=[],
                    help="with --summarize-*: a command to record in the summary")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, commands=args.command)
        return
    if args.summarize_kernels:
        summarize_kernels(*args.summarize_kernels, commands=args.command)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU; multi-GPU runs are not supported "
              "(a slab decomposition with all-to-all transposes would be the way to shard it)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_08834_amd import inputs, poisson

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    poisson.lib()  # fail loudly if the HIP library is missing

    if args.copy_calibration:
        print(json.dumps(copy_calibration(args.steps, args.warmup)), flush=True)
        return

    if args.batch_only:
        print(json.dumps({"batch_mixed64": bench_batch(args.steps, args.warmup)}), flush=True)
        return

    prob = inputs.workload(args.workload)
    npts = prob.npoints
    dx, dy, dz = prob.spacings()
    rhs = torch.from_numpy(prob.f).cuda()
    out = torch.empty_like(rhs)
    print(f"[bench] workload {prob.name} {prob.nx}x{prob.ny}x{prob.nz} ready", file=sys.stderr,
          flush=True)

    result = {"metric": METRIC, "value": None, "unit": "Mpoints/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f32+f64", "data": "synthetic",
              "config": {"workload": f"{prob.name}: {DESCRIPTIONS[prob.name]}",
                         "grid": [prob.nx, prob.ny, prob.nz],
                         "bc_z": "walls" if prob.bc_z == 1 else "periodic",
                         "rtol": 1e-10, "parallelism": "single GPU"}}

    solutions = {}  # returned fields, for the error against the oracle

    # ---- FP32 + FP64-residual refinement --------------------------------
    if args.only in (None, "fp32_refine"):
        plan = poisson.Plan(prob.nx, prob.ny, prob.nz, dx, dy, dz, prob.bc_z, "fp32_refine",
                            rtol=1e-10, max_refine=8)
        if not args.no_tune:
            plan.autotune()
        result["schedule_fp32_refine"] = plan.describe().strip()
        for _ in range(args.warmup):
            plan.solve(rhs, out)
        ms32, st = time_solves(plan, rhs, out, args.steps, sync_each=True)
        print(f"[bench] fp32+refine {ms32:.3f} ms/solve, stats {st}", file=sys.stderr,
              flush=True)
        # per-pass timing over a second timed region
        plan.set_timing(True)
        plan.reset_timing()
        for _ in range(args.steps):
            plan.solve(rhs, out)
        passes = plan.timing()
        plan.set_timing(False)
        # the same solves through the captured-graph loop
        if not args.no_graph:
            plan.set_graph("graph")
            for _ in range(args.warmup):
                plan.solve(rhs, out)
            msg, stg = time_solves(plan, rhs, out, args.steps, sync_each=True)
            result["fp32refine_graph_loop"] = {"ms_per_step": msg,
                                               "mpoints_s": npts / (msg * 1e-3) / 1e6,
                                               "rel_residual": stg["rel_residual"]}
        plan.close()
        solutions["fp32_refine"] = out.cpu().numpy()
        result["value"] = npts / (ms32 * 1e-3) / 1e6
        result["ms_per_step"] = ms32
        result["refine_iterations"] = st["iterations"]
        result["rel_residual"] = st["rel_residual"]
        step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in passes.values()) / max(
            1, args.steps)
        result["model_bytes_per_point"] = step_bytes / npts
        result["model_hbm_gbs"] = step_bytes / (ms32 * 1e-3) / 1e9
        result["model_hbm_frac"] = result["model_hbm_gbs"] / HBM_PEAK_GBS
        dom_name, dom = max(((k, v) for k, v in passes.items() if k != "sum_partials"),
                            key=lambda kv: kv[1]["total_ms"])
        avg_ms = dom["total_ms"] / dom["launches"]
        achieved = dom["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
        traffic = read_traffic(dom_name)
        result["roofline"] = {"bound": "hbm", "kernel_pass": dom_name,
                              "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": achieved / HBM_PEAK_GBS,
                              "traffic": traffic,
                              "algorithmic_bytes_per_launch": dom["bytes_per_launch"],
                              "avg_launch_ms": avg_ms}
        result["passes"] = {k: {"avg_ms": v["total_ms"] / v["launches"],
                                "launches_per_step": v["launches"] / args.steps,
                                "gbs": v["bytes_per_launch"] / (v["total_ms"] / v["launches"]
                                                                * 1e-3) / 1e9}
                            for k, v in passes.items()}

    # ---- plain FP64 -----------------------------------------------------
    if args.only in (None, "fp64"):
        plan = poisson.Plan(prob.nx, prob.ny, prob.nz, dx, dy, dz, prob.bc_z, "fp64")
        if not args.no_tune:
            plan.autotune()
        result["schedule_fp64"] = plan.describe().strip()
        for _ in range(args.warmup):
            plan.solve(rhs, out)
        ms64, _ = time_solves(plan, rhs, out, args.steps, sync_each=False)
        plan.set_timing(True)
        plan.reset_timing()
        for _ in range(args.steps):
            plan.solve_async(rhs, out)
        p64 = plan.timing()
        plan.close()
        solutions["fp64"] = out.cpu().numpy()
        print(f"[bench] fp64 {ms64:.3f} ms/solve", file=sys.stderr, flush=True)
        b64 = sum(v["bytes_per_launch"] * v["launches"] for v in p64.values()) / args.steps
        result["fp64_plain"] = {
            "mpoints_s": npts / (ms64 * 1e-3) / 1e6, "ms_per_step": ms64,
            "model_hbm_gbs": b64 / (ms64 * 1e-3) / 1e9,
            "model_hbm_frac": b64 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "passes": {k: {"avg_ms": v["total_ms"] / v["launches"],
                           "gbs": v["bytes_per_launch"] / (v["total_ms"] / v["launches"]
                                                           * 1e-3) / 1e9}
                       for k, v in p64.items()}}
        if result["value"] is None:
            result["value"] = result["fp64_plain"]["mpoints_s"]
            result["ms_per_step"] = ms64
            result["dtype"] = "f64"
        else:
            result["fp32refine_over_fp64_speed"] = ms64 / result["ms_per_step"]

    if not args.no_project:
        print("[bench] projection step", file=sys.stderr, flush=True)
        del rhs, out
        torch.cuda.empty_cache()
        result["projection"] = bench_project(prob, max(3, args.steps // 2), 2,
                                             not args.no_tune)

    if not args.no_walls:
        print("[bench] wall-bounded boxes", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        result["walls"] = bench_walls(max(3, args.steps // 2), 2, not args.no_tune)

    if not args.no_batch:
        print("[bench] batched mixed-64 workload", file=sys.stderr, flush=True)
        result["batch_mixed64"] = bench_batch(max(3, args.steps // 4), 2)

    extra = None
    if not args.no_extra and prob.name != "hit256":
        print("[bench] hit256 workload", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        result["hit256"], extra_prob, extra_sols = bench_extra_workload(
            "hit256", args.steps, args.warmup, not args.no_tune, not args.no_cpu)
        if extra_prob is not None:
            extra = (extra_prob, extra_sols)

    if not args.no_extra:
        print("[bench] stretched z", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        result["stretched"] = bench_stretched(max(3, args.steps // 2), 2, not args.no_tune)
        if prob.name != "rb1024":
            print("[bench] rb1024 workload", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
            result["rb1024"] = bench_rb1024(5, not args.no_tune)

    if not args.no_cpu:
        import oracle
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        planes = prob.nz if args.cpu_planes <= 0 else min(args.cpu_planes, prob.nz)
        result["cpu_baseline"], ref = cpu_baseline(prob, planes)
        if ref is not None:
            # the error of each returned field against the FP64 oracle
            result["err_vs_oracle"] = {k: error_vs_oracle(v, ref) for k, v in solutions.items()}
        if extra is not None:
            xp, xs = extra
            print(f"[bench] {xp.name}: oracle solve for the error check", file=sys.stderr,
                  flush=True)
            xref = oracle.solve(xp.f, *xp.spacings(), xp.bc_z)
            result[xp.name]["err_vs_oracle"] = {k: error_vs_oracle(v, xref) for k, v in xs.items()}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
