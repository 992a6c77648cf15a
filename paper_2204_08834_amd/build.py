"""Build libpoisson.so (HIP, gfx950) in-tree.

    python -m paper_2204_08834_amd.build          # or build() from Python

Every kernel source is compiled with hipcc for gfx950 only; the
precision-templated sources (.hip with PK_REAL) are compiled once per
precision.  Objects go to paper_2204_08834_amd/_build/, the library to
paper_2204_08834_amd/libpoisson.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpoisson.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (plain scalar/vector FP32 only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    f"-I{CSRC}", f"-I{INCLUDE}",
]

PRECISION_SOURCES = ["k_xpass.hip", "k_xlist.hip", "k_ypass.hip", "k_zwalls.hip", "k_zperiodic.hip"]
PLAIN_SOURCES = ["k_misc.hip", "api.cpp"]


def _jobs():
    jobs = []
    for src in PRECISION_SOURCES:
        stem = src.rsplit(".", 1)[0]
        for tag, real in (("f32", "float"), ("f64", "double")):
            obj = os.path.join(OUT, f"{stem}_{tag}.o")
            jobs.append((src, obj, [f"-DPK_REAL={real}", f"-DPK_TAG={tag}"]))
    for src in PLAIN_SOURCES:
        stem = src.rsplit(".", 1)[0]
        jobs.append((src, os.path.join(OUT, f"{stem}.o"), []))
    return jobs


def _compile(job, verbose=False):
    src, obj, defs = job
    cmd = [HIPCC, *COMMON_FLAGS, *defs, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # host-pass warnings about the packed-fp32 feature flag are expected
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source for gfx950 and link libpoisson.so (always rebuilds)."""
    os.makedirs(OUT, exist_ok=True)
    todo = _jobs()
    n = jobs or min(len(todo), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(lambda j: _compile(j, verbose), todo))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
