"""Build libgmls.so for gfx950 with hipcc (in-tree, next to this file).

Every translation unit is compiled for gfx950 only, with packed FP32
instructions disabled; the neighbour search additionally forbids
floating-point contraction so that squared distances are evaluated exactly
as (dx*dx + dy*dy) + dz*dz.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libgmls.so")
ARCH = os.environ.get("GMLS_OFFLOAD_ARCH", "gfx950")

SOURCES = {
    "search.hip": ["-ffp-contract=off"],
    "stencil_bins.hip": [],
    "stencil_fp64.hip": [],
    "qr_2d_scalar.hip": [],
    "qr_3d_scalar.hip": [],
    "qr_2d_divfree.hip": [],
    "qr_3d_divfree.hip": [],
    "stencil_mixed.hip": [],
    "apply.hip": [],
    "api.cpp": [],
}

COMMON = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(cand) or cand == "hipcc":
            return cand
    return "hipcc"


def _compile(name: str, extra: list[str], verbose: bool) -> str:
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, name + ".o")
    lang = ["-x", "hip"] if name.endswith(".cpp") else []
    cmd = [hipcc()] + COMMON + extra + lang + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, n, e, verbose) for n, e in SOURCES.items()]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
