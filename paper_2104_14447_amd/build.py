"""Build libgmls.so for gfx950 with hipcc (in-tree, next to this file).

Every translation unit is compiled for gfx950 only, with packed FP32
instructions disabled; the neighbour search additionally forbids
floating-point contraction so that squared distances are evaluated exactly
as (dx*dx + dy*dy) + dz*dz.  The stencil kernels are compiled once per
(dimension, order, basis) from the unit sources so that the objects build in
parallel.
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

COMMON = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def units():
    """(object name, source, extra flags), heaviest first."""
    out = []
    for unit in ("mixed_unit.hip", "wave_unit.hip", "qr_unit.hip"):
        stem = unit.split("_")[0]
        for order in (4, 3, 2, 1):
            # basis 0 scalar, 1 divergence-free; 2 staggered (FP64 QR only)
            for basis in ((1, 0, 2) if stem == "qr" else (1, 0)):
                for dim in (3, 2):
                    defs = [f"-DGMLS_DIM={dim}", f"-DGMLS_ORDER={order}", f"-DGMLS_BASIS={basis}"]
                    name = f"{stem}_d{dim}_o{order}_b{basis}"
                    if basis == 1 and stem in ("qr", "wave"):  # the shared kernels in an object of their own
                        out.append((name + "_p0", unit, defs + ["-DGMLS_PART=0"]))
                        out.append((name + "_p1", unit, defs + ["-DGMLS_PART=1"]))
                    else:
                        out.append((name, unit, defs))
    out += [
        ("search", "search.hip", ["-ffp-contract=off"]),
        ("stencil_bins", "stencil_bins.hip", []),
        ("stencil_fp64", "stencil_fp64.hip", []),
        ("stencil_mixed", "stencil_mixed.hip", []),
        ("apply", "apply.hip", []),
        ("assemble", "assemble.hip", []),
        ("api", "api.cpp", ["-x", "hip"]),
    ]
    return out


def hipcc() -> str:
    return "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"


def _compile(name: str, src: str, extra: list[str], verbose: bool) -> str:
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc()] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or int(os.environ.get("MAX_JOBS", 0)) or max(1, os.cpu_count() or 2)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, n, s, e, verbose) for n, s, e in units()]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


SAN_DIR = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_DIR, "libgmls_san.so")


def build_sanitized(verbose: bool = False) -> str:
    """The library with its ABI layer (api.cpp: argument validation, reports,
    workspace, the autotune table and its JSON files) built with
    AddressSanitizer and UndefinedBehaviorSanitizer on the host side only,
    linked with the objects of build() (call that first) into
    _build/san/libgmls_san.so for tests/test_sanitizers.py.  Device code is
    not instrumented (no GPU sanitizer here)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    obj = os.path.join(SAN_DIR, "api.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
    cmd = [hipcc()] + COMMON + san + ["-x", "hip", "-c", os.path.join(CSRC, "api.cpp"), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the sanitized api.cpp:\n{r.stdout}\n{r.stderr}")
    objs = [os.path.join(BUILD, n + ".o") for n, _, _ in units() if n != "api"]
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", tmp, obj] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_sanitized(verbose="-v" in sys.argv))
