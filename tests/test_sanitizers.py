"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The oracle (plain C) and the library's ABI layer (api.cpp, host side) are
built with both sanitizers by __graft_entry__.build() into _build/san/.  Each
test runs a workload in a fresh Python process with the sanitizer runtime
preloaded (the interpreter itself is not instrumented); a report makes the
process fail, and its output is shown."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SAN = os.path.join(ROOT, "_build", "san", "liboracle_san.so")
LIB_SAN = os.path.join(ROOT, "_build", "san", "libgmls_san.so")


def gcc_asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def clang_asan_runtime():
    import glob

    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def run_sanitized(code, preload, extra_env):
    env = dict(os.environ)
    env.update(extra_env)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "SANITIZED-RUN-OK" in r.stdout, out[-6000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]


def test_oracle_under_sanitizers():
    rt = gcc_asan_runtime()
    if not rt or not os.path.exists(ORACLE_SAN):
        pytest.skip("sanitizer build of the oracle or the ASan runtime missing (run __graft_entry__.build())")
    run_sanitized("""
        import numpy as np
        import oracle, workloads as W
        assert oracle._LIB_PATH.endswith("liboracle_san.so")
        for dim, n, k in ((2, 600, 12), (3, 1500, 30)):
            pts = W.jittered_grid(n, dim, 5)
            for grid in (False, True):
                rp, col, eps = oracle.knn(pts, pts, k, 1.5, use_grid=grid)
                rp2, col2, eps2 = oracle.radius(pts, pts, W.radius_for_mean_count(n) if dim == 3 else 0.08, 10,
                                                use_grid=grid)
            for basis, order, mask in (("scalar", 2, 7), ("scalar", 3, 6), ("divfree", 2, 13)):
                w, st, F, C = oracle.stencils(pts, pts, order, basis, mask, 4, eps, rp, col)
                assert np.isfinite(w).all()
        # rank-deficient targets (fewer rows than functions) and empty rows
        pts = W.jittered_grid(200, 2, 6)
        rp, col, eps = oracle.knn(pts, pts, 4, 1.5)
        w, st, F, C = oracle.stencils(pts, pts, 2, "scalar", 4, 4, eps, rp, col)
        assert (st == 1).all()
        far = np.full((5, 2), 9.0)
        rp, col, eps = oracle.radius(pts, far, 0.05, 0)
        assert rp[-1] == 0
        print("SANITIZED-RUN-OK")
    """, rt, {"GMLS_ORACLE_LIB": ORACLE_SAN})


def test_library_abi_layer_under_sanitizers():
    """The host-only calls and the argument checks of the ABI layer: the
    stencil shapes of every (dim, order, basis, mask), and every call with a
    null or invalid context or argument (no device is needed for these)."""
    rt = clang_asan_runtime()
    if not rt or not os.path.exists(LIB_SAN):
        pytest.skip("sanitizer build of the library or the ASan runtime missing (run __graft_entry__.build())")
    run_sanitized(f"""
        import ctypes
        L = ctypes.CDLL({LIB_SAN!r})
        F, C, Q = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        seen = 0
        for dim in range(0, 5):
            for order in range(-1, 10):
                for basis in (-1, 0, 1, 2):
                    for mask in range(0, 18):
                        st = L.gmls_stencil_shape(dim, order, basis, mask, ctypes.byref(F), ctypes.byref(C),
                                                  ctypes.byref(Q))
                        seen += st == 0
        assert seen > 0
        vp = ctypes.c_void_p
        assert L.gmls_set_option(None, 0, ctypes.c_double(1.0)) != 0
        L.gmls_destroy(None)
        L.gmls_last_error.restype = ctypes.c_char_p
        assert L.gmls_last_error(None)
        assert L.gmls_check(None) != 0
        assert L.gmls_spmv(None, 10, None, None, None, None, None) != 0
        assert L.gmls_spmv_noalloc(None, 10, None, None, None, None, None) != 0
        assert L.gmls_autotune_save(None, b"/dev/null") != 0
        assert L.gmls_autotune_load(None, b"/dev/null") != 0
        h = vp()
        st = L.gmls_create(ctypes.byref(h), 10 ** 6, None)  # no such device
        assert st != 0 and not h.value
        print("SANITIZED-RUN-OK")
    """, rt, {})
