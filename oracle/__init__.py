"""FP64 CPU oracle for GMLS stencil generation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.

The arithmetic lives in ``gmls_oracle.c`` (plain C, IEEE double, built with
``-ffp-contract=off`` by ``oracle/build.py``); this module only marshals numpy
arrays.  The divergence-free basis matrix is computed here, in numpy, as an
orthonormal basis of the kernel of the divergence map (``divfree.py``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import divfree  # noqa: F401  (re-exported helper module)

_HERE = os.path.dirname(os.path.abspath(__file__))
# GMLS_ORACLE_LIB selects another build of the same source (the sanitizer
# build of oracle/build.py, loaded by the sanitizer test in a subprocess)
_LIB_PATH = os.environ.get("GMLS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

F_VALUE, F_GRAD, F_LAPLACIAN, F_DIV = 1, 2, 4, 8
BASIS = {"scalar": 0, "divfree": 1}

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def lib():
    """Load (building if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build

            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.gmls_oracle_num_monomials.argtypes = [ctypes.c_int, ctypes.c_int]
        L.gmls_oracle_monomials.argtypes = [ctypes.c_int, ctypes.c_int, _i32]
        L.gmls_oracle_num_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint]
        L.gmls_oracle_knn.argtypes = [_d, ctypes.c_int64, _d, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int, _i32, _d, ctypes.c_int]
        L.gmls_oracle_radius_count.argtypes = [_d, ctypes.c_int64, _d, ctypes.c_int64, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int]
        L.gmls_oracle_radius_fill.argtypes = [_d, ctypes.c_int64, _d, ctypes.c_int64, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_int, ctypes.c_int, _i64, _i32, _d,
                                              ctypes.c_int]
        L.gmls_oracle_stencils.argtypes = [_d, _d, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           _d, ctypes.c_int, ctypes.c_uint, ctypes.c_int, _d, _i64, _i32, _d,
                                           _u8, ctypes.c_int]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a, dim=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if dim is not None:
        a = a.reshape(-1, dim)
    return a


def monomials(dim: int, order: int) -> np.ndarray:
    """Exponents of the oracle's scalar basis, ``[Q, dim]`` int32 (graded)."""
    L = lib()
    q = L.gmls_oracle_num_monomials(dim, order)
    ex = np.zeros((q, dim), dtype=np.int32)
    L.gmls_oracle_monomials(dim, order, _p(ex, _i32))
    return ex


def num_rows(dim: int, basis: str, mask: int) -> int:
    return lib().gmls_oracle_num_rows(dim, BASIS[basis], mask)


def knn(src, tgt, k: int, eps_mult: float = 1.5, use_grid: bool | None = None, nthreads: int = 0):
    """k nearest neighbours (rows sorted by (d^2, index)); returns
    ``(row_ptr int64, col int32, eps float64)``."""
    dim = np.asarray(src).shape[1]
    src, tgt = _f64(src, dim), _f64(tgt, dim)
    n_src, n_tgt = src.shape[0], tgt.shape[0]
    if use_grid is None:
        use_grid = n_src > 5000
    col = np.zeros(n_tgt * k, dtype=np.int32)
    eps = np.zeros(n_tgt, dtype=np.float64)
    rc = lib().gmls_oracle_knn(_p(src, _d), n_src, _p(tgt, _d), n_tgt, dim, k, eps_mult, int(use_grid),
                               _p(col, _i32), _p(eps, _d), nthreads)
    if rc:
        raise ValueError(f"oracle knn failed ({rc})")
    row_ptr = np.arange(n_tgt + 1, dtype=np.int64) * k
    return row_ptr, col, eps


def radius(src, tgt, r0: float, k_min: int, use_grid: bool | None = None, nthreads: int = 0):
    """All sources with d < r0, floored to the k_min nearest (then
    eps = (d_kmin + d_kmin+1)/2); returns ``(row_ptr, col, eps)``."""
    dim = np.asarray(src).shape[1]
    src, tgt = _f64(src, dim), _f64(tgt, dim)
    n_src, n_tgt = src.shape[0], tgt.shape[0]
    if use_grid is None:
        use_grid = n_src > 5000
    L = lib()
    counts = np.zeros(n_tgt, dtype=np.int64)
    rc = L.gmls_oracle_radius_count(_p(src, _d), n_src, _p(tgt, _d), n_tgt, dim, r0, k_min, int(use_grid),
                                    _p(counts, _i64), nthreads)
    if rc:
        raise ValueError(f"oracle radius count failed ({rc})")
    row_ptr = np.zeros(n_tgt + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.zeros(max(int(row_ptr[-1]), 1), dtype=np.int32)
    eps = np.zeros(n_tgt, dtype=np.float64)
    rc = L.gmls_oracle_radius_fill(_p(src, _d), n_src, _p(tgt, _d), n_tgt, dim, r0, k_min, int(use_grid),
                                   _p(row_ptr, _i64), _p(col, _i32), _p(eps, _d), nthreads)
    if rc:
        raise ValueError(f"oracle radius fill failed ({rc})")
    return row_ptr, col[: int(row_ptr[-1])], eps


def stencils(src, tgt, order: int, basis: str, mask: int, p: int, eps, row_ptr, col, T=None,
             nthreads: int = 0):
    """Stencil weights for every target (layout: target t owns
    ``F*C*row_ptr[t]...``, entry ``(f*N + j)*C + c``).  Returns
    ``(weights float64, status uint8, F, C)``.  ``T`` defaults to the oracle's
    own orthonormal divergence-free basis."""
    dim = np.asarray(src).shape[1]
    src, tgt = _f64(src, dim), _f64(tgt, dim)
    n_tgt = tgt.shape[0]
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    b = BASIS[basis]
    F = num_rows(dim, basis, mask)
    if F <= 0:
        raise ValueError("functional not defined on this basis")
    C = 1 if b == 0 else dim
    if b == 1:
        if T is None:
            T = divfree.nullspace_basis(dim, order)
        T = np.ascontiguousarray(T, dtype=np.float64)
        Qd = T.shape[1]
    else:
        T = np.zeros(1)
        Qd = 0
    nnz = int(row_ptr[-1] - row_ptr[0]) if n_tgt else 0
    if n_tgt and row_ptr[0] != 0:
        raise ValueError("row_ptr must start at 0")
    w = np.zeros(max(F * C * nnz, 1), dtype=np.float64)
    st = np.zeros(max(n_tgt, 1), dtype=np.uint8)
    if n_tgt:
        rc = lib().gmls_oracle_stencils(_p(src, _d), _p(tgt, _d), n_tgt, dim, order, b, _p(T, _d), Qd, mask, p,
                                        _p(eps, _d), _p(row_ptr, _i64), _p(col, _i32), _p(w, _d), _p(st, _u8),
                                        nthreads)
        if rc:
            raise ValueError(f"oracle stencils failed ({rc})")
    return w[: F * C * nnz], st[:n_tgt], F, C


def subset_csr(row_ptr, col, eps, targets):
    """CSR rows of the selected targets (for computing sampled outputs one by
    one); returns ``(row_ptr, col, eps)`` of the subset."""
    targets = np.asarray(targets, dtype=np.int64)
    counts = row_ptr[targets + 1] - row_ptr[targets]
    rp = np.zeros(len(targets) + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    c = np.concatenate([col[row_ptr[t]:row_ptr[t + 1]] for t in targets]) if len(targets) else np.zeros(0, np.int32)
    return rp, c.astype(np.int32), np.asarray(eps)[targets]
