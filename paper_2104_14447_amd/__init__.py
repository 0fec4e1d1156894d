"""Python binding of libgmls (MI355X GMLS stencil generation).

Argument marshalling only: every step of neighbour search, stencil
generation and stencil application runs in the HIP kernels of
``libgmls.so``.  PyTorch supplies device memory and the stream.  There is no
CPU fallback: importing works without the library (so the package can be
inspected), but every call raises if ``libgmls.so`` is missing.

The names mirror the C ABI in ``include/libgmls.h``:
``gmls_neighbors``, ``gmls_stencil_shape``, ``gmls_stencils``, ``gmls_apply``.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "LIB_PATH", "GmlsError", "Context", "SearchSpec", "Report", "load_library",
    "gmls_neighbors", "gmls_stencil_shape", "gmls_stencils", "gmls_stencils_constrained",
    "gmls_stencils_staggered", "gmls_assemble_stokes", "gmls_spmv", "StokesStencils", "gmls_apply",
    "BASIS_SCALAR", "BASIS_DIVFREE", "F_VALUE", "F_GRAD", "F_LAPLACIAN", "F_DIV",
    "PREC_FP64", "PREC_MIXED", "SEARCH_KNN", "SEARCH_RADIUS",
    "OPT_COND_THRESHOLD", "OPT_MAX_SWEEPS", "OPT_REFINE_TOL", "OPT_FORCE_FALLBACK", "OPT_MIXED_SCHEME",
    "OPT_PIPE_CHUNK", "OPT_RADIUS_SCRATCH_MB", "OPT_CAPTURE_SAFE", "OPT_ROW_ORDER", "ROW_ORDER_CELL",
    "ROW_ORDER_INDEX", "SCHEME_AUTO", "SCHEME_ROWS", "SCHEME_GRAM", "SCHEME_PIPE", "SCHEME_WAVE",
    "OPT_PIPE_SHAPE", "OPT_SOURCE_STRIDE", "OPT_WAVE_SHAPE", "OPT_QR_SHAPE", "TUNE_SHARED", "TUNE_STAGGERED",
    "gmls_neighbors_sorted", "TuneResult", "gmls_autotune", "gmls_autotune_save", "gmls_autotune_load",
    "StencilSet", "gmls_stencils_multi", "gmls_spmv_noalloc", "NOALLOC_SPMV_MAX_ROWS",
    "EXPORTED_SYMBOLS",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgmls.so")

BASIS_SCALAR, BASIS_DIVFREE = 0, 1
F_VALUE, F_GRAD, F_LAPLACIAN, F_DIV = 1, 2, 4, 8
PREC_FP64, PREC_MIXED = 0, 1
SEARCH_KNN, SEARCH_RADIUS = 0, 1
OPT_COND_THRESHOLD, OPT_MAX_SWEEPS, OPT_REFINE_TOL, OPT_FORCE_FALLBACK = 0, 1, 2, 3
OPT_MIXED_SCHEME, OPT_PIPE_CHUNK, OPT_RADIUS_SCRATCH_MB, OPT_CAPTURE_SAFE, OPT_ROW_ORDER = 4, 5, 6, 7, 8
OPT_PIPE_SHAPE, OPT_SOURCE_STRIDE, OPT_WAVE_SHAPE, OPT_QR_SHAPE = 9, 10, 11, 12
TUNE_STAGGERED, TUNE_SHARED = 2, 3  # gmls_autotune's basis for gmls_stencils_staggered's QR kernel,
# and for gmls_stencils_multi's shared kernels
ROW_ORDER_CELL, ROW_ORDER_INDEX = 0, 1
NOALLOC_SPMV_MAX_ROWS = 1 << 23  # rows gmls_spmv_noalloc takes (its static scratch)
SCHEME_AUTO, SCHEME_ROWS, SCHEME_GRAM, SCHEME_PIPE, SCHEME_WAVE = 0, 1, 2, 3, 4
GMLS_OK, GMLS_ERR_CAPACITY, GMLS_ERR_UNSUPPORTED, GMLS_WARN_TARGET_FLAGS = 0, 4, 5, 6
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_HIP", 3: "ERR_NOMEM", 4: "ERR_CAPACITY", 5: "ERR_UNSUPPORTED",
           6: "WARN_TARGET_FLAGS"}
EXPORTED_SYMBOLS = ("gmls_create", "gmls_destroy", "gmls_last_error", "gmls_set_option", "gmls_neighbors",
                    "gmls_stencil_shape", "gmls_stencils", "gmls_stencils_constrained", "gmls_stencils_staggered",
                    "gmls_assemble_stokes", "gmls_spmv", "gmls_apply", "gmls_check", "gmls_autotune",
                    "gmls_autotune_save", "gmls_autotune_load", "gmls_stencils_multi", "gmls_spmv_noalloc",
                    "gmls_neighbors_sorted")


class GmlsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libgmls {_STATUS.get(status, status)}: {msg}")
        self.status = status


class SearchSpec(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("k", ctypes.c_int32), ("eps_mult", ctypes.c_double),
                ("radius", ctypes.c_double), ("k_min", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class StencilSet(ctypes.Structure):
    _fields_ = [("basis", ctypes.c_int32), ("functional_mask", ctypes.c_uint32), ("weights", ctypes.c_void_p),
                ("target_status", ctypes.c_void_p)]


class TuneResult(ctypes.Structure):
    """gmls_tune_result: [kernel 0 moments, 1 weights, 2 wave, 3 qr][bin][candidate]."""
    _fields_ = [(f, ctypes.c_int32 * 3 * 6 * 4) for f in ("lanes", "rows", "waves_per_simd", "lds_round",
                                                           "waves_per_cu")] + \
        [("ms", ctypes.c_float * 3 * 6 * 4), ("chosen", ctypes.c_int32 * 6 * 4)]
    KERNELS = ("moments", "weights", "wave", "qr")

    def shape(self, k, b, q):
        """The candidate's distinguishing shape: (lanes, rows per lane) for the
        pipeline, (waves per SIMD, moments per LDS round) for the wavefront
        kernel, (rows per lane, waves per SIMD compiled for (0: the
        compiler's choice), waves per CU) for the QR kernel."""
        if k < 2:
            return (self.lanes[k][b][q], self.rows[k][b][q])
        if k == 2:
            return (self.waves_per_simd[k][b][q], self.lds_round[k][b][q])
        return (self.rows[k][b][q], self.waves_per_simd[k][b][q], self.waves_per_cu[k][b][q])

    def as_dict(self):
        out = {}
        for k, kname in enumerate(self.KERNELS):
            bins = {}
            for b in range(1, 6):
                c = self.chosen[k][b]
                if c < 0:
                    continue
                bins[b] = {"chosen": self.shape(k, b, c), "candidate": c,
                           "ms": {self.shape(k, b, q): round(self.ms[k][b][q], 4) for q in range(3)}}
            if bins:
                out[kname] = bins
        return out


class StokesStencils(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("reserved", ctypes.c_int32)] + \
        [(k, ctypes.c_void_p) for k in ("row_ptr", "col", "boundary", "normals", "vlap", "grad", "plap", "plap_t",
                                         "nlap", "nlap_h")]


class Report(ctypes.Structure):
    _fields_ = [("n_targets", ctypes.c_int64), ("n_ok", ctypes.c_int64), ("n_rank_deficient", ctypes.c_int64),
                ("n_fallback", ctypes.c_int64), ("n_not_converged", ctypes.c_int64),
                ("sweep_hist", ctypes.c_int32 * 16), ("cond_max", ctypes.c_double), ("t_bin_ms", ctypes.c_double),
                ("t_stencil_ms", ctypes.c_double), ("t_fallback_ms", ctypes.c_double),
                ("cond_min", ctypes.c_double), ("cond_med", ctypes.c_double), ("t_search_ms", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "sweep_hist"}
        d["sweep_hist"] = list(self.sweep_hist)
        return d


_lib = None
_vp, _i64, _i32, _d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double


def load_library():
    """Load libgmls.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    L.gmls_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _vp]
    L.gmls_create.restype = ctypes.c_int
    L.gmls_destroy.argtypes = [_vp]
    L.gmls_destroy.restype = None
    L.gmls_last_error.argtypes = [_vp]
    L.gmls_last_error.restype = ctypes.c_char_p
    L.gmls_set_option.argtypes = [_vp, ctypes.c_int, _d]
    L.gmls_set_option.restype = ctypes.c_int
    L.gmls_neighbors.argtypes = [_vp, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.POINTER(SearchSpec), _vp, _vp, _i64,
                                 _vp, ctypes.POINTER(_i64)]
    L.gmls_neighbors.restype = ctypes.c_int
    L.gmls_neighbors_sorted.argtypes = list(L.gmls_neighbors.argtypes) + [_vp, _vp]
    L.gmls_neighbors_sorted.restype = ctypes.c_int
    L.gmls_stencil_shape.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int)]
    L.gmls_stencil_shape.restype = ctypes.c_int
    L.gmls_stencils.argtypes = [_vp, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, ctypes.POINTER(Report)]
    L.gmls_stencils.restype = ctypes.c_int
    L.gmls_apply.argtypes = [_vp, _i64, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp]
    L.gmls_apply.restype = ctypes.c_int
    L.gmls_stencils_constrained.argtypes = [_vp, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                            ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp,
                                            ctypes.POINTER(Report)]
    L.gmls_stencils_constrained.restype = ctypes.c_int
    # ctx, coords, n_src, targets, n_tgt, dim, order, mask, p, eps, row_ptr, col, prec, weights, t_weights,
    # status, report
    L.gmls_stencils_staggered.argtypes = [_vp, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                          ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp,
                                          ctypes.POINTER(Report)]
    L.gmls_stencils_staggered.restype = ctypes.c_int
    L.gmls_assemble_stokes.argtypes = [_vp, ctypes.POINTER(StokesStencils), _d, _vp, _vp, _vp, _i64,
                                       ctypes.POINTER(ctypes.c_int64)]
    L.gmls_assemble_stokes.restype = ctypes.c_int
    L.gmls_spmv.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp, _vp]
    L.gmls_spmv.restype = ctypes.c_int
    L.gmls_spmv_noalloc.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp, _vp]
    L.gmls_spmv_noalloc.restype = ctypes.c_int
    L.gmls_check.argtypes = [_vp]
    L.gmls_check.restype = ctypes.c_int
    L.gmls_autotune.argtypes = [_vp, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, ctypes.POINTER(TuneResult)]
    L.gmls_autotune.restype = ctypes.c_int
    L.gmls_stencils_multi.argtypes = [_vp, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                                      _vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(StencilSet),
                                      ctypes.POINTER(Report)]
    L.gmls_stencils_multi.restype = ctypes.c_int
    L.gmls_autotune_save.argtypes = [_vp, ctypes.c_char_p]
    L.gmls_autotune_save.restype = ctypes.c_int
    L.gmls_autotune_load.argtypes = [_vp, ctypes.c_char_p]
    L.gmls_autotune_load.restype = ctypes.c_int
    _lib = L
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _check_dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libgmls takes device tensors only")


class Context:
    """Owns a libgmls context (stream, device workspace, options)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        L = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = L.gmls_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != GMLS_OK:
            raise GmlsError(st, "gmls_create failed")
        self._h = h
        self._col_cap = 0
        self.capture_safe = False
        self.source_stride = 0

    def close(self):
        if getattr(self, "_h", None):
            load_library().gmls_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        msg = load_library().gmls_last_error(self._h).decode()
        raise GmlsError(st, msg)

    def set_option(self, option: int, value: float):
        st = load_library().gmls_set_option(self._h, option, float(value))
        if st != GMLS_OK:
            self._raise(st)
        if option == OPT_CAPTURE_SAFE:
            self.capture_safe = bool(value)
        if option == OPT_SOURCE_STRIDE:
            self.source_stride = int(value)

    def check(self):
        """Raise for errors that capture-safe calls left on the device."""
        st = load_library().gmls_check(self._h)
        if st != GMLS_OK:
            self._raise(st)


def gmls_stencil_shape(dim: int, order: int, basis: int, mask: int):
    """(F, C_in, Q) of a basis/order/functional mask."""
    F, C, Q = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    st = load_library().gmls_stencil_shape(dim, order, basis, mask, ctypes.byref(F), ctypes.byref(C), ctypes.byref(Q))
    if st != GMLS_OK:
        raise GmlsError(st, "unsupported basis/functional combination")
    return F.value, C.value, Q.value


def _neighbors(ctx, coords, targets, mode, k, eps_mult, radius, k_min, col, col_sorted, sorted_out, records=None):
    _check_dev(coords, targets)
    n_src, dim = coords.shape
    n_tgt = targets.shape[0]
    dev = coords.device
    spec = SearchSpec(mode, k, eps_mult, radius, k_min, 0)
    row_ptr = torch.empty(n_tgt + 1, dtype=torch.int64, device=dev)
    eps = torch.empty(n_tgt, dtype=torch.float64, device=dev)
    if sorted_out and records is None:
        records = torch.empty((n_src, 4), dtype=torch.float64, device=dev)
    if sorted_out and (records.shape != (n_src, 4) or records.dtype != torch.float64 or not records.is_contiguous()):
        raise ValueError("records must be a contiguous float64 tensor [n_src, 4]")
    if col is None or (sorted_out and col_sorted is None):
        if ctx.capture_safe:
            raise ValueError("capture-safe mode: pass preallocated col (and col_sorted) buffers")
        cap = n_tgt * k if mode == SEARCH_KNN else max(ctx._col_cap, n_tgt * max(k_min, 1) * 2)
        if col is None:
            col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        if sorted_out and col_sorted is None:
            col_sorted = torch.empty(col.numel(), dtype=torch.int32, device=dev)
    if sorted_out and col_sorted.numel() < col.numel():
        raise ValueError("col_sorted must hold as many entries as col")
    nnz = ctypes.c_int64()
    L = load_library()

    def call(c, cs):
        a = (ctx._h, _ptr(coords), n_src, _ptr(targets), n_tgt, dim, ctypes.byref(spec), _ptr(row_ptr), _ptr(c),
             c.numel(), _ptr(eps), ctypes.byref(nnz))
        return L.gmls_neighbors_sorted(*a, _ptr(records), _ptr(cs)) if sorted_out else L.gmls_neighbors(*a)

    st = call(col, col_sorted)
    if ctx.capture_safe:
        if st != GMLS_OK:
            ctx._raise(st)
        return row_ptr, col, eps, records, col_sorted
    if st == GMLS_ERR_CAPACITY:
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
        if sorted_out:
            col_sorted = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
        st = call(col, col_sorted)
    if st != GMLS_OK:
        ctx._raise(st)
    ctx._col_cap = max(ctx._col_cap, nnz.value)
    return row_ptr, col[: nnz.value], eps, records, (col_sorted[: nnz.value] if sorted_out else None)


def gmls_neighbors(ctx: Context, coords: torch.Tensor, targets: torch.Tensor, mode: int, k: int = 0,
                   eps_mult: float = 1.5, radius: float = 0.0, k_min: int = 0, col: torch.Tensor | None = None):
    """Neighbour lists: returns (row_ptr int64 [n_tgt+1], col int32 [nnz], eps float64 [n_tgt]).

    In capture-safe mode the total is not known on the host: the whole `col`
    buffer (which the caller must supply) is returned, row_ptr[-1] holds the
    total, and capacity errors surface through Context.check()."""
    return _neighbors(ctx, coords, targets, mode, k, eps_mult, radius, k_min, col, None, False)[:3]


def gmls_neighbors_sorted(ctx: Context, coords: torch.Tensor, targets: torch.Tensor, mode: int, k: int = 0,
                          eps_mult: float = 1.5, radius: float = 0.0, k_min: int = 0,
                          col: torch.Tensor | None = None, col_sorted: torch.Tensor | None = None,
                          records: torch.Tensor | None = None):
    """gmls_neighbors plus the search's cell-ordered source records and the
    rows as positions in them.  Returns (row_ptr, col, eps, records float64
    [n_src, 4] (x, y, z, index), col_sorted int32 [nnz]).  Stencil calls on
    (records, col_sorted) with OPT_SOURCE_STRIDE = 4 give the weights of
    (coords, col)."""
    return _neighbors(ctx, coords, targets, mode, k, eps_mult, radius, k_min, col, col_sorted, True, records)


def _source_shape(ctx: Context, coords: torch.Tensor, targets: torch.Tensor):
    """(n_src, dim) of a stencil call: dim from the targets, the coords'
    width checked against the context's source stride."""
    dim = targets.shape[1]
    stride = ctx.source_stride or dim
    if coords.dim() != 2 or coords.shape[1] != stride:
        raise ValueError(f"coords must be [n_src, {stride}] (dim {dim}, source stride option {ctx.source_stride})")
    return coords.shape[0], dim


def gmls_stencils(ctx: Context, coords: torch.Tensor, targets: torch.Tensor, order: int, basis: int, mask: int,
                  weight_p: int, eps: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor,
                  prec: int = PREC_FP64, weights: torch.Tensor | None = None, status: torch.Tensor | None = None,
                  report: bool = False):
    """Stencil weights.  Returns (weights float64, status uint8, report dict or None)."""
    _check_dev(coords, targets, eps, row_ptr, col)
    n_src, dim = _source_shape(ctx, coords, targets)
    n_tgt = targets.shape[0]
    F, C, _ = gmls_stencil_shape(dim, order, basis, mask)
    nnz = col.numel()
    if weights is None:
        weights = torch.empty(max(F * C * nnz, 1), dtype=torch.float64, device=coords.device)
    if status is None:
        status = torch.empty(max(n_tgt, 1), dtype=torch.uint8, device=coords.device)
    rep = Report()
    st = load_library().gmls_stencils(ctx._h, _ptr(coords), n_src, _ptr(targets), n_tgt, dim, order, basis, mask,
                                      weight_p, _ptr(eps), _ptr(row_ptr), _ptr(col), prec, _ptr(weights),
                                      _ptr(status), ctypes.byref(rep) if report else None)
    if st not in (GMLS_OK, GMLS_WARN_TARGET_FLAGS):
        ctx._raise(st)
    return weights[: F * C * nnz], status[:n_tgt], (rep.as_dict() if report else None)


def gmls_stencils_multi(ctx: Context, coords: torch.Tensor, targets: torch.Tensor, order: int, weight_p: int,
                        eps: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor, sets, prec: int = PREC_FP64,
                        outputs=None, report: bool = False):
    """Several (basis, functional mask) sets on the same neighbour lists.
    `sets` is a list of (basis, mask); `outputs` an optional list of
    (weights, status) tensors.  Returns ([(weights, status), ...], report)."""
    _check_dev(coords, targets, eps, row_ptr, col)
    n_src, dim = _source_shape(ctx, coords, targets)
    n_tgt = targets.shape[0]
    nnz = col.numel()
    arr = (StencilSet * len(sets))()
    outs = []
    for k, (basis, mask) in enumerate(sets):
        F, C, _ = gmls_stencil_shape(dim, order, basis, mask)
        if outputs is not None:
            w, stt = outputs[k]
        else:
            w = torch.empty(max(F * C * nnz, 1), dtype=torch.float64, device=coords.device)
            stt = torch.empty(max(n_tgt, 1), dtype=torch.uint8, device=coords.device)
        arr[k] = StencilSet(basis, mask, _ptr(w).value, _ptr(stt).value)
        outs.append((w[: F * C * nnz], stt[:n_tgt]))
    rep = Report()
    st = load_library().gmls_stencils_multi(ctx._h, _ptr(coords), n_src, _ptr(targets), n_tgt, dim, order,
                                            weight_p, _ptr(eps), _ptr(row_ptr), _ptr(col), prec, len(sets), arr,
                                            ctypes.byref(rep) if report else None)
    if st not in (GMLS_OK, GMLS_WARN_TARGET_FLAGS):
        ctx._raise(st)
    return outs, (rep.as_dict() if report else None)


def gmls_autotune(ctx: Context, coords: torch.Tensor, targets: torch.Tensor, order: int, basis: int, mask: int,
                  weight_p: int, eps: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor, reps: int = 3):
    """Autotune the per-bin shapes of the kernels this problem runs (the
    choice is kept in the context).  basis TUNE_SHARED tunes the shared
    kernels of gmls_stencils_multi; mask then holds the scalar set's mask in
    bits 0-3 and the divergence-free set's in bits 4-7.  basis TUNE_STAGGERED
    tunes the QR kernel of gmls_stencils_staggered (order: its vector order).  Returns the tuning
    result as a dict {kernel: {bin: {...}}}."""
    _check_dev(coords, targets, eps, row_ptr, col)
    n_src, dim = _source_shape(ctx, coords, targets)
    n_tgt = targets.shape[0]
    if basis == TUNE_SHARED:
        Fs, _, _ = gmls_stencil_shape(dim, order, BASIS_SCALAR, mask & 15)
        Fv, Cv, _ = gmls_stencil_shape(dim, order, BASIS_DIVFREE, (mask >> 4) & 15)
        nw, ns = (Fs + Fv * Cv) * col.numel(), 2 * n_tgt
    elif basis == TUNE_STAGGERED:
        nw, ns = ((dim if mask & F_GRAD else 0) + (1 if mask & F_LAPLACIAN else 0)) * col.numel(), n_tgt
    else:
        F, C, _ = gmls_stencil_shape(dim, order, basis, mask)
        nw, ns = F * C * col.numel(), n_tgt
    weights = torch.empty(max(nw, 1), dtype=torch.float64, device=coords.device)
    status = torch.empty(max(ns, 1), dtype=torch.uint8, device=coords.device)
    res = TuneResult()
    st = load_library().gmls_autotune(ctx._h, _ptr(coords), n_src, _ptr(targets), n_tgt, dim, order, basis, mask,
                                      weight_p, _ptr(eps), _ptr(row_ptr), _ptr(col), reps, _ptr(weights),
                                      _ptr(status), ctypes.byref(res))
    if st != GMLS_OK:
        ctx._raise(st)
    return res.as_dict()


def gmls_autotune_save(ctx: Context, path: str):
    st = load_library().gmls_autotune_save(ctx._h, os.fsencode(path))
    if st != GMLS_OK:
        ctx._raise(st)


def gmls_autotune_load(ctx: Context, path: str):
    st = load_library().gmls_autotune_load(ctx._h, os.fsencode(path))
    if st != GMLS_OK:
        ctx._raise(st)


def gmls_stencils_constrained(ctx: Context, coords: torch.Tensor, targets: torch.Tensor, order: int, mask: int,
                              weight_p: int, eps: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor,
                              normals: torch.Tensor, prec: int = PREC_FP64, weights: torch.Tensor | None = None,
                              h_weights: torch.Tensor | None = None, status: torch.Tensor | None = None,
                              report: bool = False):
    """Neumann-constrained stencils (scalar basis).  Returns (weights float64,
    h_weights float64 [n_tgt, F], status uint8, report dict or None)."""
    _check_dev(coords, targets, eps, row_ptr, col, normals)
    if normals.shape != targets.shape or normals.dtype != torch.float64 or not normals.is_contiguous():
        raise ValueError("normals must be a contiguous float64 tensor shaped like targets [n_tgt, dim]")
    n_src, dim = _source_shape(ctx, coords, targets)
    n_tgt = targets.shape[0]
    F, C, _ = gmls_stencil_shape(dim, order, BASIS_SCALAR, mask)
    nnz = col.numel()
    dev = coords.device
    if weights is None:
        weights = torch.empty(max(F * C * nnz, 1), dtype=torch.float64, device=dev)
    if h_weights is None:
        h_weights = torch.empty((max(n_tgt, 1), F), dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(max(n_tgt, 1), dtype=torch.uint8, device=dev)
    rep = Report()
    st = load_library().gmls_stencils_constrained(ctx._h, _ptr(coords), n_src, _ptr(targets), n_tgt, dim, order,
                                                  mask, weight_p, _ptr(eps), _ptr(row_ptr), _ptr(col),
                                                  _ptr(normals), prec, _ptr(weights), _ptr(h_weights),
                                                  _ptr(status), ctypes.byref(rep) if report else None)
    if st not in (GMLS_OK, GMLS_WARN_TARGET_FLAGS):
        ctx._raise(st)
    return weights[: F * C * nnz], h_weights[:n_tgt], status[:n_tgt], (rep.as_dict() if report else None)


def gmls_stencils_staggered(ctx: Context, coords: torch.Tensor, targets: torch.Tensor, order: int, mask: int,
                            weight_p: int, eps: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor,
                            prec: int = PREC_FP64, weights: torch.Tensor | None = None,
                            t_weights: torch.Tensor | None = None, status: torch.Tensor | None = None,
                            report: bool = False):
    """Staggered stencils (gradient and/or Laplacian of a scalar, vector order
    `order`).  Returns (weights float64, target weights float64 [n_tgt, F],
    status uint8, report dict or None)."""
    _check_dev(coords, targets, eps, row_ptr, col)
    n_src, dim = _source_shape(ctx, coords, targets)
    n_tgt = targets.shape[0]
    F = (dim if mask & F_GRAD else 0) + (1 if mask & F_LAPLACIAN else 0)
    nnz = col.numel()
    dev = coords.device
    if weights is None:
        weights = torch.empty(max(F * nnz, 1), dtype=torch.float64, device=dev)
    if t_weights is None:
        t_weights = torch.empty((max(n_tgt, 1), max(F, 1)), dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(max(n_tgt, 1), dtype=torch.uint8, device=dev)
    rep = Report()
    st = load_library().gmls_stencils_staggered(ctx._h, _ptr(coords), n_src, _ptr(targets), n_tgt, dim, order, mask,
                                                weight_p, _ptr(eps), _ptr(row_ptr), _ptr(col), prec, _ptr(weights),
                                                _ptr(t_weights), _ptr(status), ctypes.byref(rep) if report else None)
    if st not in (GMLS_OK, GMLS_WARN_TARGET_FLAGS):
        ctx._raise(st)
    return weights[: F * nnz], t_weights[:n_tgt], status[:n_tgt], (rep.as_dict() if report else None)


def gmls_assemble_stokes(ctx: Context, row_ptr: torch.Tensor, col: torch.Tensor, boundary: torch.Tensor,
                         normals: torch.Tensor, vlap: torch.Tensor, grad: torch.Tensor, plap: torch.Tensor,
                         plap_t: torch.Tensor, nlap: torch.Tensor, nlap_h: torch.Tensor, nu: float = 1.0):
    """Global Stokes operator from stencils (see gmls_assemble_stokes in
    libgmls.h).  Returns the CSR (row_ptr int64, col int32, val float64)."""
    _check_dev(row_ptr, col, boundary, normals, vlap, grad, plap, plap_t, nlap, nlap_h)
    n = row_ptr.numel() - 1
    dim = normals.shape[1]
    dev = row_ptr.device
    st = StokesStencils(n, dim, 0, *[_ptr(t).value for t in (row_ptr, col, boundary, normals, vlap, grad, plap,
                                                           plap_t, nlap, nlap_h)])
    rows = dim * n + n + 1
    a_rp = torch.empty(rows + 1, dtype=torch.int64, device=dev)
    cap = (dim + 1) * col.numel() + 2 * n + 1
    nnz = ctypes.c_int64()
    L = load_library()
    for _ in range(2):
        a_col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        a_val = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        rc = L.gmls_assemble_stokes(ctx._h, ctypes.byref(st), float(nu), _ptr(a_rp), _ptr(a_col), _ptr(a_val), cap,
                                    ctypes.byref(nnz))
        if rc != GMLS_ERR_CAPACITY:
            break
        cap = nnz.value
    if rc != GMLS_OK:
        ctx._raise(rc)
    return a_rp, a_col[: nnz.value], a_val[: nnz.value]


def gmls_spmv(ctx: Context, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, x: torch.Tensor,
              y: torch.Tensor | None = None):
    """y = A x for a CSR matrix (device tensors)."""
    _check_dev(row_ptr, col, val, x)
    rows = row_ptr.numel() - 1
    if y is None:
        y = torch.empty(max(rows, 1), dtype=torch.float64, device=x.device)
    st = load_library().gmls_spmv(ctx._h, rows, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y))
    if st != GMLS_OK:
        ctx._raise(st)
    return y[:rows]


def gmls_apply(ctx: Context, row_ptr: torch.Tensor, col: torch.Tensor, weights: torch.Tensor, F: int, C: int,
               field: torch.Tensor, out: torch.Tensor | None = None):
    """out[t, f] = sum_j sum_c alpha[t, f, j, c] field[col_j, c]."""
    _check_dev(row_ptr, col, weights, field)
    n_tgt = row_ptr.numel() - 1
    if out is None:
        out = torch.empty((max(n_tgt, 1), F), dtype=torch.float64, device=field.device)
    st = load_library().gmls_apply(ctx._h, n_tgt, _ptr(row_ptr), _ptr(col), _ptr(weights), F, C, _ptr(field),
                                   _ptr(out))
    if st != GMLS_OK:
        ctx._raise(st)
    return out[:n_tgt]


def gmls_spmv_noalloc(ctx: Context, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, x: torch.Tensor,
                      y: torch.Tensor):
    """y = A x like gmls_spmv, with no device allocation in the library (the
    caller passes y; the long-row list lives in the library's static scratch)."""
    _check_dev(row_ptr, col, val, x, y)
    rows = row_ptr.numel() - 1
    st = load_library().gmls_spmv_noalloc(ctx._h, rows, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y))
    if st != GMLS_OK:
        ctx._raise(st)
    return y[:rows]
