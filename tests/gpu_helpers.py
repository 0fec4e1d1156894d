"""Helpers shared by the GPU tests: device transfer, the HIP context and the
per-row relative error used by every parity gate."""
from __future__ import annotations

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2104_14447_amd as G

    G.load_library()  # raises if the HIP library is missing: no silent fallback
    return G


_CTX = {}


def ctx():
    G = require_gpu()
    if "c" not in _CTX:
        _CTX["c"] = G.Context(0)
    return _CTX["c"]


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def row_errors(w_gpu, w_ref, row_ptr, F, C, zero_rows=()):
    """Relative error per (target, functional row): ||a - b|| / ||b||.  Rows
    listed in zero_rows are identically zero; they are judged against the
    norm of row 0 of the same target."""
    errs = np.zeros((len(row_ptr) - 1, F))
    for t in range(len(row_ptr) - 1):
        n = row_ptr[t + 1] - row_ptr[t]
        a = w_gpu[F * C * row_ptr[t]: F * C * row_ptr[t + 1]].reshape(F, n * C)
        b = w_ref[F * C * row_ptr[t]: F * C * row_ptr[t + 1]].reshape(F, n * C)
        for f in range(F):
            den = np.linalg.norm(b[0] if f in zero_rows else b[f])
            errs[t, f] = np.linalg.norm(a[f] - b[f]) / den if den > 0 else np.linalg.norm(a[f] - b[f])
    return errs


def flush(msg):
    print(msg, flush=True)


def row_sorted(rp, col):
    """Each CSR row sorted ascending (radius rows compared as sets)."""
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return col[np.lexsort((col, rows))]
