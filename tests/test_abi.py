"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and the pure host call (stencil shape)
gives the dimensions of Sections 2.1-2.2."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libgmls.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(gmls_\w+)\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    assert names == sorted(["gmls_create", "gmls_destroy", "gmls_last_error", "gmls_set_option", "gmls_neighbors",
                            "gmls_stencil_shape", "gmls_stencils", "gmls_stencils_constrained",
                            "gmls_stencils_staggered", "gmls_assemble_stokes", "gmls_spmv", "gmls_apply",
                            "gmls_check", "gmls_autotune", "gmls_autotune_save", "gmls_autotune_load",
                            "gmls_stencils_multi", "gmls_spmv_noalloc", "gmls_neighbors_sorted"])


def test_library_exports_every_declared_symbol():
    import paper_2104_14447_amd as G

    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libgmls.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", G.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gmls_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
    L = G.load_library()
    for name in G.EXPORTED_SYMBOLS:
        assert hasattr(L, name)


def test_library_has_no_unresolved_internal_symbols():
    import paper_2104_14447_amd as G

    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libgmls.so not built")
    out = subprocess.run(["nm", "-D", "--undefined-only", G.LIB_PATH], capture_output=True, text=True).stdout
    assert "gmls" not in out, out


@pytest.mark.parametrize("dim,order,basis,mask,expect", [
    (2, 2, 0, 2 | 4, (3, 1, 6)),
    (2, 4, 0, 1 | 2 | 4, (4, 1, 15)),
    (3, 2, 1, 4, (3, 3, 26)),
    (3, 3, 0, 4, (1, 1, 20)),
    (3, 4, 0, 2 | 4, (4, 1, 35)),
    (3, 4, 1, 4 | 8, (4, 3, 85)),
    (2, 2, 1, 1 | 4 | 8, (5, 2, 9)),
])
def test_stencil_shape(dim, order, basis, mask, expect):
    import paper_2104_14447_amd as G

    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libgmls.so not built")
    assert G.gmls_stencil_shape(dim, order, basis, mask) == expect


def test_stencil_shape_rejects_undefined_functionals():
    import paper_2104_14447_amd as G

    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libgmls.so not built")
    with pytest.raises(G.GmlsError):
        G.gmls_stencil_shape(3, 2, 0, 8)  # divergence of a scalar basis
    with pytest.raises(G.GmlsError):
        G.gmls_stencil_shape(3, 2, 1, 2)  # gradient of a vector basis


def test_null_context_is_rejected():
    import paper_2104_14447_amd as G

    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libgmls.so not built")
    L = G.load_library()
    assert L.gmls_set_option(None, 0, 1.0) == 1
    assert L.gmls_last_error(None) == b"null context"
    assert L.gmls_autotune_save(None, b"/nonexistent") == 1
    assert L.gmls_autotune_load(None, b"/nonexistent") == 1


def test_product_package_has_no_oracle_dependency():
    """The product path never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2104_14447_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f
