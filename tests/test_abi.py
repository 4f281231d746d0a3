"""The C-ABI library loads and exports every entry point declared in include/spfd.h (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spfd.h")
LIB = os.path.join(ROOT, "paper_2010_12879_amd", "libspfd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spfd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["spfd_create", "spfd_destroy", "spfd_set_geometry", "spfd_set_sigma_table", "spfd_build",
              "spfd_set_source", "spfd_solve", "spfd_efield"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspfd.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (same HIP runtime as in use)
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n
    import paper_2010_12879_amd as P
    assert set(P.EXPORTS) >= set(n for n in declared_functions() if n in P.EXPORTS)
    for n in declared_functions():
        assert hasattr(P, n), f"python binding lacks {n}"


def test_binding_refuses_without_library(tmp_path):
    import paper_2010_12879_amd as P
    saved = P._lib
    P._lib = None
    try:
        with pytest.raises(RuntimeError):
            P.load_library(str(tmp_path / "missing.so"))
    finally:
        P._lib = saved


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspfd.so not built")
def test_create_rejects_half_an_allocator():
    # argument validation only (returns before any device call): alloc without free
    import paper_2010_12879_amd as P
    P.load_library()
    half = P.Allocator()
    half.alloc = P._ALLOC_FN(lambda n, u: None)
    h = ctypes.c_void_p()
    st = P._lib.spfd_create(0, None, ctypes.byref(half), ctypes.byref(h))
    assert st == 1 and not h.value
