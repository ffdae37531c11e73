"""The C-ABI library loads and exports every function include/taps.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "taps.h")
LIB = os.path.join(ROOT, "paper_2503_13933_amd", "libtaps.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(taps_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("taps_shape1d", "taps_assemble1d", "taps_contract", "taps_solve_dim",
                     "taps_reconstruct", "taps_residual"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_declared_symbol():
    from paper_2503_13933_amd import capi
    assert set(declared_functions()) == set(capi.FUNCTIONS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_gives_every_function_a_signature():
    # the loader refuses a function without argument types (ctypes would
    # otherwise pass 64-bit pointers as C ints)
    from paper_2503_13933_amd import capi
    L = capi.lib()
    for name in capi.FUNCTIONS:
        assert getattr(L, name).argtypes is not None, name
