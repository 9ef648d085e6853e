"""The C-ABI library loads without a GPU and exports every entry point that
include/m2n.h declares; the Python binding exposes the same names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "m2n.h")
LIB = os.path.join(ROOT, "paper_2407_01943_amd", "libm2n.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)       # drop comments
    src = re.sub(r"//[^\n]*", "", src)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*"
                       r"([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("m2n_create", "m2n_destroy", "m2n_last_error", "gpss_tapers",
              "m2nufft_eigcoeffs", "m2nufft_psd", "m2n_check"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libm2n.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libm2n.so not built")
def test_binding_names_match_header():
    import paper_2407_01943_amd as m2n
    for n in declared_functions():
        assert n in m2n.EXPORTED, n
    for n in ("gpss_tapers", "m2nufft_eigcoeffs", "m2nufft_psd"):
        assert callable(getattr(m2n, n))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libm2n.so not built")
def test_last_error_is_empty_string_initially():
    lib = ctypes.CDLL(LIB)
    lib.m2n_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.m2n_last_error(), bytes)
