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
              "m2nufft_eigcoeffs", "m2nufft_psd", "m2n_check", "m2n_stream_status"):
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
    lib.m2n_last_error.argtypes = [ctypes.c_void_p]
    assert isinstance(lib.m2n_last_error(None), bytes)


def _header_src():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.sub(r"//[^\n]*", "", src)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libm2n.so not built")
def test_binding_argument_counts_match_header():
    # every prototype's parameter count equals the binding's argtypes length
    import paper_2407_01943_amd as m2n
    src = _header_src()
    L = m2n.lib
    checked = 0
    for name in declared_functions():
        m = re.search(r"\b" + name + r"\s*\(([^)]*)\)\s*;", src, flags=re.S)
        assert m, name
        params = m.group(1).strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        argtypes = getattr(L, name).argtypes
        if argtypes is None:
            continue
        assert len(argtypes) == n, (name, len(argtypes), n)
        checked += 1
    assert checked >= 10


def _struct_fields(tag):
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + tag + r"\s*;", _header_src(), flags=re.S).group(1)
    fields = []
    for decl in body.split(";"):
        if decl.strip():
            # "const double *t, *x" -> t, x: the last word of each declarator
            fields += [part.split()[-1].lstrip("*") for part in decl.split(",")]
    return fields


@pytest.mark.skipif(not os.path.exists(LIB), reason="libm2n.so not built")
@pytest.mark.parametrize("tag,cls", [("m2n_series", "M2NSeries"), ("m2n_subband", "M2NSubBand"),
                                     ("m2n_batch_info", "M2NBatchInfo")])
def test_structs_match_header(tag, cls):
    # the ctypes mirrors of the header's structs have its fields, in order
    import paper_2407_01943_amd as m2n
    fields = _struct_fields(tag)
    names = [f[0] for f in getattr(m2n, cls)._fields_]
    assert len(names) == len(fields), (names, fields)
    for a, b in zip(names, fields):
        assert a == b or (a, b) == ("lam", "lambda"), (a, b)
