"""The C-ABI library loads on the CPU host and exports every declared entry
point (no GPU calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sssp.h")
LIB = os.path.join(ROOT, "paper_2506_19349_amd", "libsssp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sssp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for required in ("sssp_graph_create", "sssp_solve", "sssp_solve_batch"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsssp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsssp.so not built")
def test_status_strings_and_version():
    lib = ctypes.CDLL(LIB)
    lib.sssp_status_str.restype = ctypes.c_char_p
    lib.sssp_version.restype = ctypes.c_char_p
    assert lib.sssp_status_str(0) == b"ok"
    assert lib.sssp_status_str(-2) == b"graph is not symmetric"
    assert b"gfx950" in lib.sssp_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsssp.so not built")
def test_binding_marshals_the_same_names():
    import paper_2506_19349_amd._lib as L
    for n in declared_functions():
        assert hasattr(L, n), n
