"""The C-ABI library loads and exports every entry point that include/nd.h
declares.  CPU only: nothing is called that needs a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nd.h")
LIB = os.path.join(ROOT, "paper_1704_00386_amd", "libnd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(nd_[a-z0-9_]+)\s*\(", text)
    # drop the callback typedef name
    return sorted(set(names) - {"nd_iter_cb"})


def test_header_declares_expected_surface():
    names = declared_functions()
    for must in ("nd_ctx_create", "nd_graph_from_edges", "nd_graph_from_csr",
                 "nd_prepare", "nd_decompose", "nd_update", "nd_incidence",
                 "nd_batch_decompose", "nd_server_submit", "nd_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libnd.so is not built (python paper_1704_00386_amd/build.py)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.nd_status_str.restype = ctypes.c_char_p
    assert lib.nd_status_str(0) == b"ok"
    assert lib.nd_status_str(5) == b"not converged"
