"""The C-ABI library loads and exports every entry point include/fab.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fab.h")
LIB = os.path.join(ROOT, "paper_2212_12758_amd", "libfab.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(fab_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fab_init", "fab_create_matrix_stencil", "fab_create_matrix_csr", "fab_destroy_matrix",
                 "fab_solve", "fab_submit", "fab_poll", "fab_wait", "fab_finalize", "fab_strerror"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfab.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.fab_strerror.restype = ctypes.c_char_p
    assert lib.fab_strerror(0) == b"ok"
    lib.fab_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.fab_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfab.so not built")
def test_binding_marshalling_matches_header_struct_sizes():
    from paper_2212_12758_amd import fab

    # fab_params: 5 ints, u64 seed, 2 ints, double tol -> 48 bytes with natural alignment
    assert ctypes.sizeof(fab.fab_params) == 48
    # fab_info: 7 doubles, 5 ints (+4 padding), 1 double -> 88 bytes
    assert ctypes.sizeof(fab.fab_info) == 88
    assert ctypes.sizeof(fab.fab_func) == 48
