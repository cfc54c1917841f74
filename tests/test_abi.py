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

    # fab_params: 5 ints, u64 seed, 2 ints, double tol, 2 ints -> 56 bytes with natural alignment
    assert ctypes.sizeof(fab.fab_params) == 56
    assert fab.fab_params.basis.offset == 48 and fab.fab_params.ls_maxit.offset == 52
    # fab_info: 7 doubles, 8 ints, 1 double -> 96 bytes
    assert ctypes.sizeof(fab.fab_info) == 96
    assert ctypes.sizeof(fab.fab_func) == 48


def test_binding_struct_layouts_match_the_c_header(tmp_path):
    """Sizes and offsets the C compiler gives the header's structs equal the binding's."""
    import shutil
    import subprocess

    from paper_2212_12758_amd import fab

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {"fab_params": fab.fab_params, "fab_info": fab.fab_info, "fab_func": fab.fab_func,
              "fab_diag": fab.fab_diag}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fab.h"', "int main(void) {"]
    for name, st in fields.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in st._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for name, st in fields.items():
        assert int(got[name]) == ctypes.sizeof(st), name
        for fname, _ in st._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(st, fname).offset, (name, fname)
