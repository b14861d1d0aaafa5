"""The C ABI library loads (no GPU needed) and exports every function that
include/ehh.h declares; the ctypes binding declares the same set."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ehh.h")
LIB = os.path.join(ROOT, "paper_1806_11277_amd", "libehh.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ehh_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["ehh_setup_operator", "ehh_vcycle", "ehh_precondition", "ehh_solve", "ehh_apply",
                 "ehh_destroy", "ehh_last_error"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libehh.so not built")
def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_1806_11277_amd import ehh
    assert sorted(ehh._SIGS) == _declared()


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what gcc
    computes from include/ehh.h."""
    import ctypes
    import shutil
    import subprocess
    from paper_1806_11277_amd import ehh
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [ehh.ehh_problem_t, ehh.ehh_options_t, ehh.ehh_stats_t, ehh.ehh_kernel_time_t]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ehh.h"', 'int main(void) {']
    expect = []
    for S in structs:
        nm = S.__name__
        lines.append(f'printf("%zu\\n", sizeof({nm}));')
        expect.append(ctypes.sizeof(S))
        for f, _ in S._fields_:
            lines.append(f'printf("%zu\\n", offsetof({nm}, {f}));')
            expect.append(getattr(S, f).offset)
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == expect
