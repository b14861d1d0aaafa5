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


def test_struct_layouts_match_header_sizes():
    import ctypes
    from paper_1806_11277_amd import ehh
    # int32 dim, n[3], double h, omega, shift, int32 abl[3], double abl_max, atten0
    assert ctypes.sizeof(ehh.ehh_problem_t) == 72
    assert ctypes.sizeof(ehh.ehh_stats_t) == 8 + 24
