"""The C-ABI library loads and exports every function include/dwf.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dwf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\**\s*([a-z_][a-z_0-9]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dwf_dslash", "mobius_dslash", "cg_ne", "mobius_accel_solve", "fermion_force"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1111_5059_amd as dwf
    if not os.path.exists(dwf.LIB_PATH):
        pytest.fail("libdwf.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(dwf.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    # the binding covers the same set
    assert set(declared_functions()) == set(dwf.SIGNATURES)


def test_argument_validation_without_gpu():
    import paper_1111_5059_amd as dwf
    p = dwf.params((4, 4, 4, 4), 8)
    assert dwf.dwf_field_bytes(p, dwf.KIND_FULL, dwf.FP64) == 2 * 128 * 12 * 8 * 16
    assert dwf.dwf_field_bytes(p, dwf.KIND_GAUGE, dwf.FP32) == 2 * 128 * 72 * 8
    bad = dwf.params((3, 4, 4, 4), 8)
    assert dwf.dwf_field_bytes(bad, dwf.KIND_FULL, dwf.FP64) == 0
    assert dwf.lib().dwf_dslash(None, ctypes.byref(p), None, None, None, 0, 0, 0) == dwf.DWF_ERR_ARG
    assert b"ctx" in dwf.lib().dwf_last_error()
