"""The C-ABI library loads on the CPU and exports every entry point that
include/pndf.h declares (no compute calls: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2505_08985_amd", "libpndf.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pndf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pndf_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2505_08985_amd.build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("pndf_build_mesh", "pndf_build_hierarchy", "pndf_eval_batch", "pndf_eval_hits",
                 "pndf_destroy_mesh", "pndf_destroy_hierarchy", "pndf_status_string",
                 "pndf_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    src = open(os.path.join(ROOT, "paper_2505_08985_amd", "binding.py")).read()
    missing = [n for n in declared_functions() if '"%s"' % n not in src]
    assert not missing, missing


def test_status_strings_and_null_handling(lib):
    lib.pndf_status_string.restype = ctypes.c_char_p
    lib.pndf_status_string.argtypes = [ctypes.c_int]
    assert lib.pndf_status_string(0) == b"ok"
    assert lib.pndf_status_string(4) == b"buffer too small"
    lib.pndf_last_error.restype = ctypes.c_char_p
    # argument validation happens before any device call
    lib.pndf_build_mesh.restype = ctypes.c_int
    lib.pndf_build_mesh.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]
    out = ctypes.c_void_p(1)
    assert lib.pndf_build_mesh(None, 64, 1e-6, None, ctypes.byref(out)) == 1
    assert out.value is None
    assert b"NULL" in lib.pndf_last_error()
    assert lib.pndf_build_mesh(ctypes.c_void_p(16), 48, 1e-6, None, ctypes.byref(out)) == 1
    assert lib.pndf_build_mesh(ctypes.c_void_p(16), 16384, 1e-6, None, ctypes.byref(out)) == 5
    lib.pndf_eval_batch.restype = ctypes.c_int
    lib.pndf_eval_batch.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] + [ctypes.c_void_p] * 3
    assert lib.pndf_eval_batch(None, None, 0, None, None, None) == 1
    lib.pndf_destroy_mesh.argtypes = [ctypes.c_void_p]
    lib.pndf_destroy_mesh(None)
    lib.pndf_destroy_hierarchy.argtypes = [ctypes.c_void_p]
    lib.pndf_destroy_hierarchy(None)
