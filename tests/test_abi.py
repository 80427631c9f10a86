"""The C ABI library loads and exports every entry point that include/gss.h
declares (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gss.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gss_[a-z_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2012_03119_amd import build, gss
    if not os.path.exists(gss.LIB_PATH):
        build.build()
    return gss.LIB_PATH


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gss_create", "gss_destroy", "gss_add_clauses", "gss_remove_clauses",
                     "gss_set_assignments", "gss_test", "gss_fetch_reports", "gss_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol(lib_path):
    from paper_2012_03119_amd import gss
    lib = gss.load_library(lib_path)
    for n in declared_functions():
        assert getattr(lib, n).argtypes is not None or n == "gss_destroy", n


def test_config_struct_layout_matches_header():
    from paper_2012_03119_amd import gss
    # num_vars, max_slots (2x4) + budget, capacity (2x8) + 4 pointers + hot_vars, reserved (2x4)
    assert ctypes.sizeof(gss.gss_config) == 8 + 16 + 4 * 8 + 8
    assert gss.REPORT_DTYPE.itemsize == 16


def test_null_context_is_rejected(lib_path):
    from paper_2012_03119_amd import gss
    lib = gss.load_library(lib_path)
    assert lib.gss_test(None, 0, None) == gss.GSS_ERR_INVALID_ARG
    assert lib.gss_remove_clauses(None, None, 0) == gss.GSS_ERR_INVALID_ARG
    lib.gss_destroy(None)  # accepted


def test_create_rejects_bad_config_without_device(lib_path):
    # argument validation happens before any HIP call
    from paper_2012_03119_amd import gss
    lib = gss.load_library(lib_path)
    for nv, ms in ((0, 64), (10, 0), (10, 100), (10, 8192)):
        cfg = gss.gss_config()
        cfg.num_vars, cfg.max_slots = nv, ms
        out = ctypes.c_void_p()
        assert lib.gss_create(ctypes.byref(cfg), ctypes.byref(out)) == gss.GSS_ERR_INVALID_ARG
        assert out.value is None
        assert lib.gss_last_error(None)
