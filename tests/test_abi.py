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
    # num_vars, max_slots (2x4) + budget, capacity (2x8) + 4 pointers + hot_vars, timing_interval (2x4)
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
    for nv, ms in ((0, 64), (10, 0), (10, 100), (10, 64 * 64 * 64 + 64)):
        cfg = gss.gss_config()
        cfg.num_vars, cfg.max_slots = nv, ms
        out = ctypes.c_void_p()
        assert lib.gss_create(ctypes.byref(cfg), ctypes.byref(out)) == gss.GSS_ERR_INVALID_ARG
        assert out.value is None
        assert lib.gss_last_error(None)


STRUCTS = ["gss_config", "gss_stats", "gss_schedule", "gss_server_config", "gss_serve_result", "gss_sim_config",
           "gss_adam_config", "gss_priority_config"]


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the ctypes binding equals what a C
    compiler makes of include/gss.h."""
    import subprocess
    from paper_2012_03119_amd import gss
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gss.h"', "int main(void) {"]
    for s in STRUCTS:
        cls = getattr(gss, s)
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for name, _ in cls._fields_:
            lines.append(f'printf("{s}.{name} %zu\\n", offsetof({s}, {name}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    c_side = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                     text=True).stdout.splitlines())
    for s in STRUCTS:
        cls = getattr(gss, s)
        assert int(c_side[s]) == ctypes.sizeof(cls), s
        for name, _ in cls._fields_:
            assert int(c_side[f"{s}.{name}"]) == getattr(cls, name).offset, f"{s}.{name}"


def test_null_server_is_rejected(lib_path):
    from paper_2012_03119_amd import gss
    lib = gss.load_library(lib_path)
    n = ctypes.c_uint64()
    assert lib.gss_server_send(None, 0, 0, None, None, None) == gss.GSS_ERR_INVALID_ARG
    assert lib.gss_server_insert(None, 0, None, None, 0) == gss.GSS_ERR_INVALID_ARG
    assert lib.gss_server_poll(None, 0, None, 0, ctypes.byref(n), None) == gss.GSS_ERR_INVALID_ARG
    assert lib.gss_server_stop(None, None) == gss.GSS_ERR_INVALID_ARG
    assert lib.gss_server_start(None, None, None) == gss.GSS_ERR_INVALID_ARG
    assert lib.gss_serve_simulate(None, None, None) == gss.GSS_ERR_INVALID_ARG
