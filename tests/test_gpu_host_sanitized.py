"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`paper_2012_03119_amd.build.build_sanitized` (run by `__graft_entry__.build`)
builds a copy of the library whose host passes are instrumented, and a driver
(tests/sanitize/host_driver.cpp) built with the same sanitizers that exercises
the C ABI on small stores: every test mode and fetch, host, device, packed and
queued deltas, removals with compaction, ranking, the allocation-free test, the
learned priority, a batch of two stores and a served session with late and
partial polls, each plain test compared with the C oracle.  The run aborts on a
host access out of bounds, a use of freed memory or undefined behaviour.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

DRIVER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sanitize", "host_driver")


def test_library_host_code_under_asan_and_ubsan():
    if not os.path.exists(DRIVER):
        pytest.skip("the sanitized driver is not built (paper_2012_03119_amd.build.build_sanitized)")
    env = dict(os.environ)
    # leaks are not checked: the HIP runtime keeps allocations until the process ends
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    print("[sanitize] running the host-sanitized driver", flush=True)
    r = subprocess.run([DRIVER], env=env, capture_output=True, text=True, timeout=240)
    print(r.stdout[-4000:])
    print(r.stderr[-4000:])
    assert r.returncode == 0, f"driver exited with {r.returncode}"
    assert "host sanitizer run: ok" in r.stdout
