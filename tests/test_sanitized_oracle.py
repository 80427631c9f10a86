"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
CPU) and run on small cases of every mode in a child process: an out-of-bounds
access, a use of freed memory or undefined behaviour aborts the child.  Its
results must also equal the pure-Python twin's."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
OUT_DIR = os.path.join(ROOT, "_build")

CHILD = r"""
import numpy as np
import oracle
from paper_2012_03119_amd import gen


def twin(lits, offs, vals, mode, active):
    clauses = [lits[offs[i]:offs[i + 1]].tolist() for i in range(len(offs) - 1)]
    rows = oracle.py_masks(clauses, oracle.values_to_dicts(vals), mode=mode)
    out = np.array(rows, dtype=np.uint64).reshape(len(clauses), -1)
    keep = np.zeros(out.shape[1], dtype=np.uint64)
    for a in np.flatnonzero(active):
        keep[a // 64] |= np.uint64(1) << np.uint64(a % 64)
    return out & keep


rng = np.random.default_rng(3)
for seed in (1, 2):
    w = gen.tiny(seed, n_clauses=300, n_vars=80, n_slots=130, assigned=0.7)
    active = rng.random(130) < 0.8
    for mode in ("falsified", "trigger"):
        got = oracle.masks(w.lits, w.offsets, w.values, mode=mode, active=active)
        assert np.array_equal(got, twin(w.lits, w.offsets, w.values, mode, active)), (seed, mode)
# an empty clause, a unit clause, repeated literals and a tautology
lits = np.array([1, -2, 2, 3, 3, -3, 4], dtype=np.int32)
offs = np.array([0, 1, 1, 3, 5, 7], dtype=np.int64)
vals = gen.assignments_bernoulli(rng, 64, 4, 0.8)
every = np.ones(64, dtype=bool)
for mode in ("falsified", "trigger"):
    assert np.array_equal(oracle.masks(lits, offs, vals, mode=mode), twin(lits, offs, vals, mode, every)), mode
print("sanitized oracle ok")
"""


def _sanitizer_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _sanitizer_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    os.makedirs(OUT_DIR, exist_ok=True)
    lib = os.path.join(OUT_DIR, "liboracle_sanitized.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-shared", "-fPIC",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", lib, SRC])
    # The sanitizer runtime must come first; whatever the environment already preloads stays after it.
    preload = ":".join(p for p in (asan, os.environ.get("LD_PRELOAD", "")) if p)
    env = dict(os.environ, ORACLE_LIBRARY=lib, LD_PRELOAD=preload,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
