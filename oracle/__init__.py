"""Reference computation of the GpuShareSat clause test -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library and
imports nothing from it; both sides read the same seeded inputs from the workload
generator module, which holds none of the method's arithmetic.

Two implementations of the same definitions live here:

* ``liboracle.so`` (``oracle.c``): plain C loops over clauses x assignments x
  literals, OpenMP over clauses, for inputs of any size;
* a pure-Python twin (``py_*``) on dictionaries, for tiny cases and brute force.

Definitions followed (GpuShareSat):

* Section 3.1: truth values {T, F, U}, negation with not(U) = U, literal values.
* Section 3.3, Definition 1: a clause of size s *triggers* on an assignment when
  no literal is T and at least s-1 literals are F.  Its conflict half -- every
  literal F -- is what this repository calls *falsified*.
* Section 4.2, Definitions 2-7 and Proposition 1: aggregates (subsets of
  {T, F, U}), the aggregate assignment of a group of assignments, and a clause
  triggering on an aggregate assignment.
* Section 4.3 (the group-testing procedure): test the aggregate of each group
  first and test the individual assignments of a group only where the aggregate
  test is positive.
* Section 7 (future work, aggregates of aggregates): the same procedure one
  level up, on the aggregate of several groups' aggregates.

Every function here is pinned by ``tests/test_oracle_pins.py`` against the
paper's worked examples, brute force over all partial assignments of small
clauses, and invariants; none of those pins reuses this code's arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from itertools import product
from typing import Dict, Iterable, List, Mapping, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

T, F, U = 1, -1, 0  # int8 encoding of the truth values
_NAMES = {"T": T, "F": F, "U": U}


def build(verbose: bool = False) -> str:
    """Compiles oracle.c with gcc into liboracle.so next to it (always rebuilds)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", _LIB_PATH + ".tmp", _SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    global _lib
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIBRARY")  # another build of oracle.c (e.g. with sanitizers)
        if not path:
            path = _LIB_PATH
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
                build()
        lib = ctypes.CDLL(path)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_transpose.argtypes = [i64, i64, p, p]
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        for name in ("oracle_falsified", "oracle_trigger"):
            fn = getattr(lib, name)
            fn.argtypes = [i64, p, p, i64, i64, p, p, p]
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    """Threads the C oracle runs on (OpenMP)."""
    return int(_load().oracle_max_threads())


def set_threads(n: int) -> int:
    """Runs the C oracle's loops on n threads from now on; returns the count in use."""
    return int(_load().oracle_set_threads(int(n)))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def transpose(values: np.ndarray) -> np.ndarray:
    """Slot-major int8 [n_slots][n_vars] -> var-major int8 [n_vars][n_slots]."""
    values = np.ascontiguousarray(values, dtype=np.int8)
    n_slots, n_vars = values.shape
    out = np.empty((n_vars, n_slots), dtype=np.int8)
    rc = _load().oracle_transpose(n_slots, n_vars, _ptr(values), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_transpose failed ({rc})")
    return out


def masks(lits: np.ndarray, offsets: np.ndarray, values: np.ndarray | None = None, *,
          n_vars: int | None = None, mode: str = "falsified", active: np.ndarray | None = None,
          values_vm: np.ndarray | None = None) -> np.ndarray:
    """Dense result of the C oracle: uint64 [n_clauses][ceil(n_slots/64)].

    ``values`` is slot-major int8 [n_slots][n_vars] (+1 T, -1 F, 0 U); pass the
    var-major ``values_vm`` instead to skip the transpose.  ``active`` is a
    bool/uint8 per slot (None: all slots hold an assignment).  ``mode`` is
    ``"falsified"`` (every literal F) or ``"trigger"`` (Definition 1).
    """
    lits = np.ascontiguousarray(lits, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    if values_vm is None:
        values_vm = transpose(values)
    values_vm = np.ascontiguousarray(values_vm, dtype=np.int8)
    nv, n_slots = values_vm.shape
    if n_vars is None:
        n_vars = nv
    if n_vars != nv:
        raise ValueError("n_vars does not match the values array")
    n = len(offsets) - 1
    out = np.zeros((n, (n_slots + 63) // 64), dtype=np.uint64)
    act = None
    if active is not None:
        act = np.ascontiguousarray(active, dtype=np.uint8)
        if act.shape != (n_slots,):
            raise ValueError("active must have one entry per slot")
    fn = {"falsified": _load().oracle_falsified, "trigger": _load().oracle_trigger}[mode]
    rc = fn(n, _ptr(offsets), _ptr(lits), n_vars, n_slots, _ptr(values_vm),
            _ptr(act) if act is not None else None, _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle rejected its input ({rc})")
    return out


def report_set(dense: np.ndarray, ids: np.ndarray | None = None) -> np.ndarray:
    """Sparse form of a dense mask array: rows (id, word, mask) with mask != 0,
    sorted by (id, word), as a structured array."""
    n, w = dense.shape
    if ids is None:
        ids = np.arange(n, dtype=np.uint32)
    c, k = np.nonzero(dense)
    out = np.empty(len(c), dtype=[("clause_id", "<u4"), ("word", "<u4"), ("mask", "<u8")])
    out["clause_id"] = np.asarray(ids, dtype=np.uint32)[c]
    out["word"] = k.astype(np.uint32)
    out["mask"] = dense[c, k]
    return np.sort(out, order=["clause_id", "word"])


# ---------------------------------------------------------------------------
# Pure-Python twin (tiny inputs).  An assignment is a mapping var -> 'T'/'F'/'U'
# (or +1/-1/0); a missing var is U.  A clause is a sequence of DIMACS literals.
# ---------------------------------------------------------------------------

def _tv(x) -> int:
    return _NAMES[x] if isinstance(x, str) else int(x)


def py_negate(value: int) -> int:
    """Section 3.1: not T = F, not F = T, not U = U."""
    return {T: F, F: T, U: U}[value]


def py_literal_value(assignment: Mapping[int, object], lit: int) -> int:
    """Section 3.1: A(v) for the literal v and not A(v) for the literal -v."""
    v = abs(lit)
    val = _tv(assignment.get(v, U))
    return val if lit > 0 else py_negate(val)


def py_falsified(clause: Sequence[int], assignment: Mapping[int, object]) -> bool:
    """Every literal of the clause is F under the assignment."""
    return all(py_literal_value(assignment, l) == F for l in clause)


def py_trigger(clause: Sequence[int], assignment: Mapping[int, object]) -> bool:
    """Definition 1: no literal T, and at least s-1 of the s literals F."""
    vals = [py_literal_value(assignment, l) for l in clause]
    return all(v != T for v in vals) and sum(v == F for v in vals) >= len(clause) - 1


def py_masks(clauses: Sequence[Sequence[int]], assignments: Sequence[Mapping[int, object]],
             mode: str = "falsified") -> List[List[int]]:
    """Dense masks for a list of clauses against a list of assignments (slot a =
    bit a%64 of word a//64)."""
    test = {"falsified": py_falsified, "trigger": py_trigger}[mode]
    n_words = (len(assignments) + 63) // 64
    out = []
    for c in clauses:
        row = [0] * n_words
        for a, asg in enumerate(assignments):
            if test(c, asg):
                row[a // 64] |= 1 << (a % 64)
        out.append(row)
    return out


def values_to_dicts(values: np.ndarray) -> List[Dict[int, int]]:
    """int8 [n_slots][n_vars] -> one dict per slot (var numbering from 1)."""
    return [{v + 1: int(x) for v, x in enumerate(row) if x != U} for row in values]


# ---------------------------------------------------------------------------
# Aggregates (Section 4.2) and group testing (Section 4.3), pure Python.
# ---------------------------------------------------------------------------

def py_negate_aggregate(g: Iterable[int]) -> frozenset:
    """Definition 3: the negation of an aggregate negates each of its values."""
    return frozenset(py_negate(w) for w in g)


def py_aggregate(assignments: Sequence[Mapping[int, object]], variables: Iterable[int]) -> Dict[int, frozenset]:
    """Definition 6: G(v) is the set of the values A_i(v) over the group."""
    return {v: frozenset(_tv(a.get(v, U)) for a in assignments) for v in variables}


def py_aggregate_literal(G: Mapping[int, frozenset], lit: int) -> frozenset:
    """Definition 5: G(v) for the literal v, and the negated aggregate for -v."""
    g = G[abs(lit)]
    return g if lit > 0 else py_negate_aggregate(g)


def py_trigger_aggregate(clause: Sequence[int], G: Mapping[int, frozenset]) -> bool:
    """Definition 7: every literal may be F or U, and at least s-1 literals may be F."""
    gs = [py_aggregate_literal(G, l) for l in clause]
    return all((F in g) or (U in g) for g in gs) and sum(F in g for g in gs) >= len(clause) - 1


def py_falsified_aggregate(clause: Sequence[int], G: Mapping[int, frozenset]) -> bool:
    """The conflict half of Definition 7: every literal may be F."""
    return all(F in py_aggregate_literal(G, l) for l in clause)


def py_group_test(clause: Sequence[int], groups: Sequence[Sequence[Mapping[int, object]]],
                  mode: str = "trigger") -> List[Tuple[int, int]]:
    """Group testing (Section 4.3): for each group whose aggregate test is positive,
    test the group's assignments one by one and report (group, mask) when any is
    positive.  ``mode`` selects trigger (the paper's) or its falsified half."""
    agg_test = {"trigger": py_trigger_aggregate, "falsified": py_falsified_aggregate}[mode]
    one_test = {"trigger": py_trigger, "falsified": py_falsified}[mode]
    vars_ = {abs(l) for l in clause}
    out = []
    for gi, group in enumerate(groups):
        G = py_aggregate(group, vars_)
        if not agg_test(clause, G):
            continue
        mask = 0
        for j, a in enumerate(group):
            if one_test(clause, a):
                mask |= 1 << j
        if mask:
            out.append((gi, mask))
    return out


def py_aggregate_of_aggregates(aggregates: Sequence[Mapping[int, frozenset]]) -> Dict[int, frozenset]:
    """Section 7 (future work): the aggregate of several aggregate assignments
    takes, per variable, every value any of them allows -- the aggregate
    (Definition 6) of all the assignments of their groups together."""
    out: Dict[int, frozenset] = {}
    for G in aggregates:
        for v, g in G.items():
            out[v] = out.get(v, frozenset()) | g
    return out


def py_group_test_levels(clause: Sequence[int], super_groups: Sequence[Sequence[Sequence[Mapping[int, object]]]],
                         mode: str = "trigger") -> List[Tuple[int, int, int]]:
    """Group testing one level up (Section 4.3 applied to aggregates, as Section 7
    proposes): a super-group is a list of groups of assignments.  Test the clause
    on the aggregate of each super-group's group aggregates; where that is
    positive, on each group's aggregate; where that is positive, on the group's
    assignments one by one.  Reports (super-group, group, mask) for every group
    with a positive assignment."""
    agg_test = {"trigger": py_trigger_aggregate, "falsified": py_falsified_aggregate}[mode]
    one_test = {"trigger": py_trigger, "falsified": py_falsified}[mode]
    vars_ = {abs(l) for l in clause}
    out = []
    for si, groups in enumerate(super_groups):
        aggs = [py_aggregate(group, vars_) for group in groups]
        if not aggs or not agg_test(clause, py_aggregate_of_aggregates(aggs)):
            continue
        for gi, (group, G) in enumerate(zip(groups, aggs)):
            if not agg_test(clause, G):
                continue
            mask = 0
            for j, a in enumerate(group):
                if one_test(clause, a):
                    mask |= 1 << j
            if mask:
                out.append((si, gi, mask))
    return out


def all_partial_assignments(variables: Sequence[int]):
    """Every map from the variables to {T, F, U} (3^n of them)."""
    for vals in product((T, F, U), repeat=len(variables)):
        yield dict(zip(variables, vals))
