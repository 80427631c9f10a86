"""Pins of the oracle to facts outside itself (CPU only).

* the paper's worked examples (tests/golden/, each file cites its passage);
* brute force over every clause on up to four distinct variables and every
  partial assignment, against semantic definitions (all total extensions, and
  the restriction of the clause to the assignment);
* invariants that hold for any input (hypothesis);
* Theorem 1 (an individual trigger implies an aggregate trigger);
* planted pairs of the seeded workloads, and the expected number of chance hits
  from the workload's closed form;
* an independent numpy formulation on the tiny workload.
"""
import itertools

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from golden_fixtures import all_files, load
from paper_2012_03119_amd import gen

T, F, U = 1, -1, 0


def _values_from_dicts(assignments, n_vars):
    vals = np.zeros((len(assignments), n_vars), dtype=np.int8)
    for a, asg in enumerate(assignments):
        for v, x in asg.items():
            vals[a, v - 1] = x
    return vals


def _csr(clauses):
    offsets = np.zeros(len(clauses) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(c) for c in clauses])
    lits = np.array([l for c in clauses for l in c], dtype=np.int32)
    return lits, offsets


def _bits(row, n):
    return [int((int(row[a // 64]) >> (a % 64)) & 1) for a in range(n)]


# ---------------------------------------------------------------------------
# worked examples
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", all_files())
def test_golden_examples(name):
    g = load(name)
    asg, n_vars = g["assignments"], g["n_vars"]
    values = _values_from_dicts(asg, n_vars)
    if g["aggregate"] is not None:
        assert oracle.py_aggregate(asg, g["aggregate"].keys()) == g["aggregate"]
    if not g["clauses"]:
        return
    lits, offsets = _csr([c for c, _ in g["clauses"]])
    c_masks = {m: oracle.masks(lits, offsets, values, mode=m) for m in ("falsified", "trigger")}
    for i, (clause, expect) in enumerate(g["clauses"]):
        for key, want in expect.items():
            if key in ("trigger_aggregate", "falsified_aggregate"):
                G = oracle.py_aggregate(asg, {abs(l) for l in clause})
                fn = oracle.py_trigger_aggregate if key == "trigger_aggregate" else oracle.py_falsified_aggregate
                assert [int(fn(clause, G))] == want, (name, clause, key)
                continue
            py = oracle.py_trigger if key == "trigger" else oracle.py_falsified
            assert [int(py(clause, a)) for a in asg] == want, (name, clause, key, "python")
            assert _bits(c_masks[key][i], len(asg)) == want, (name, clause, key, "C")


# ---------------------------------------------------------------------------
# brute force against semantic definitions
# ---------------------------------------------------------------------------

def _semantic_falsified(clause, asg):
    """Falsified <=> the clause is false under every total extension of asg."""
    free = sorted({abs(l) for l in clause if asg.get(abs(l), U) == U})
    for bits in itertools.product((T, F), repeat=len(free)):
        full = dict(asg)
        full.update(zip(free, bits))
        if any((full[abs(l)] == T) == (l > 0) for l in clause):
            return False  # some extension satisfies a literal
    return True


def _semantic_trigger(clause, asg):
    """Trigger <=> the clause restricted to asg is not satisfied and keeps at most
    one literal (clauses here have distinct variables)."""
    rest = []
    for l in clause:
        x = asg.get(abs(l), U)
        if x == U:
            rest.append(l)
        elif (x == T) == (l > 0):
            return False  # satisfied
    return len(rest) <= 1


def _all_clauses(vars_):
    out = []
    for signs in itertools.product((0, 1, -1), repeat=len(vars_)):
        c = [s * v for s, v in zip(signs, vars_) if s != 0]
        if c:
            out.append(c)
    return out


def test_bruteforce_four_vars():
    vars_ = [1, 2, 3, 4]
    clauses = _all_clauses(vars_)
    assert len(clauses) == 80
    asgs = list(oracle.all_partial_assignments(vars_))
    assert len(asgs) == 81
    values = _values_from_dicts(asgs, 4)
    lits, offsets = _csr(clauses)
    fals = oracle.masks(lits, offsets, values, mode="falsified")
    trig = oracle.masks(lits, offsets, values, mode="trigger")
    for i, c in enumerate(clauses):
        want_f = [int(_semantic_falsified(c, a)) for a in asgs]
        want_t = [int(_semantic_trigger(c, a)) for a in asgs]
        assert _bits(fals[i], 81) == want_f, c
        assert _bits(trig[i], 81) == want_t, c
        assert [int(oracle.py_falsified(c, a)) for a in asgs] == want_f, c
        assert [int(oracle.py_trigger(c, a)) for a in asgs] == want_t, c


def test_bruteforce_active_mask_and_word_edges():
    # 130 slots (three words, ragged); inactive slots give 0 bits in both modes.
    rng = np.random.default_rng(7)
    values = rng.integers(-1, 2, size=(130, 6)).astype(np.int8)
    active = rng.random(130) < 0.7
    clauses = [[1], [-2, 3], [4, -5, 6], [1, 2, 3, 4, 5, 6]]
    lits, offsets = _csr(clauses)
    for mode, py in (("falsified", oracle.py_falsified), ("trigger", oracle.py_trigger)):
        got = oracle.masks(lits, offsets, values, mode=mode, active=active)
        dicts = oracle.values_to_dicts(values)
        for i, c in enumerate(clauses):
            want = [int(active[a] and py(c, dicts[a])) for a in range(130)]
            assert _bits(got[i], 130) == want
            assert int(got[i][2]) >> 2 == 0  # bits beyond slot 129


def test_rejects_bad_literals():
    values = np.zeros((3, 4), dtype=np.int8)
    for bad in ([0], [5], [-5], [1, 2, 9]):
        lits, offsets = _csr([bad])
        with pytest.raises(ValueError):
            oracle.masks(lits, offsets, values)


# ---------------------------------------------------------------------------
# invariants (hypothesis)
# ---------------------------------------------------------------------------

N_VARS = 8


@st.composite
def instance(draw, max_slots=70):
    n_slots = draw(st.integers(1, max_slots))
    vals = draw(st.lists(st.lists(st.sampled_from([T, F, U]), min_size=N_VARS, max_size=N_VARS),
                         min_size=n_slots, max_size=n_slots))
    clause = draw(st.lists(st.integers(1, N_VARS).flatmap(lambda v: st.sampled_from([v, -v])),
                           min_size=1, max_size=10))
    return np.array(vals, dtype=np.int8), clause


def _one(clause, values, mode="falsified"):
    lits, offsets = _csr([clause])
    return oracle.masks(lits, offsets, values, mode=mode)[0]


def _bitset(row, n):
    return {a for a in range(n) if (int(row[a // 64]) >> (a % 64)) & 1}


@settings(max_examples=200, deadline=None)
@given(instance())
def test_invariant_all_undef(inst):
    values, clause = inst
    zero = np.zeros_like(values)
    assert not _bitset(_one(clause, zero), len(values))
    if len(clause) >= 2:
        assert not _bitset(_one(clause, zero, "trigger"), len(values))


@settings(max_examples=200, deadline=None)
@given(instance(), st.integers(1, N_VARS))
def test_invariant_tautology(inst, v):
    values, clause = inst
    taut = clause + [v, -v]
    assert not _bitset(_one(taut, values), len(values))
    assert not _bitset(_one(taut, values, "trigger"), len(values))


@settings(max_examples=200, deadline=None)
@given(instance(), st.data())
def test_invariant_extension_only_adds(inst, data):
    values, clause = inst
    ext = values.copy()
    undef = np.argwhere(ext == U)
    for (a, v) in undef:
        if data.draw(st.booleans()):
            ext[a, v] = data.draw(st.sampled_from([T, F]))
    n = len(values)
    assert _bitset(_one(clause, values), n) <= _bitset(_one(clause, ext), n)


@settings(max_examples=200, deadline=None)
@given(instance(), st.randoms(use_true_random=False))
def test_invariant_literal_order(inst, rnd):
    values, clause = inst
    perm = list(clause)
    rnd.shuffle(perm)
    for mode in ("falsified", "trigger"):
        assert _bitset(_one(clause, values, mode), len(values)) == _bitset(_one(perm, values, mode), len(values))


@settings(max_examples=200, deadline=None)
@given(instance(), st.randoms(use_true_random=False))
def test_invariant_slot_permutation(inst, rnd):
    values, clause = inst
    n = len(values)
    perm = list(range(n))
    rnd.shuffle(perm)
    for mode in ("falsified", "trigger"):
        base = _bitset(_one(clause, values, mode), n)
        moved = _bitset(_one(clause, values[perm], mode), n)
        assert moved == {i for i in range(n) if perm[i] in base}


@settings(max_examples=200, deadline=None)
@given(instance())
def test_invariant_global_negation(inst):
    values, clause = inst
    n = len(values)
    for mode in ("falsified", "trigger"):
        assert _bitset(_one(clause, values, mode), n) == _bitset(_one([-l for l in clause], -values, mode), n)


@settings(max_examples=200, deadline=None)
@given(instance(), st.lists(st.integers(1, N_VARS).flatmap(lambda v: st.sampled_from([v, -v])), max_size=5))
def test_invariant_superset_clause(inst, extra):
    values, clause = inst
    n = len(values)
    assert _bitset(_one(clause + extra, values), n) <= _bitset(_one(clause, values), n)


@settings(max_examples=150, deadline=None)
@given(instance(max_slots=12), st.integers(1, 4))
def test_theorem1_individual_implies_aggregate(inst, n_groups):
    values, clause = inst
    dicts = oracle.values_to_dicts(values)
    groups = [dicts[g::n_groups] for g in range(n_groups)]
    vars_ = {abs(l) for l in clause}
    for group in groups:
        if not group:
            continue
        G = oracle.py_aggregate(group, vars_)
        if any(oracle.py_trigger(clause, a) for a in group):
            assert oracle.py_trigger_aggregate(clause, G)
        if any(oracle.py_falsified(clause, a) for a in group):
            assert oracle.py_falsified_aggregate(clause, G)
    # group testing finds exactly the individual results (no false negatives)
    for mode, one in (("trigger", oracle.py_trigger), ("falsified", oracle.py_falsified)):
        got = dict(oracle.py_group_test(clause, groups, mode))
        for gi, group in enumerate(groups):
            mask = sum(1 << j for j, a in enumerate(group) if one(clause, a))
            assert got.get(gi, 0) == mask


# ---------------------------------------------------------------------------
# aggregate tests (Section 4.2, Definition 7) by enumeration of choices
# ---------------------------------------------------------------------------

_SUBSETS = [frozenset(s) for r in (1, 2, 3) for s in itertools.combinations((T, F, U), r)]


def _choices(G, vars_):
    """Every assignment that takes, for each variable, one value of its aggregate."""
    for vals in itertools.product(*(sorted(G[v]) for v in vars_)):
        yield dict(zip(vars_, vals))


def _clauses_over(vars_, max_len):
    """Every clause of 1..max_len literals over the variables (repeats allowed)."""
    lits = [l for v in vars_ for l in (v, -v)]
    for n in range(1, max_len + 1):
        yield from itertools.combinations_with_replacement(lits, n)


def test_aggregate_tests_by_enumeration():
    """For a clause whose variables are distinct, the aggregate test is positive
    exactly when some assignment drawing each variable's value from its aggregate
    is positive: a literal that may be F can be made F independently of the
    others.  For any clause (repeats included) each literal is looked at on its
    own: the falsified half is positive exactly when every literal is F under
    some such assignment, and the trigger test exactly when every literal is F
    or U under some assignment and at most one literal is F under none."""
    for n_vars in (1, 2, 3):
        vars_ = list(range(1, n_vars + 1))
        choices_by_G = {}
        for gs in itertools.product(_SUBSETS, repeat=n_vars):
            G = dict(zip(vars_, gs))
            choices_by_G[gs] = (G, list(_choices(G, vars_)))
        for clause in _clauses_over(vars_, 3):
            distinct = len({abs(l) for l in clause}) == len(clause)
            for G, choices in choices_by_G.values():
                fa = oracle.py_falsified_aggregate(clause, G)
                ta = oracle.py_trigger_aggregate(clause, G)
                if distinct:
                    assert fa == any(oracle.py_falsified(clause, a) for a in choices), (clause, G)
                    assert ta == any(oracle.py_trigger(clause, a) for a in choices), (clause, G)
                vals = [[oracle.py_literal_value(a, l) for a in choices] for l in clause]
                assert fa == all(F in v for v in vals), (clause, G)
                not_f = sum(F not in v for v in vals)
                assert ta == (all((F in v) or (U in v) for v in vals) and not_f <= 1), (clause, G)


def test_aggregate_of_a_group_is_tight():
    """Every aggregate assignment over distinct variables is the aggregate of the
    group of all its choices, and for such a group the aggregate test is positive
    exactly when some member of the group is (the converse of Theorem 1 fails
    only across members, as Example 5 shows, never within one member)."""
    vars_ = [1, 2]
    for gs in itertools.product(_SUBSETS, repeat=2):
        G = dict(zip(vars_, gs))
        group = list(_choices(G, vars_))
        assert oracle.py_aggregate(group, vars_) == G
        for clause in ([1, 2], [1, -2], [-1, -2], [1], [-2]):
            assert oracle.py_falsified_aggregate(clause, G) == any(oracle.py_falsified(clause, a) for a in group)


@settings(max_examples=120, deadline=None)
@given(instance(max_slots=16), st.integers(1, 3), st.integers(1, 3))
def test_three_level_group_testing(inst, n_super, n_groups):
    """The aggregate of the group aggregates is the aggregate of all the
    super-group's assignments; a positive individual makes its group aggregate
    and its super-group aggregate positive (Theorem 1 twice); and three-level
    group testing finds exactly the individual results."""
    values, clause = inst
    dicts = oracle.values_to_dicts(values)
    vars_ = {abs(l) for l in clause}
    sgs = [[dicts[s::n_super][g::n_groups] for g in range(n_groups)] for s in range(n_super)]
    for mode, one, agg in (("trigger", oracle.py_trigger, oracle.py_trigger_aggregate),
                           ("falsified", oracle.py_falsified, oracle.py_falsified_aggregate)):
        got = {(s, g): m for s, g, m in oracle.py_group_test_levels(clause, sgs, mode)}
        for si, groups in enumerate(sgs):
            members = [a for group in groups for a in group]
            if not members:
                continue
            top = oracle.py_aggregate_of_aggregates([oracle.py_aggregate(group, vars_) for group in groups if group])
            assert top == oracle.py_aggregate(members, vars_)
            if any(one(clause, a) for a in members):
                assert agg(clause, top)
            for gi, group in enumerate(groups):
                mask = sum(1 << j for j, a in enumerate(group) if one(clause, a))
                assert got.get((si, gi), 0) == mask


def test_three_level_filters_at_the_top():
    """A super-group whose aggregate test is negative is not looked into: with the
    top-level test replaced by one that is always negative, nothing is found,
    while the individuals are positive (the filter is really applied)."""
    clause = [1, 2]
    sgs = [[[{1: F, 2: F}], [{1: T, 2: F}]]]
    assert oracle.py_group_test_levels(clause, sgs, "falsified") == [(0, 0, 1)]
    real = oracle.py_falsified_aggregate
    calls = []

    def spy(c, G):
        calls.append(G)
        return real(c, G)

    oracle.py_falsified_aggregate = spy
    try:
        oracle.py_group_test_levels(clause, sgs, "falsified")
    finally:
        oracle.py_falsified_aggregate = real
    # the top-level aggregate is tested first: A may be T or F, B only F
    assert calls[0] == {1: frozenset({T, F}), 2: frozenset({F})}


# ---------------------------------------------------------------------------
# seeded workloads: planted pairs, chance hits, an independent formulation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_planted_pairs_reported(seed):
    w = gen.tiny(seed)
    m = oracle.masks(w.lits, w.offsets, w.values)
    for c, a in w.planted.tolist():
        assert (int(m[c, a // 64]) >> (a % 64)) & 1, (c, a)


def test_chance_hits_match_closed_form():
    # Tiny workload: a literal is F with probability 0.6 * 1/2 = 0.3 per slot, so an
    # unplanted clause of length L is falsified by a slot with probability 0.3**L.
    hits, expect, var = 0, 0.0, 0.0
    for seed in range(1, 6):
        w = gen.tiny(seed)
        m = oracle.masks(w.lits, w.offsets, w.values)
        planted = np.zeros(w.n_clauses, dtype=bool)
        planted[w.planted[:, 0]] = True
        p = 0.3 ** w.lengths[~planted].astype(np.float64)
        expect += 64 * p.sum()
        var += 64 * (p * (1 - p)).sum()
        hits += sum(bin(int(x)).count("1") for x in m[~planted, 0])
    assert abs(hits - expect) < 5 * np.sqrt(var), (hits, expect, np.sqrt(var))


def _numpy_falsified(lits, offsets, values):
    """Independent formulation: gather every literal's value per slot with numpy
    and require all of them F."""
    n = len(offsets) - 1
    n_slots = values.shape[0]
    out = np.zeros((n, (n_slots + 63) // 64), dtype=np.uint64)
    for c in range(n):
        cl = lits[offsets[c]:offsets[c + 1]]
        lv = values[:, np.abs(cl) - 1] * np.sign(cl)[None, :]   # literal values per slot
        hit = np.all(lv == F, axis=1)
        for a in np.flatnonzero(hit):
            out[c, a // 64] |= np.uint64(1) << np.uint64(a % 64)
    return out


def test_numpy_formulation_tiny():
    w = gen.tiny(4, n_clauses=3000)
    np.testing.assert_array_equal(oracle.masks(w.lits, w.offsets, w.values), _numpy_falsified(w.lits, w.offsets, w.values))


def test_python_twin_matches_c_on_random():
    rng = np.random.default_rng(11)
    values = rng.integers(-1, 2, size=(100, 12)).astype(np.int8)
    clauses = [list(rng.choice(np.arange(1, 13), size=rng.integers(1, 7), replace=True) * rng.choice([-1, 1], size=1))
               for _ in range(60)]
    clauses = [[int(x) for x in c] for c in clauses]
    lits, offsets = _csr(clauses)
    dicts = oracle.values_to_dicts(values)
    for mode in ("falsified", "trigger"):
        got = oracle.masks(lits, offsets, values, mode=mode)
        want = oracle.py_masks(clauses, dicts, mode=mode)
        assert [[int(x) for x in row] for row in got] == want


def test_special_case_unit_and_binary():
    # s = 1: the mask is the set of slots where the literal is F; s = 2: the AND of two.
    w = gen.tiny(5, n_clauses=10)
    vals = w.values
    for v in (1, 17, 1999):
        for sign in (1, -1):
            m = oracle.masks(np.array([sign * v], np.int32), np.array([0, 1], np.int64), vals)[0, 0]
            want = sum(1 << a for a in range(64) if vals[a, v - 1] == -sign)
            assert int(m) == want
    a_bits = lambda v, s: sum(1 << a for a in range(64) if vals[a, v - 1] == -s)
    m = oracle.masks(np.array([3, -40], np.int32), np.array([0, 2], np.int64), vals)[0, 0]
    assert int(m) == a_bits(3, 1) & a_bits(40, -1)


def test_thread_count_does_not_change_results():
    # the timing leg runs the oracle on one thread as well: same masks in both modes
    w = gen.tiny(6, n_clauses=4000)
    cores = oracle.max_threads()
    want = {m: oracle.masks(w.lits, w.offsets, w.values, mode=m) for m in ("falsified", "trigger")}
    try:
        assert oracle.set_threads(1) == 1
        for m, x in want.items():
            np.testing.assert_array_equal(oracle.masks(w.lits, w.offsets, w.values, mode=m), x)
    finally:
        oracle.set_threads(cores)
    assert oracle.max_threads() == cores
