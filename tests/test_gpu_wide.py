"""Rows wider than 4096 slots and the aggregate of aggregates (GPU).

With more than 64 words a plane row is stored in chunks of 64 words, each chunk a
super-group of 4096 slots; the aggregate pre-test then runs on three levels
(super-group, word, slot), the extension Section 7 proposes.  Every test compares
the HIP path with the oracle's dense masks, bit for bit, at 8192 and 32768 slots
and at widths whose last chunk is partly or wholly unused, in both modes, with
and without the aggregate pre-test, after full sets, var-major deltas, packed
word deltas in every chunk and cleared slots.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import full_values, gpu_dense, mismatch_summary
from paper_2012_03119_amd import gen, gss

pytestmark = pytest.mark.gpu

FLAGS = [("falsified", 0), ("falsified", gss.GSS_TEST_AGGREGATE), ("trigger", gss.GSS_TEST_TRIGGER),
         ("trigger", gss.GSS_TEST_TRIGGER | gss.GSS_TEST_AGGREGATE)]


def _clauses(seed, n, n_vars):
    rng = np.random.default_rng(seed)
    # short clauses (hits even where aggregates are selective) and some long ones
    lengths = np.where(rng.random(n) < 0.85, rng.integers(1, 4, n), rng.integers(4, 40, n))
    return gen.random_clauses(rng, lengths, n_vars)


def _values(seed, n_slots, n_vars):
    n_super = (n_slots + 4095) // 4096
    v = gen.assignments_hierarchical(np.random.default_rng(seed), n_super, n_vars)
    return v[:n_slots]


def _check_all(ctx, lits, offsets, vals, active, n):
    for mode, flags in FLAGS:
        got = gpu_dense(ctx, n, flags)
        want = oracle.masks(lits, offsets, vals, mode=mode, active=active)
        assert np.array_equal(got, want), f"{mode} flags={flags}: " + mismatch_summary(got, want)
    assert ctx.test(gss.GSS_TEST_DENSE) == 0
    got = ctx.fetch_masks(np.arange(n, dtype=np.uint32))
    want = oracle.masks(lits, offsets, vals, active=active)
    assert np.array_equal(got, want), "dense: " + mismatch_summary(got, want)


@pytest.mark.parametrize("max_slots", [8192, 32768])
def test_wide_rows_all_modes(max_slots):
    n_vars, n = 700, 3000
    print(f"wide max_slots={max_slots}", flush=True)
    lits, offsets = _clauses(max_slots, n, n_vars)
    vals = _values(max_slots + 1, max_slots, n_vars)
    active = np.ones(max_slots, dtype=bool)
    with gss.Context(n_vars, max_slots, report_capacity=1 << 20) as ctx:
        ctx.add_clauses(lits, offsets)
        ctx.set_assignments(0, vals)
        _check_all(ctx, lits, offsets, vals, active, n)


def test_maximum_width():
    """262144 slots, the largest max_slots: 4096 words in 64 chunks, so the
    super-group mask uses all 64 bits; the last word's slots are left inactive."""
    n_vars, n, max_slots = 200, 400, 262144
    print("wide max_slots=262144", flush=True)
    lits, offsets = _clauses(77, n, n_vars)
    vals = _values(78, max_slots, n_vars)
    vals[-64:] = 0
    with gss.Context(n_vars, max_slots, report_capacity=1 << 22) as ctx:
        ctx.add_clauses(lits, offsets)
        ctx.set_assignments(0, vals[:-64])
        active = np.zeros(max_slots, dtype=bool)
        active[:-64] = True
        _check_all(ctx, lits, offsets, vals, active, n)


@pytest.mark.parametrize("max_slots,first,count", [(4160, 0, 4160), (12288, 64, 8000), (8192, 4096, 4096)])
def test_wide_rows_partial_chunks(max_slots, first, count):
    """The last chunk partly used (4160 slots: a chunk of one word), unused chunks
    (12288 slots, 8000 active from slot 64: chunk 2 half empty) and a first chunk
    with no active slot (its super-group is skipped)."""
    n_vars, n = 500, 2500
    print(f"wide partial max_slots={max_slots} first={first} count={count}", flush=True)
    lits, offsets = _clauses(count, n, n_vars)
    part = _values(first + 7, count, n_vars)
    vals, active = full_values(part, max_slots, first)
    with gss.Context(n_vars, max_slots, report_capacity=1 << 20) as ctx:
        ctx.add_clauses(lits, offsets)
        ctx.set_assignments(first, part)
        _check_all(ctx, lits, offsets, vals, active, n)


def test_wide_rows_after_every_kind_of_update():
    """Var-major deltas across a chunk boundary, packed word deltas in chunks 0, 1
    and 7 (which keep the aggregate bits in step), cleared slots; the aggregate
    test is checked after each against the oracle."""
    max_slots, n_vars, n = 32768, 600, 2000
    rng = np.random.default_rng(5)
    lits, offsets = _clauses(55, n, n_vars)
    vals = _values(56, max_slots, n_vars)
    active = np.ones(max_slots, dtype=bool)
    with gss.Context(n_vars, max_slots, report_capacity=1 << 20) as ctx:
        ctx.add_clauses(lits, offsets)
        ctx.set_assignments(0, vals)
        # var-major delta over slots 4000..4200 (chunks 0 and 1)
        vs = np.sort(rng.choice(n_vars, 80, replace=False)) + 1
        new = rng.integers(-1, 2, (80, 200)).astype(np.int8)
        ctx.set_var_values(4000, vs, new)
        vals[4000:4200, vs - 1] = new.T
        _check_all(ctx, lits, offsets, vals, active, n)
        # packed word deltas in words 3 (chunk 0), 70 (chunk 1) and 511 (chunk 7)
        for word in (3, 70, 511):
            vs = np.sort(rng.choice(n_vars, 120, replace=False)) + 1
            x = rng.integers(-1, 2, (120, 64)).astype(np.int8)
            f = np.packbits(x == -1, axis=1, bitorder="little").view(np.uint64).ravel()
            t = np.packbits(x == 1, axis=1, bitorder="little").view(np.uint64).ravel()
            ctx.update_words(word, vs, f, t)
            vals[64 * word:64 * word + 64, vs - 1] = x.T
            for mode, flags in FLAGS:
                got = gpu_dense(ctx, n, flags)
                want = oracle.masks(lits, offsets, vals, mode=mode, active=active)
                assert np.array_equal(got, want), f"word {word} {mode} flags={flags}: " + mismatch_summary(got, want)
        # clear slots 8000..12999 (chunks 1-3)
        ctx.clear_slots(8000, 5000)
        vals[8000:13000] = 0
        active[8000:13000] = False
        _check_all(ctx, lits, offsets, vals, active, n)


def test_wide_rows_refused_where_unsupported():
    import torch
    stream = torch.cuda.Stream()
    with gss.Context(100, 8192, stream=stream) as wide, gss.Context(100, 4096, stream=stream) as narrow:
        gss.Batch([narrow]).close()
        with pytest.raises(gss.GssError) as e:
            gss.Batch([wide, narrow])
        assert e.value.code == gss.GSS_ERR_INVALID_ARG
    with pytest.raises(gss.GssError) as e:
        gss.Context(100, 64 * 64 * 64 + 64)
    assert e.value.code == gss.GSS_ERR_INVALID_ARG
