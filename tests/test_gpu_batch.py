"""Batched test (several independent stores, one persistent launch), GPU.

Per store, the batched results equal the oracle's element by element, under
every schedule, with and without hipGraph replay (replays interleaved with
changes of the assignments and of the stores), and equal each store's own
gss_test.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import full_values, mismatch_summary, reports_to_dense
from paper_2012_03119_amd import gen, gss

pytestmark = pytest.mark.gpu

# (clauses, vars, slots): uneven sizes, variable counts and widths, like the
# batched workload at a scale the oracle checks in seconds
STORES = [(1000, 4000, 1024), (2500, 500, 64), (5000, 3000, 512), (10000, 850, 128),
          (15000, 2000, 768), (20000, 1400, 256), (25000, 4100, 384), (30000, 2400, 192)]


def _make(seed):
    import torch
    stream = torch.cuda.Stream()
    items = []
    for i, (n, v, a) in enumerate(STORES):
        w = gen.paper(seed * 100 + i, n_clauses=n, n_vars=v, n_slots=a, planted_rate=0.0)
        ctx = gss.Context(v, a, stream=stream)
        ctx.add_clauses(w.lits, w.offsets)
        ctx.set_assignments(0, w.values)
        items.append([w, ctx, w.values.copy()])
    return stream, items


def _dense(ctx, n_ids):
    r = ctx.fetch_reports()
    return reports_to_dense(r, n_ids, ctx.n_words)


def _check_all(items, counts, mode="falsified"):
    for (w, ctx, vals), n in zip(items, counts):
        got = _dense(ctx, w.n_clauses)
        assert int(np.count_nonzero(got)) == int(n)
        want = oracle.masks(w.lits, w.offsets, vals, mode=mode)
        assert np.array_equal(got, want), mismatch_summary(got, want)


@pytest.mark.parametrize("order,chunk,bpc", [
    (gss.GSS_ORDER_STORE, 0, 0), (gss.GSS_ORDER_INTERLEAVE, 1, 0), (gss.GSS_ORDER_INTERLEAVE, 64, 2),
    (gss.GSS_ORDER_LONGEST_FIRST, 16, 0), (gss.GSS_ORDER_LONGEST_FIRST, 256, 1),
])
@pytest.mark.parametrize("mode", ["falsified", "trigger"])
def test_batch_schedules(order, chunk, bpc, mode):
    _, items = _make(3)
    flags = gss.GSS_TEST_TRIGGER if mode == "trigger" else 0
    print(f"batch order={order} chunk={chunk} bpc={bpc} mode={mode}", flush=True)
    with gss.Batch([it[1] for it in items]) as b:
        b.set_schedule(order, chunk, bpc)
        counts = b.test(flags)
        _check_all(items, counts, mode)
    for it in items:
        it[1].close()


def test_batch_equals_plain_and_graph_replays():
    _, items = _make(4)
    plain = []
    for w, ctx, vals in items:
        ctx.test()
        plain.append(_dense(ctx, w.n_clauses))
    with gss.Batch([it[1] for it in items]) as b:
        b.set_schedule(gss.GSS_ORDER_INTERLEAVE, 32)
        counts = b.test(gss.GSS_TEST_GRAPH)
        for (w, ctx, vals), ref in zip(items, plain):
            assert np.array_equal(_dense(ctx, w.n_clauses), ref)
        assert b.info()["captures"] == 1
        rng = np.random.default_rng(8)
        for rep in range(4):
            # eager work between replays: new values for some variables of every store
            for it in items:
                w, ctx, vals = it
                vs = np.sort(rng.choice(w.n_vars, max(1, w.n_vars // 20), replace=False)) + 1
                vals[:, vs - 1] = -vals[:, vs - 1]
                ctx.set_var_values(0, vs, np.ascontiguousarray(vals[:, vs - 1].T))
            counts = b.test(gss.GSS_TEST_GRAPH)
            print(f"graph replay {rep}", flush=True)
            _check_all(items, counts)
        assert b.info()["captures"] == 1          # replayed, not re-captured
        # a store change forces a new capture, and results follow it
        w, ctx, vals = items[2]
        extra = gen.paper(77, n_clauses=3000, n_vars=w.n_vars, n_slots=w.n_slots)
        ids = ctx.add_clauses(extra.lits, extra.offsets)
        lits = np.concatenate([w.lits, extra.lits])
        offs = np.concatenate([w.offsets, w.offsets[-1] + extra.offsets[1:]])
        items[2][0] = gen.Workload("x", w.n_vars, lits, offs, vals, w.planted, 0)
        counts = b.test(gss.GSS_TEST_GRAPH)
        assert b.info()["captures"] == 2
        _check_all(items, counts)
    for it in items:
        it[1].close()


def test_batch_overflow_regrows():
    _, items = _make(5)
    with gss.Batch([it[1] for it in items]) as b:
        counts = b.test()
        _check_all(items, counts)


def test_autotuner_picks_and_caches(tmp_path):
    from paper_2012_03119_amd import autotune
    import torch
    _, items = _make(6)
    shapes = [(it[0].n_clauses, it[0].n_vars, it[0].n_slots) for it in items]
    cache = str(tmp_path / "tune.json")
    with gss.Batch([it[1] for it in items]) as b:
        first = autotune.autotune(b, shapes, torch.cuda.get_device_name(0), reps=1, cache_path=cache)
        assert first["source"] == "measured" and len(first["trials"]) == len(autotune.CANDIDATES)
        assert first["ms"] == min(t["ms"] for t in first["trials"])
        counts = b.test()
        _check_all(items, counts)            # the chosen schedule is still exact
        again = autotune.autotune(b, shapes, torch.cuda.get_device_name(0), cache_path=cache)
        assert again["source"] == "cache" and again["order"] == first["order"]
    for it in items:
        it[1].close()


def test_batch_with_queued_deltas_and_their_errors():
    """Queued (asynchronous) deltas of every store land before a batched test, in
    graph replays too; a failed device-side check is reported by the batched test,
    which applies nothing of that store's queued updates and leaves the others."""
    import torch
    _, items = _make(6)
    rng = np.random.default_rng(9)
    with gss.Batch([it[1] for it in items]) as b:
        for rep in range(3):
            for it in items:
                w, ctx, vals = it
                vs = np.sort(rng.choice(w.n_vars, max(1, w.n_vars // 20), replace=False)).astype(np.uint32) + 1
                vals[:, vs - 1] = -vals[:, vs - 1]
                ctx.set_var_values_async(0, vs, torch.from_numpy(np.ascontiguousarray(vals[:, vs - 1].T)).cuda())
            counts = b.test(gss.GSS_TEST_GRAPH)
            print(f"queued deltas, replay {rep}", flush=True)
            _check_all(items, counts)
        # store 3: a bad value; store 5: a good delta queued in the same round
        w3, ctx3, vals3 = items[3]
        bad = torch.zeros((4, w3.values.shape[0]), dtype=torch.int8, device="cuda")
        bad[1, 2] = 7
        ctx3.set_var_values_async(0, np.array([1, 2, 3, 4], np.uint32), bad)
        w5, ctx5, vals5 = items[5]
        vs = np.arange(1, 30, dtype=np.uint32)
        vals5[:, vs - 1] = -vals5[:, vs - 1]
        ctx5.set_var_values_async(0, vs, torch.from_numpy(np.ascontiguousarray(vals5[:, vs - 1].T)).cuda())
        with pytest.raises(gss.GssError) as e:
            b.test(gss.GSS_TEST_GRAPH)
        assert e.value.code == gss.GSS_ERR_INVALID_ARG and "store 3" in str(e.value)
        counts = b.test(gss.GSS_TEST_GRAPH)  # reported once; store 3 unchanged, store 5 updated
        _check_all(items, counts)
    for it in items:
        it[1].close()


def test_batch_async_with_the_next_round_queued_behind_it():
    """gss_batch_test_async, then the next round's deltas queued while it runs,
    then gss_batch_wait: each round equals the oracle on the values queued before
    its launch.  While the batch is in flight its members refuse direct tests and
    waits, and the batch refuses a second launch."""
    import torch
    _, items = _make(8)
    rng = np.random.default_rng(10)

    def queue_round():
        for it in items:
            w, ctx, vals = it
            vs = np.sort(rng.choice(w.n_vars, max(1, w.n_vars // 20), replace=False)).astype(np.uint32) + 1
            vals[:, vs - 1] = -vals[:, vs - 1]
            ctx.set_var_values_async(0, vs, torch.from_numpy(np.ascontiguousarray(vals[:, vs - 1].T)).cuda())

    with gss.Batch([it[1] for it in items]) as b:
        b.test(0)  # sizes the report segments
        queue_round()
        for rep in range(4):
            at_launch = [it[2].copy() for it in items]
            b.test_async(gss.GSS_TEST_GRAPH)
            if rep == 0:
                ctx = items[2][1]
                for call in (lambda: ctx.test(0), ctx.test_wait, ctx.fetch_reports,
                             lambda: b.test(0), lambda: b.test_async(0)):
                    with pytest.raises(gss.GssError) as e:
                        call()
                    assert e.value.code == gss.GSS_ERR_STATE
            queue_round()  # the next round, behind the test in flight
            counts = b.wait()
            print(f"async batch, round {rep}", flush=True)
            for (w, ctx, _), vals, n in zip(items, at_launch, counts):
                got = _dense(ctx, w.n_clauses)
                assert int(np.count_nonzero(got)) == int(n)
                want = oracle.masks(w.lits, w.offsets, vals)
                assert np.array_equal(got, want), mismatch_summary(got, want)
        with pytest.raises(gss.GssError) as e:
            b.wait()
        assert e.value.code == gss.GSS_ERR_STATE
        counts = b.test(0)  # the last queued round
        _check_all(items, counts)
    for it in items:
        it[1].close()


def test_batch_async_overflow():
    """Stores that overflow in an asynchronous batched test: with nothing changed
    since the launch the wait repeats the batch (exact records); with a change
    queued behind the launch the wait reports the overflow (the segments are
    grown), and the next test fits."""
    import torch
    stream = torch.cuda.Stream()
    items = []
    for i, (n, v, a) in enumerate([(20000, 300, 256), (3000, 900, 64)]):
        w = gen.paper(900 + i, n_clauses=n, n_vars=v, n_slots=a, planted_rate=0.0)
        ctx = gss.Context(v, a, stream=stream, report_capacity=64)
        ctx.add_clauses(w.lits, w.offsets)
        vals = w.values.copy() if i == 0 else np.zeros_like(w.values)  # store 1: all U, no records
        ctx.set_assignments(0, vals)
        items.append([w, ctx, vals])
    with gss.Batch([it[1] for it in items]) as b:
        b.test_async(0)
        counts = b.wait()  # store 0 overflowed, grown and repeated inside the wait
        _check_all(items, counts)
        assert counts[1] == 0
        # store 1 takes its real values (records far beyond its minimal segments),
        # and one variable is queued again behind the launch
        w, ctx, vals = items[1]
        vs = np.arange(1, w.n_vars + 1, dtype=np.uint32)
        new = w.values.copy()
        ctx.set_var_values_async(0, vs, torch.from_numpy(np.ascontiguousarray(new.T)).cuda())
        b.test_async(0)
        ctx.set_var_values_async(0, vs[:1], torch.from_numpy(np.ascontiguousarray(new[:, :1].T)).cuda())
        vals[:] = new
        with pytest.raises(gss.GssError) as e:
            b.wait()
        assert e.value.code == gss.GSS_ERR_REPORT_OVERFLOW
        counts = b.test(0)  # fits now
        _check_all(items, counts)
    for it in items:
        it[1].close()


def test_batch_refuses_a_member_with_an_async_test_in_flight():
    """The batched test would overwrite the report segments of a member whose own
    asynchronous test is still pending: it is refused before anything is queued,
    and the member's test completes with its own records."""
    _, items = _make(7)
    w, ctx, vals = items[1]
    with gss.Batch([it[1] for it in items]) as b:
        ctx.test_async(0)
        with pytest.raises(gss.GssError) as e:
            b.test(0)
        assert e.value.code == gss.GSS_ERR_STATE
        n = ctx.test_wait()
        got = _dense(ctx, w.n_clauses)
        assert int(np.count_nonzero(got)) == int(n)
        want = oracle.masks(w.lits, w.offsets, vals)
        assert np.array_equal(got, want), mismatch_summary(got, want)
        counts = b.test(0)
        _check_all(items, counts)



@pytest.mark.parametrize("mode", ["falsified", "trigger"])
def test_batch_aggregate_pretest_with_graph_replays(mode):
    """GSS_TEST_AGGREGATE in the batched kernel: Table 1 words (where the
    aggregate bits are selective), per-store parity with the oracle, and graph
    replays after bulk updates that leave the bits stale (refreshed before each
    launch)."""
    import torch
    stream = torch.cuda.Stream()
    rng = np.random.default_rng(21)
    items = []
    for i, (n, v, a) in enumerate(STORES[:5]):
        lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n), v)
        vals = np.concatenate([gen.assignments_table1(rng, 64, v) for _ in range(a // 64)])
        ctx = gss.Context(v, a, stream=stream, report_capacity=1 << 21)  # no regrowth: one capture
        ctx.add_clauses(lits, offs)
        ctx.set_assignments(0, vals)
        items.append([lits, offs, ctx, vals])
    flags = gss.GSS_TEST_AGGREGATE | (gss.GSS_TEST_TRIGGER if mode == "trigger" else 0)
    with gss.Batch([it[2] for it in items]) as b:
        b.set_schedule(gss.GSS_ORDER_INTERLEAVE, 16)
        for rep in range(3):
            print(f"batch aggregate mode={mode} replay {rep}", flush=True)
            counts = b.test(flags | gss.GSS_TEST_GRAPH)
            for (lits, offs, ctx, vals), cnt in zip(items, counts):
                got = _dense(ctx, len(offs) - 1)
                assert int(np.count_nonzero(got)) == int(cnt)
                want = oracle.masks(lits, offs, vals, mode=mode)
                assert np.array_equal(got, want), mismatch_summary(got, want)
            for lits, offs, ctx, vals in items:  # a bulk update: the aggregate bits go stale
                V = vals.shape[1]
                flip = 1 + rng.choice(V, max(1, V // 10), replace=False).astype(np.uint32)
                vals[:, flip - 1] = -vals[:, flip - 1]
                ctx.set_var_values(0, flip, np.ascontiguousarray(vals[:, flip - 1].T))
        assert b.info()["captures"] == 1
    for it in items:
        it[2].close()
