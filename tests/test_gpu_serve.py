"""Served test (manager thread, producers, continuous batching), GPU.

The server logs every change it applies (deltas, inserts, removals), every run
with its active words, and every record, in the order the device sees them.  A
replay rebuilds the store and the planes at each run and recomputes that run
with the oracle: the records of each word must equal the oracle's for that word
on the store of the moment, whatever else the run tested beside it.  A second
test sends the same snapshot alone and in a full mix and compares its records.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2012_03119_amd import gen, gss

pytestmark = pytest.mark.gpu

REC = [("clause_id", "<u4"), ("word", "<u4"), ("mask", "<u8")]


def _store(seed, n, V):
    rng = np.random.default_rng(seed)
    lengths = gen.lengths_mix(rng, n)
    return gen.random_clauses(rng, lengths, V)


def _values(F, T, W, V):
    """Slot-major int8 values [W*64][V] from per-word F/T plane words [W][V+1]."""
    bits = np.arange(64, dtype=np.uint64)[:, None]
    vals = np.zeros((W * 64, V), dtype=np.int8)
    for w in range(W):
        fb = ((F[w, 1:][None, :] >> bits) & np.uint64(1)).astype(bool)
        tb = ((T[w, 1:][None, :] >> bits) & np.uint64(1)).astype(bool)
        vals[w * 64:(w + 1) * 64][fb] = -1
        vals[w * 64:(w + 1) * 64][tb] = 1
    return vals


def _expected(clauses, F, T, act, W, V, mode):
    ids = np.array(sorted(clauses), dtype=np.uint32)
    if len(ids) == 0:
        return np.zeros(0, dtype=REC)
    offs = np.zeros(len(ids) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(clauses[i]) for i in ids])
    lits = np.concatenate([clauses[i] for i in ids]).astype(np.int32)
    active = np.zeros(W * 64, dtype=bool)
    for w, a in enumerate(act):
        if a:
            active[w * 64:(w + 1) * 64] = [(a >> b) & 1 for b in range(64)]
    dense = oracle.masks(lits, offs, _values(F, T, W, V), mode=mode, active=active)
    return oracle.report_set(dense, ids)


def replay(path, lits0, offs0, V, W, mode="falsified"):
    """Replays a server log against the oracle; returns per-tag counts."""
    clauses = {i: np.asarray(lits0[offs0[i]:offs0[i + 1]]) for i in range(len(offs0) - 1)}
    F = np.zeros((W, V + 1), dtype=np.uint64)
    T = np.zeros((W, V + 1), dtype=np.uint64)
    expected, got = {}, {}
    counts = dict(W=0, A=0, R=0, T=0, E=0, X=0, records=0)
    with open(path) as fh:
        lines = fh.read().splitlines()
    i = 0
    while i < len(lines):
        p = lines[i].split()
        i += 1
        if not p:
            continue
        tag = p[0]
        if tag == "W":
            w, n = int(p[1]), int(p[2])
            rows = [l.split() for l in lines[i:i + n]]
            i += n
            v = np.array([int(r[0]) for r in rows], dtype=np.int64)
            F[w, v] = np.array([int(r[1], 16) for r in rows], dtype=np.uint64)
            T[w, v] = np.array([int(r[2], 16) for r in rows], dtype=np.uint64)
            assert not (F[w] & T[w]).any()
        elif tag == "A":
            cid, L = int(p[1]), int(p[2])
            assert cid not in clauses, "clause id reused"
            clauses[cid] = np.array(p[3:3 + L], dtype=np.int32)
        elif tag == "R":
            for x in p[2:]:
                del clauses[int(x)]
        elif tag == "T":
            run = int(p[1])
            act = [int(x, 16) for x in p[2:]]
            assert len(act) == W
            expected[run] = _expected(clauses, F, T, act, W, V, mode)
            got[run] = []
        elif tag == "P":
            got[int(p[1])].append((int(p[2]), int(p[3]), int(p[4], 16)))
        elif tag == "E":
            run, n = int(p[1]), int(p[2])
            g = np.array(got.pop(run), dtype=REC)
            assert len(g) == n
            g = np.sort(g, order=["clause_id", "word"])
            want = expected.pop(run)
            assert len(g) == len(want), f"run {run}: {len(g)} records, oracle {len(want)}"
            assert (g == want).all(), f"run {run}: records differ from the oracle"
            counts["records"] += n
        elif tag == "X":
            run, n = int(p[1]), int(p[2])
            assert n == len(expected.pop(run)), f"run {run}: overflow count differs from the oracle"
            got.pop(run)
        counts[tag] = counts.get(tag, 0) + 1
    assert not expected, f"runs without an end: {sorted(expected)}"
    return counts, clauses, F, T


@pytest.mark.parametrize("store,report_capacity,mode", [("mix", 1 << 16, "falsified"), ("short", 1, "falsified"),
                                                        ("mix", 1 << 16, "trigger"), ("mix", 1 << 16, "aggregate")])
def test_served_runs_equal_oracle_replay(tmp_path, store, report_capacity, mode):
    W, P = 4, 4
    if store == "mix":  # the length mix of the large workloads
        V = 3000
        lits, offs = _store(41, 20_000, V)
    else:  # two-literal clauses: dense hits that overflow the smallest report segments
        V = 1000
        lits, offs = gen.random_clauses(np.random.default_rng(42), np.full(20_000, 2, dtype=np.int64), V)
    ctx = gss.Context(V, W * 64, report_capacity=report_capacity)
    ids = ctx.add_clauses(lits, offs)
    assert (ids == np.arange(len(offs) - 1)).all()
    log = tmp_path / "serve.log"
    print(f"[serve] replay case store={store} capacity={report_capacity} mode={mode}", flush=True)
    res = ctx.serve_simulate(n_threads=P, duration_s=1.0, snapshot_rate=25.0, redraw_fraction=0.05,
                             insert_rate=400.0, delete_fraction=0.1, seed=7,
                             test_flags={"trigger": gss.GSS_TEST_TRIGGER, "aggregate": gss.GSS_TEST_AGGREGATE}.get(mode, 0),
                             log_path=str(log))
    # the aggregate pre-test changes no record: the replay checks the falsified result
    counts, clauses, F, T = replay(str(log), lits, offs, V, W, "trigger" if mode == "trigger" else "falsified")
    assert res["runs"] == counts["E"] + counts["X"] and counts["E"] >= 5
    assert res["overflowed_runs"] == counts["X"]
    if report_capacity == 1:
        # the first run overflowed: repeated inside the wait when nothing changed
        # meanwhile, else reported (X) and its words tested again
        assert counts["X"] >= 1 or ctx.stats()["regrows"] >= 1
    assert res["inserted"] == counts["A"] > 0
    assert res["deleted"] > 0 and counts["R"] > 0
    assert res["reports"] == counts["records"]
    assert res["tested"] + res["dropped"] <= res["snapshots"]
    assert res["tested"] > 0 and 0 < res["p50_ms"] <= res["p99_ms"] <= res["max_ms"]
    assert res["live_end"] == ctx.store_info()["live_clauses"] == len(clauses)
    # the context is usable again: a plain test equals the oracle on the final state
    ones = np.full(W, 2**64 - 1, dtype=np.uint64)
    ctx.set_active(ones)
    flags = {"trigger": gss.GSS_TEST_TRIGGER, "aggregate": gss.GSS_TEST_AGGREGATE}.get(mode, 0)
    n = ctx.test(flags)
    got = np.sort(ctx.fetch_reports(n), order=["clause_id", "word"])
    want = _expected(clauses, F, T, [2**64 - 1] * W, W, V, "trigger" if mode == "trigger" else "falsified")
    assert len(got) == len(want) and (got == want).all()
    ctx.close()


def _snapshot(seed, V):
    rng = np.random.default_rng(seed)
    vals = gen.assignments_table1(rng, 64, V)  # [64][V]
    f = np.zeros(V, dtype=np.uint64)
    t = np.zeros(V, dtype=np.uint64)
    for b in range(64):
        f |= (vals[b] == -1).astype(np.uint64) << np.uint64(b)
        t |= (vals[b] == 1).astype(np.uint64) << np.uint64(b)
    return vals, f, t


def _collect(srv, p, after, timeout=20.0):
    """Records routed to producer p by the first run after `after` that tested it."""
    out, t0 = [], time.time()
    while time.time() - t0 < timeout:
        r, run = srv.poll(p)
        out.append(r)
        if run is not None and (after is None or run > after):
            return np.sort(np.concatenate(out), order=["clause_id", "word"]), run
        time.sleep(0.002)
    raise AssertionError("no run tested the snapshot in time")


def test_late_pollers_receive_every_routed_record(tmp_path):
    """Producers that do not poll for many runs: their records wait in the pinned
    blocks they were fetched into until the block pool runs out, then are copied
    out for them; polls with a small cap resume where they stopped.  What each
    producer collects equals the records the log shows routed to its word."""
    V, W = 2000, 4
    lits, offs = _store(47, 15_000, V)
    ctx = gss.Context(V, W * 64)
    ctx.add_clauses(lits, offs)
    var_ids = np.arange(1, V + 1, dtype=np.uint32)
    log = tmp_path / "late.log"
    srv = gss.Server(ctx, W, log_path=str(log))
    got = {p: [] for p in range(W)}
    seen = {p: None for p in range(W)}
    try:
        for k in range(16):  # more runs than the pool has blocks; nobody polls
            for p in range(W):
                _, f, t = _snapshot(1000 + 16 * p + k, V)
                srv.send(p, var_ids, f, t)
            time.sleep(0.03)
        time.sleep(0.5)
        for p in range(W):
            while True:
                r, run = srv.poll(p, cap=777)
                got[p].append(r)
                seen[p] = run
                if len(r) == 0:
                    break
    finally:
        res = srv.stop()
    runs = set()
    want = {p: [] for p in range(W)}
    with open(log) as fh:
        for line in fh:
            q = line.split()
            if q and q[0] == "P":
                run, cid, w, m = int(q[1]), int(q[2]), int(q[3]), int(q[4], 16)
                runs.add(run)
                if seen[w] is not None and run <= seen[w]:
                    want[w].append((cid, w, m))
    print(f"[serve] late pollers: {res['runs']} runs, {len(runs)} with records", flush=True)
    assert len(runs) > 10
    for p in range(W):
        g = np.sort(np.concatenate(got[p]).astype(REC), order=["clause_id", "word", "mask"])
        e = np.sort(np.array(want[p], dtype=REC), order=["clause_id", "word", "mask"])
        assert len(e) > 0 and len(g) == len(e) and (g == e).all(), f"producer {p}: {len(g)} vs {len(e)}"


def test_snapshot_alone_equals_snapshot_in_mix():
    V, W = 2000, 8
    lits, offs = _store(43, 15_000, V)
    ctx = gss.Context(V, W * 64)
    ids = ctx.add_clauses(lits, offs)
    snaps = [_snapshot(100 + p, V) for p in range(W)]
    var_ids = np.arange(1, V + 1, dtype=np.uint32)
    srv = gss.Server(ctx, W)
    try:
        # producer 0 alone
        srv.send(0, var_ids, snaps[0][1], snaps[0][2])
        alone, run = _collect(srv, 0, None)
        # the same snapshot again, now beside every other producer's
        for p in range(W):
            srv.send(p, var_ids, snaps[p][1], snaps[p][2])
        mixed = {}
        for p in range(W):
            mixed[p], _ = _collect(srv, p, run if p == 0 else None)
    finally:
        res = srv.stop()
    assert res["runs"] >= 2
    np.testing.assert_array_equal(alone, mixed[0])
    for p in range(W):
        want = oracle.report_set(oracle.masks(lits, offs, snaps[p][0]), ids)
        want["word"] = p
        assert len(mixed[p]) == len(want) and (mixed[p] == want).all(), f"producer {p}"
        assert (mixed[p]["word"] == p).all()
    ctx.close()


def test_inserts_wait_for_the_hbm_budget():
    V = 1000
    lits, offs = _store(44, 2000, V)
    ctx0 = gss.Context(V, 64)
    ctx0.add_clauses(lits, offs)
    used = ctx0.store_info()["device_bytes"]
    ctx0.close()
    # a budget that holds the store but not a large insert
    budget = used + (4 << 20)
    ctx = gss.Context(V, 64, hbm_budget_bytes=budget)
    ctx.add_clauses(lits, offs)
    big_l, big_o = _store(45, 200_000, V)
    # an insert beyond the admission queue is refused whatever the queue holds
    srv = gss.Server(ctx, 1, max_queued_lits=1000)
    try:
        with pytest.raises(gss.GssError) as e:
            srv.insert(0, big_l, big_o)
        assert e.value.code == gss.GSS_ERR_CAPACITY
    finally:
        res = srv.stop()
    assert res["refused"] == len(big_o) - 1 and res["inserted"] == 0
    # an insert beyond the budget is held; tests go on meanwhile
    srv = gss.Server(ctx, 1)
    try:
        srv.insert(0, big_l, big_o)
        vals, f, t = _snapshot(200, V)
        srv.send(0, np.arange(1, V + 1, dtype=np.uint32), f, t)
        got, _ = _collect(srv, 0, None)
    finally:
        res = srv.stop()
    assert res["inserted"] == 0 and res["refused"] == 0
    assert res["live_end"] == len(offs) - 1
    assert res["device_bytes_end"] <= budget
    want = oracle.report_set(oracle.masks(lits, offs, vals), np.arange(len(offs) - 1))
    want["word"] = 0
    assert len(got) == len(want) and (got == want).all()
    ctx.close()


def test_server_argument_errors():
    V = 500
    lits, offs = _store(46, 1000, V)
    ctx = gss.Context(V, 128)
    ctx.add_clauses(lits, offs)
    for bad_n in (0, 3):  # 1..W producers, W = 2
        with pytest.raises(gss.GssError) as e:
            gss.Server(ctx, bad_n)
        assert e.value.code == gss.GSS_ERR_INVALID_ARG
    ctx.set_active(np.full(2, 2**64 - 1, dtype=np.uint64))
    ctx.test_async()
    with pytest.raises(gss.GssError) as e:  # a test in flight
        gss.Server(ctx, 1)
    assert e.value.code == gss.GSS_ERR_STATE
    ctx.test_wait()
    srv = gss.Server(ctx, 2)
    try:
        one = np.ones(1, dtype=np.uint64)
        for args, code in [((2, [1], one, 0 * one), gss.GSS_ERR_INVALID_ARG),      # no such producer
                           ((0, [V + 1], one, 0 * one), gss.GSS_ERR_BAD_LITERAL),  # variable out of range
                           ((0, [3], one, one), gss.GSS_ERR_INVALID_ARG)]:         # F and T in one slot
            with pytest.raises(gss.GssError) as e:
                srv.send(*args)
            assert e.value.code == code
        for (l, o), code in [(([1, -(V + 1)], [0, 2]), gss.GSS_ERR_BAD_LITERAL),
                             (([1, 2], [0, 0, 2]), gss.GSS_ERR_INVALID_ARG)]:     # an empty clause
            with pytest.raises(gss.GssError) as e:
                srv.insert(0, np.array(l, dtype=np.int32), np.array(o, dtype=np.uint64))
            assert e.value.code == code
        with pytest.raises(gss.GssError) as e:
            srv.poll(5)
        assert e.value.code == gss.GSS_ERR_INVALID_ARG
        # a valid snapshot still goes through after the refused calls
        vals, f, t = _snapshot(300, V)
        srv.send(1, np.arange(1, V + 1, dtype=np.uint32), f, t)
        got, run = _collect(srv, 1, None)
    finally:
        res = srv.stop()
    assert res["snapshots"] == 1 and res["tested"] == 1 and res["inserted"] == 0
    want = oracle.report_set(oracle.masks(lits, offs, vals), np.arange(len(offs) - 1))
    want["word"] = 1
    assert len(got) == len(want) and (got == want).all()
    # the context is usable on its own again
    ctx.set_active(np.array([0, 2**64 - 1], dtype=np.uint64))
    n = ctx.test()
    assert n == len(want)
    ctx.close()


def check_evictions(path, n_initial, decay=0.999):
    """Replays the activities of a served log as the device computes them (float32
    additions of the float32 bump) and checks that every eviction ("V n" and the
    removal after it) took the n least active live clauses, the older among
    equals (Section 3.7).  Returns the number of evictions."""
    with open(path) as fh:
        lines = fh.read().splitlines()
    hit = {}  # run -> clauses with a record in it
    for l in lines:
        if l.startswith("P "):
            p = l.split()
            hit.setdefault(int(p[1]), set()).add(int(p[2]))
    act = {}
    live = set(range(n_initial))
    bump, n_ev, i = 1.0, 0, 0
    while i < len(lines):
        p = lines[i].split()
        i += 1
        if not p:
            continue
        if p[0] == "A":
            live.add(int(p[1]))
        elif p[0] == "B":
            b = np.float32(bump)
            for cid in hit.get(int(p[1]), ()):
                act[cid] = np.float32(act.get(cid, np.float32(0)) + b)
            bump /= decay
        elif p[0] == "V":
            n = int(p[1])
            q = lines[i].split()
            i += 1
            assert q[0] == "R" and int(q[1]) == n
            gone = [int(x) for x in q[2:]]
            order = sorted(live, key=lambda c: (float(act.get(c, np.float32(0))), c))
            assert set(gone) == set(order[:n]), "an eviction did not take the least active clauses"
            live -= set(gone)
            n_ev += 1
        elif p[0] == "R":
            live -= {int(x) for x in p[2:]}
    return n_ev


def _class_bytes(lits_offs, T=64):
    """Bytes of each length class of a store as the library lays it out: a slot
    of stride S (the power of two >= max(length, 4)) holds S codes of 4 bytes
    plus 8 bytes of metadata; slots come in whole tiles of T."""
    _, offs = lits_offs
    lengths = np.diff(offs)
    stride = np.maximum(4, 2 ** np.ceil(np.log2(np.maximum(lengths, 1))).astype(np.int64))
    out = {}
    for s in np.unique(stride):
        n = int((stride == s).sum())
        out[int(s)] = -(-n // T) * T * (int(s) * 4 + 8)
    return out


def test_activity_eviction_admits_inserts_under_a_tight_budget(tmp_path):
    W, P, V = 4, 4, 3000
    lits, offs = _store(51, 20_000, V)
    # the device bytes of this store with its activity state, and a budget with
    # room to compact its largest length class but not to grow the classes
    ctx0 = gss.Context(V, W * 64)
    ctx0.add_clauses(lits, offs)
    ctx0.priority_enable(n_sources=P)
    ctx0.set_active(np.full(W, 2**64 - 1, dtype=np.uint64))
    ctx0.test()
    used = ctx0.store_info()["device_bytes"]
    ctx0.close()
    largest = max(_class_bytes((lits, offs)).values())
    budget = used + int(0.9 * largest) + (2 << 20)
    ctx = gss.Context(V, W * 64, hbm_budget_bytes=budget)
    ctx.add_clauses(lits, offs)
    log = tmp_path / "evict.log"
    print(f"[serve] eviction case: budget {budget} bytes, largest class {largest}", flush=True)
    res = ctx.serve_simulate(n_threads=P, duration_s=1.5, snapshot_rate=25.0, redraw_fraction=0.05,
                             insert_rate=2000.0, delete_fraction=0.0, seed=9, log_path=str(log), evict_keep=0.5)
    counts, clauses, F, T = replay(str(log), lits, offs, V, W)
    assert res["evictions"] >= 1 and res["evicted"] > 0
    assert counts.get("V", 0) == res["evictions"]
    assert counts["B"] == counts["E"] >= 5  # every completed run bumped the activities
    assert check_evictions(str(log), len(offs) - 1) == res["evictions"]
    # inserts went on after the budget first bound
    assert res["inserted"] == counts["A"] > 0
    tags = [l.split(" ", 1)[0] for l in log.read_text().splitlines()]
    assert "A" in tags[tags.index("V"):], "no insert was admitted after the first eviction"
    assert res["live_end"] == ctx.store_info()["live_clauses"] == len(clauses)
    assert res["device_bytes_end"] <= budget
    ctx.close()
