"""Learned clause priority on the GPU: the network's kernels against the float64
oracle (forward, gradient, Adam), the per-clause features and training samples
against a replay of the runs with the clause-test oracle, the scheduled test
against the oracle restricted to the clauses the schedule runs, and the gain of
a trained schedule over the plain test on a stream, judged by the plain test."""
import numpy as np
import pytest

import oracle
from oracle import priority as P
from gpu_helpers import new_context
from paper_2012_03119_amd import gen, gss

pytestmark = pytest.mark.gpu


def _problem(seed, n, scale=0.3):
    rng = np.random.default_rng(seed)
    params = rng.normal(0, scale, P.N_PARAMS)
    params[P.N_PARAMS - 1] = 0.1
    x = rng.normal(0, 1, (n, 12))
    y = (rng.random(n) < 0.3).astype(np.float64)
    return params.astype(np.float32), x.astype(np.float32), y.astype(np.float32)


def test_mlp_forward_matches_oracle():
    params, x, _ = _problem(1, 1000)  # four workgroups and a ragged tail
    with new_context(100, 64) as ctx:
        got = gss.gss_mlp_forward(ctx.ctx, params, x)
    want = P.forward(params.astype(np.float64), x.astype(np.float64))["prob"]
    np.testing.assert_allclose(got, want, atol=2e-6, rtol=1e-5)


@pytest.mark.parametrize("n", [1, 31, 1000])
def test_mlp_gradient_matches_oracle(n):
    params, x, y = _problem(2, n)
    with new_context(100, 64) as ctx:
        loss, g = gss.gss_mlp_loss_grad(ctx.ctx, params, x, y)
    want_loss, want_g = P.loss_grad(params.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    assert abs(loss - want_loss) <= 1e-5 * max(1.0, abs(want_loss))
    scale = np.max(np.abs(want_g))
    assert np.max(np.abs(g - want_g)) <= 2e-5 * scale + 1e-8, np.max(np.abs(g - want_g)) / scale


def test_mlp_adam_matches_oracle():
    params, x, y = _problem(3, 512)
    rng = np.random.default_rng(4)
    order = np.concatenate([rng.permutation(512), rng.permutation(512)]).astype(np.uint32)
    batch, lr = 64, 1e-2
    with new_context(100, 64) as ctx:
        got, losses = gss.gss_mlp_train(ctx.ctx, params, x, y, order, batch=batch, lr=lr)
    batches = [order[i:i + batch] for i in range(0, len(order), batch)]
    want, want_losses = P.adam(params.astype(np.float64), x.astype(np.float64), y.astype(np.float64), batches, lr=lr)
    np.testing.assert_allclose(losses, want_losses, rtol=1e-4)
    # Adam divides by the gradient's own magnitude, so an entry whose gradient is
    # dominated by rounding may step the other way; such entries must be rare
    diff = np.abs(got - want)
    assert np.median(diff) < 1e-5
    assert np.mean(diff > 1e-3) < 2e-3
    assert np.max(diff) <= 2 * lr * len(batches) + 1e-6


def _stream_values(rng, n_words, V):
    return np.concatenate([gen.assignments_table1(rng, 64, V) for _ in range(n_words)])


def _redraw(rng, vals, fraction):
    """Each 64-slot word redraws a fraction of its variables from Table 1."""
    n_words = vals.shape[0] // 64
    V = vals.shape[1]
    for w in range(n_words):
        cols = rng.choice(V, size=max(1, int(fraction * V)), replace=False)
        vals[w * 64:(w + 1) * 64][:, cols] = gen.assignments_table1(rng, 64, len(cols))


def test_features_and_samples_follow_the_runs():
    rng = np.random.default_rng(10)
    V, n_words, n = 2000, 2, 5000
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n), V)
    lens = np.diff(offs)
    lbd = np.array([rng.uniform(2, max(2, L)) for L in lens], dtype=np.float32)
    src = rng.integers(0, 4, n).astype(np.uint32)
    vals = _stream_values(rng, n_words, V)
    runs = 10
    with new_context(V, 64 * n_words) as ctx:
        ids = ctx.add_clauses(lits, offs)
        ctx.priority_enable(n_sources=4, sample_period=3, sample_capacity=100_000, seed=5)
        ctx.priority_set_clause_info(ids, lbd, src)
        hist = np.zeros((n, 8), dtype=np.int64)
        expect_rows = []
        for r in range(runs):
            x_before = P.features(lens, lbd.astype(np.float64), np.full(n, r), src, 4, hist)
            hits = P.hit_counts(oracle.masks(lits, offs, vals))
            expect_rows.append(np.concatenate([x_before, (hits > 0)[:, None]], axis=1))
            ctx.set_assignments(0, vals)
            ctx.test()
            ctx.priority_observe()
            hist[:, 1:] = hist[:, :-1]
            hist[:, 0] = hits
            _redraw(rng, vals, 0.05)
        x, _, _ = ctx.priority_fetch(ids)
        sx, sy = ctx.priority_samples(100_000)
        assert ctx.priority_info()["run"] == runs
        # with sampling switched off a further run leaves the samples as they are
        ctx.priority_set_sampling(0)
        ctx.test()
        ctx.priority_observe()
        assert ctx.priority_info()["samples"] == len(sx)
        assert ctx.priority_info()["run"] == runs + 1
    want = P.features(lens, lbd.astype(np.float64), np.full(n, runs), src, 4, hist)
    np.testing.assert_allclose(x, want, rtol=2e-6, atol=1e-6)
    # every sample is the features of some clause before some run, labelled with
    # its hit in that run; about a third of the (clause, run) pairs are sampled
    def key(row):  # (run, length, source) from the age, length and source features
        return (int(round(np.expm1(row[2]))), int(round(np.expm1(row[0]))), int(round(row[3] * 3)))
    by_key = {}
    for row in np.concatenate(expect_rows):
        by_key.setdefault(key(row), []).append(row)
    got_rows = np.concatenate([sx.astype(np.float64), sy[:, None].astype(np.float64)], axis=1)
    for row in got_rows:
        cands = np.array(by_key.get(key(row), []))
        assert len(cands), f"sample {row} matches no clause and run"
        assert np.min(np.max(np.abs(cands - row), axis=1)) < 1e-5, f"sample {row} matches no clause and run"
    total = n * runs
    assert abs(len(sx) - total / 3) < 5 * np.sqrt(total / 3)


def test_scheduled_test_equals_oracle_on_scheduled_clauses():
    rng = np.random.default_rng(11)
    V, n_words, n = 3000, 4, 20_000
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n), V)
    vals = _stream_values(rng, n_words, V)
    params, _, _ = _problem(12, 1, scale=0.2)
    with new_context(V, 64 * n_words) as ctx:
        ids = ctx.add_clauses(lits, offs)
        ctx.priority_enable(n_sources=1, seed=1)
        ctx.priority_params(set_to=params)
        ctx.set_assignments(0, vals)
        for r in range(3):  # some history first
            ctx.test()
            ctx.priority_observe()
        x, _, _ = ctx.priority_fetch(ids)
        probs = P.forward(params.astype(np.float64), x.astype(np.float64))["prob"]
        tau = float(np.median(probs))
        n_low = ctx.priority_score(tau)
        x, score, low = ctx.priority_fetch(ids)
        np.testing.assert_allclose(score, probs, atol=2e-6)
        assert (low == (score < tau)).all() and n_low == low.sum() and 0 < n_low < n
        full = oracle.masks(lits, offs, vals)
        for k in range(4):  # four runs: each low clause takes its turn once
            run = ctx.priority_info()["run"]
            m = ctx.test(gss.GSS_TEST_SCHEDULED)
            got = np.sort(ctx.fetch_reports(m), order=["clause_id", "word"])
            keep = P.tested(ids, low, run)
            want = oracle.report_set(np.where(keep[:, None], full, np.uint64(0)), ids)
            assert len(got) == len(want) and (got == want).all(), f"run {run}"
            ctx.priority_observe()


def test_scheduled_runs_follow_new_marks_and_store_changes():
    """The slots a scheduled run tests follow the store, the schedule bits and the
    run number mod 4: twelve runs in a row, then a new marking, then removals and
    insertions, and a marking again; every run equals the oracle on the clauses
    the schedule tests."""
    rng = np.random.default_rng(17)
    V, n_words, n = 3000, 4, 20_000
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n), V)
    vals = _stream_values(rng, n_words, V)
    clauses = {}  # live id -> literals
    with new_context(V, 64 * n_words) as ctx:
        ids = ctx.add_clauses(lits, offs)
        assert (ids == np.arange(n)).all()
        for k, i in enumerate(ids):
            clauses[int(i)] = lits[offs[k]:offs[k + 1]]
        ctx.priority_enable(n_sources=1, seed=1)
        ctx.set_assignments(0, vals)
        low = (rng.random(n) < 0.6).astype(np.uint8)  # one flag per issued id
        ctx.priority_mark(low)

        def check(tag):
            run = ctx.priority_info()["run"]
            print(f"[scheduled] {tag}: run {run}", flush=True)
            m = ctx.test(gss.GSS_TEST_SCHEDULED)
            got = np.sort(ctx.fetch_reports(m), order=["clause_id", "word"])
            live = np.array(sorted(clauses), dtype=np.int64)
            l_lits = np.concatenate([clauses[i] for i in live])
            l_offs = np.concatenate([[0], np.cumsum([len(clauses[i]) for i in live])]).astype(np.int64)
            full = oracle.masks(l_lits, l_offs, vals)
            keep = P.tested(live, low[live], run)
            want = oracle.report_set(np.where(keep[:, None], full, np.uint64(0)), live.astype(np.uint32))
            assert len(got) == len(want) and (got == want).all(), f"{tag}: run {run}"
            ctx.priority_observe()

        for _ in range(12):
            check("same store and marks")
        low = (rng.random(n) < 0.3).astype(np.uint8)
        ctx.priority_mark(low)
        for _ in range(6):
            check("new marks")
        gone = rng.choice(n, size=3000, replace=False)
        ctx.remove_clauses(gone.astype(np.uint32))
        for i in gone:
            del clauses[int(i)]
        m2 = 2000
        lits2, offs2 = gen.random_clauses(rng, gen.lengths_mix(rng, m2), V)
        ids2 = ctx.add_clauses(lits2, offs2)
        assert (ids2 == np.arange(n, n + m2)).all()
        for k, i in enumerate(ids2):
            clauses[int(i)] = lits2[offs2[k]:offs2[k + 1]]
        low = np.concatenate([low, np.zeros(m2, np.uint8)])  # new clauses start high
        for _ in range(5):
            check("removals and insertions")
        low = (rng.random(n + m2) < 0.5).astype(np.uint8)
        ctx.priority_mark(low)
        for _ in range(5):
            check("changed store, new marks")


def test_trained_schedule_misses_at_most_one_percent():
    """Train on the hit logs of a stream, pick the threshold on the training
    samples, then run scheduled and plain tests side by side on later runs of the
    same stream: the schedule skips work and misses at most 1% of the hits."""
    rng = np.random.default_rng(20)
    V, n_words, n = 20_000, 8, 100_000
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n), V)
    vals = _stream_values(rng, n_words, V)
    with new_context(V, 64 * n_words, report_capacity=1 << 20) as ctx:
        ids = ctx.add_clauses(lits, offs)
        lens = np.diff(offs)
        ctx.priority_enable(n_sources=8, sample_period=4, sample_capacity=1 << 20, seed=3)
        ctx.priority_set_clause_info(ids, np.array([rng.uniform(2, max(2, L)) for L in lens], np.float32),
                                     rng.integers(0, 8, n).astype(np.uint32))
        for r in range(24):  # training stream: plain tests
            ctx.set_assignments(0, vals)
            ctx.test()
            ctx.priority_observe()
            _redraw(rng, vals, 0.05)
        loss = ctx.priority_train(3, batch=1024, lr=3e-3, seed=9)
        assert np.isfinite(loss)
        sx, sy = ctx.priority_samples(1 << 20)
        p = gss.gss_mlp_forward(ctx.ctx, ctx.priority_params(), sx)
        pos = np.sort(p[sy > 0.5])
        # a low clause is skipped in 3 runs of 4: keep the low positives under 0.4%
        tau = float(pos[int(0.004 * len(pos))]) if len(pos) else 0.5
        n_low = ctx.priority_score(tau)
        assert n_low > n // 4, f"threshold {tau} marks only {n_low} clauses low"
        hits_plain = hits_sched = hits_random = 0
        bits = lambda r: sum(bin(int(c)).count("1") for c in r["mask"])
        for r in range(16):  # evaluation: scheduled and plain on the same runs
            ctx.set_assignments(0, vals)
            m = ctx.test(gss.GSS_TEST_SCHEDULED)
            sched = ctx.fetch_reports(m)
            ctx.priority_observe()
            m = ctx.test()
            plain = ctx.fetch_reports(m)
            ps = {(int(a), int(b)): int(c) for a, b, c in plain}
            for a, b, c in sched:  # the schedule only drops clauses, it never changes a record
                assert ps[(int(a), int(b))] == int(c)
            hits_plain += bits(plain)
            hits_sched += bits(sched)
            # a random schedule with the same budget on the same assignments
            low = np.zeros(n, dtype=np.uint8)
            low[rng.choice(n, size=n_low, replace=False)] = 1
            ctx.priority_mark(low)
            m = ctx.test(gss.GSS_TEST_SCHEDULED)
            hits_random += bits(ctx.fetch_reports(m))
            _redraw(rng, vals, 0.05)
            n_low = ctx.priority_score(tau)  # fresh scores for the next run
    missed = 1 - hits_sched / hits_plain
    missed_random = 1 - hits_random / hits_plain
    print(f"[learned] threshold {tau:.4f}, {n_low} of {n} clauses low, missed {missed:.4f} of {hits_plain} hits; "
          f"a random schedule of the same budget missed {missed_random:.4f}", flush=True)
    assert hits_plain > 0 and missed <= 0.01, f"missed {missed:.4f} of {hits_plain} hits"
    # what the network gains over the method without it: the same budget spent at
    # random loses a large share of the hits
    assert missed_random > 0.2 and missed < missed_random / 20


def test_update_rescores_exactly_the_changed_clauses():
    rng = np.random.default_rng(13)
    V, n_words, n = 2000, 2, 8000
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n), V)
    vals = _stream_values(rng, n_words, V)
    params, _, _ = _problem(14, 1, scale=0.2)
    with new_context(V, 64 * n_words) as ctx:
        ids = ctx.add_clauses(lits, offs)
        ctx.priority_enable(n_sources=1, seed=2)
        ctx.priority_params(set_to=params)
        ctx.set_assignments(0, vals)
        ctx.test()
        ctx.priority_observe()
        x0, _, _ = ctx.priority_fetch(ids)
        tau = float(np.median(P.forward(params.astype(np.float64), x0.astype(np.float64))["prob"]))
        ctx.priority_score(tau)
        _, s0, _ = ctx.priority_fetch(ids)
        _redraw(rng, vals, 0.2)
        ctx.set_assignments(0, vals)
        ctx.test()
        ctx.priority_observe()
        x1, _, _ = ctx.priority_fetch(ids)
        n_low = ctx.priority_update()
        _, s1, low1 = ctx.priority_fetch(ids)
    # rescored: a history that moved this run and a hit that may change the clause's side
    moved = np.any(x1[:, 4:] != 0, axis=1)
    hit = x1[:, 4] > 0
    low0 = s0 < tau
    changed = moved & np.where(low0, hit, ~hit)
    assert 0 < changed.sum() < n
    want = P.forward(params.astype(np.float64), x1.astype(np.float64))["prob"]
    np.testing.assert_allclose(s1[changed], want[changed], atol=2e-6)
    np.testing.assert_array_equal(s1[~changed], s0[~changed])  # the others keep their scores
    assert (low1 == (s1 < tau)).all() and n_low == low1.sum()


def test_activity_and_reduce_follow_the_oracle():
    """Section 3.7: activities bumped on every hit and a reduction that keeps the
    most active clauses.  With decay 1/2 every bump is a power of two, so the fp32
    activities are exact and the kept set must match the oracle's."""
    rng = np.random.default_rng(15)
    V, n_words = 1500, 2
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, 4000), V)
    l2, o2 = gen.random_clauses(rng, rng.integers(1, 4, 3000), V)  # short: frequent hits
    lits = np.concatenate([lits, l2])
    offs = np.concatenate([offs, offs[-1] + o2[1:]])
    n = len(offs) - 1
    vals = _stream_values(rng, n_words, V)
    hits_by_run = []
    with new_context(V, 64 * n_words) as ctx:
        ids = ctx.add_clauses(lits, offs)
        ctx.priority_enable(n_sources=1, seed=3, activity_decay=0.5)
        for r in range(6):
            ctx.set_assignments(0, vals)
            ctx.test()
            ctx.priority_observe()
            hits_by_run.append(P.hit_counts(oracle.masks(lits, offs, vals)))
            _redraw(rng, vals, 0.3)
        act = ctx.priority_activity(ids)
        want = P.activity(hits_by_run, 0.5)
        np.testing.assert_array_equal(act, want)
        keep = n // 3
        assert ctx.priority_reduce(keep) == n - keep
        assert ctx.store_info()["live_clauses"] == keep
        kept = P.reduce_keep(want, ids, keep)
        # the store now holds exactly the kept clauses: a test on new values shows it
        ctx.set_assignments(0, vals)
        m = ctx.test()
        got = np.sort(ctx.fetch_reports(m), order=["clause_id", "word"])
        assert ctx.priority_reduce(keep) == 0  # nothing more to remove
    mask = np.zeros(n, dtype=bool)
    mask[kept] = True
    dense = oracle.masks(lits, offs, vals)
    want_r = oracle.report_set(np.where(mask[:, None], dense, np.uint64(0)), ids)
    assert len(got) == len(want_r) and (got == want_r).all()
