"""Parity at the paper's full scale (GPU): 4M clauses x 1M variables x 1024
assignments, in the launch configuration the benchmark times, with the whole
output of every round compared with the oracle.

Each round's delta (the 5% of variables whose values flip, with their new values
var-major) is queued on the device behind the test still in flight, exactly as
the benchmark's steps do; the oracle computes the dense masks of all 4M clauses
on the host for the same round and the records of the GPU must equal them word
for word.  Also at full size: the aggregate pre-test in both modes, LDS staging
of the hot rows on Zipf-distributed variables, and the batched test over the
eight database sizes of the batched workload (sampled there).
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import mismatch_summary
from paper_2012_03119_amd import gen, gss

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SEED = 2


def _dense(r, n, n_ids, W):
    """Dense masks from all n records of a test; a (clause, word) cell written
    twice would leave fewer nonzero cells than records."""
    assert len(r) == n
    assert (r["mask"] != 0).all() and (r["word"] < W).all() and (r["clause_id"] < n_ids).all()
    d = np.zeros((n_ids, W), dtype=np.uint64)
    d[r["clause_id"], r["word"]] = r["mask"]
    assert int(np.count_nonzero(d)) == n, "duplicate (clause, word) records"
    return d


@pytest.fixture(scope="module")
def paper():
    print("paper scale: generating", flush=True)
    w = gen.paper(SEED)
    return w, oracle.transpose(w.values)


def _run_rounds(w, vm0, flags, n_rounds, hot_vars=0, mode="falsified"):
    """Round 0 synchronously, rounds 1.. pipelined as the benchmark runs them;
    every round's complete output against the oracle."""
    import torch
    N, V, A = w.n_clauses, w.n_vars, w.n_slots
    W = A // 64
    vm = vm0.copy()
    flips = gen.flip_rounds(SEED + 1000, V, n_rounds)
    deltas = []
    for flip in flips[:n_rounds - 1]:
        vm[flip - 1] = -vm[flip - 1]
        deltas.append((flip.astype(np.uint32), torch.from_numpy(np.ascontiguousarray(vm[flip - 1])).cuda()))
    vm[:] = vm0
    with gss.Context(V, A, report_capacity=1 << 20, hot_vars=hot_vars) as ctx:
        ctx.add_clauses(w.lits, w.offsets)
        ctx.set_assignments(0, w.values)
        print(f"paper scale flags={flags} hot={hot_vars}: store and planes ready", flush=True)
        n = ctx.test(flags)
        for rnd in range(n_rounds):
            if rnd + 1 < n_rounds:  # the next round's delta, queued behind this round's test
                ctx.set_var_values_async(0, *deltas[rnd])
            if rnd > 0:
                n = ctx.test_wait()
            got = _dense(ctx.fetch_reports(n), n, N, W)
            if rnd + 1 < n_rounds:
                ctx.test_async(flags)
            want = oracle.masks(w.lits, w.offsets, values_vm=vm, mode=mode)
            print(f"paper scale flags={flags} round {rnd}: {n} records", flush=True)
            assert np.array_equal(got, want), f"round {rnd}: " + mismatch_summary(got, want)
            if rnd == 0 and mode == "falsified":
                c, a = w.planted[:, 0], w.planted[:, 1]
                assert ((got[c, a // 64] >> (a % 64).astype(np.uint64)) & np.uint64(1)).all()
            if rnd + 1 < n_rounds:
                flip = flips[rnd]
                vm[flip - 1] = -vm[flip - 1]


@pytest.mark.timeout(900)
def test_paper_scale_every_round_falsified(paper):
    _run_rounds(*paper, flags=0, n_rounds=20)


@pytest.mark.timeout(600)
def test_paper_scale_trigger(paper):
    _run_rounds(*paper, flags=gss.GSS_TEST_TRIGGER, n_rounds=3, mode="trigger")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", ["falsified", "trigger"])
def test_paper_scale_aggregate(paper, mode):
    flags = gss.GSS_TEST_AGGREGATE | (gss.GSS_TEST_TRIGGER if mode == "trigger" else 0)
    _run_rounds(*paper, flags=flags, n_rounds=3, mode=mode)


@pytest.mark.timeout(600)
def test_paper_scale_zipf_hot_rows():
    print("paper scale Zipf(1.1): generating", flush=True)
    w = gen.paper(SEED, var_weights=gen.zipf_weights(1_000_000, 1.1))
    _run_rounds(w, oracle.transpose(w.values), flags=0, n_rounds=3, hot_vars=64)


def _sub_csr(lits, offsets, idx):
    lengths = offsets[idx + 1] - offsets[idx]
    starts = np.repeat(offsets[idx], lengths)
    within = np.arange(int(lengths.sum())) - np.repeat(np.cumsum(lengths) - lengths, lengths)
    sub_off = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(lengths, out=sub_off[1:])
    return lits[starts + within], sub_off


#: the batched workload's eight databases: (clauses, variables, assignment slots)
BATCHED = ((100_000, 2_000_000, 1024), (250_000, 50_000, 64), (500_000, 1_180_000, 512),
           (1_000_000, 85_000, 128), (1_500_000, 698_000, 768), (2_000_000, 144_000, 256),
           (2_500_000, 412_000, 384), (3_000_000, 243_000, 192))


@pytest.mark.timeout(900)
def test_batched_at_full_database_sizes():
    """One graph-captured persistent launch over the eight full-size databases; per
    database every record is checked for range and uniqueness, and a sample of
    20,000 clauses plus every planted clause equals the oracle word for word."""
    import torch
    stream = torch.cuda.Stream()
    items = []
    for i, (n, v, a) in enumerate(BATCHED):
        w = gen.paper(300 + i, n_clauses=n, n_vars=v, n_slots=a)
        ctx = gss.Context(v, a, stream=stream, report_capacity=1 << 22)
        ctx.add_clauses(w.lits, w.offsets)
        ctx.set_assignments(0, w.values)
        rng = np.random.default_rng(i)
        sample = np.union1d(rng.choice(n, min(n, 20_000), replace=False), w.planted[:, 0])
        s_lits, s_off = _sub_csr(w.lits, w.offsets, sample)
        want = oracle.masks(s_lits, s_off, w.values)
        items.append((w.n_clauses, a // 64, ctx, sample, want))
        print(f"batched database {i}: {n} clauses ready", flush=True)
        del w
    with gss.Batch([it[2] for it in items]) as b:
        for rep in range(2):  # capture, then replay
            counts = b.test(gss.GSS_TEST_GRAPH)
            for i, (n_ids, W, ctx, sample, want) in enumerate(items):
                got = _dense(ctx.fetch_reports(int(counts[i])), int(counts[i]), n_ids, W)[sample]
                assert np.array_equal(got, want), f"database {i}: " + mismatch_summary(got, want)
            print(f"batched replay {rep}: {int(np.sum(counts))} records", flush=True)
    for it in items:
        it[2].close()
