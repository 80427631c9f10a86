"""Parity at the paper's full scale (GPU): 4M clauses x 1M variables x 1024
assignments, in the launch configuration the benchmark times.

The oracle cannot check all 4.1e9 pairs in seconds, so every round compares a
random sample of clauses (plus every planted clause) element by element, and
checks properties of the complete output that hold at any size: records are
unique per (clause, word), never empty, in range, and every planted pair of
round 0 is reported.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import mismatch_summary
from paper_2012_03119_amd import gen, gss

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _sub_csr(lits, offsets, idx):
    lengths = offsets[idx + 1] - offsets[idx]
    starts = np.repeat(offsets[idx], lengths)
    within = np.arange(int(lengths.sum())) - np.repeat(np.cumsum(lengths) - lengths, lengths)
    sub_off = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(lengths, out=sub_off[1:])
    return lits[starts + within], sub_off


@pytest.mark.timeout(900)
@pytest.mark.parametrize("flags", [0, gss.GSS_TEST_TRIGGER])
def test_paper_scale_sampled(flags):
    import torch
    mode = "trigger" if flags & gss.GSS_TEST_TRIGGER else "falsified"
    print(f"paper scale, mode={mode}: generating", flush=True)
    w = gen.paper(2)
    N, V, A = w.n_clauses, w.n_vars, w.n_slots
    W = A // 64
    vm = oracle.transpose(w.values)
    rng = np.random.default_rng(123)
    sample = np.union1d(rng.choice(N, 20_000, replace=False), w.planted[:, 0])
    s_lits, s_off = _sub_csr(w.lits, w.offsets, sample)
    flips = gen.flip_rounds(1002, V, 3)
    # the oracle on the sample for the three states, before any GPU work
    wants, deltas = [], []
    for rnd in range(3):
        wants.append(oracle.masks(s_lits, s_off, values_vm=vm, mode=mode))
        if rnd < 2:
            flip = flips[rnd]
            vm[flip - 1] = -vm[flip - 1]
            deltas.append((flip.astype(np.uint32), torch.from_numpy(np.ascontiguousarray(vm[flip - 1])).cuda()))

    def check(rnd, n):
        r = ctx.fetch_reports(n)
        assert len(r) == n
        key = r["clause_id"].astype(np.uint64) * np.uint64(W) + r["word"]
        assert len(np.unique(key)) == n
        assert (r["mask"] != 0).all() and (r["word"] < W).all() and (r["clause_id"] < N).all()
        pos = np.searchsorted(sample, r["clause_id"])
        hit = (pos < len(sample)) & (sample[np.minimum(pos, len(sample) - 1)] == r["clause_id"])
        got = np.zeros((len(sample), W), dtype=np.uint64)
        got[pos[hit], r["word"][hit]] = r["mask"][hit]
        print(f"paper scale round {rnd}: {n} records, sample of {len(sample)} clauses", flush=True)
        assert np.array_equal(got, wants[rnd]), mismatch_summary(got, wants[rnd])
        return got

    with gss.Context(V, A, report_capacity=1 << 20) as ctx:
        ids = ctx.add_clauses(w.lits, w.offsets)
        assert ids[-1] == N - 1
        ctx.set_assignments(0, w.values)
        print("paper scale: store and planes ready", flush=True)
        # round 0 synchronously (it also sizes the report segments)
        got = check(0, ctx.test(flags))
        # every planted (clause, slot) is falsified, hence also triggers
        gi = np.searchsorted(sample, w.planted[:, 0])
        bits = (got[gi, w.planted[:, 1] // 64] >> (w.planted[:, 1] % 64).astype(np.uint64)) & np.uint64(1)
        assert bits.all()
        # rounds 1 and 2 as the benchmark runs them: each delta queued on the device,
        # the second one behind the test of round 1 still in flight
        ctx.set_var_values_async(0, *deltas[0])
        ctx.test_async(flags)
        ctx.set_var_values_async(0, *deltas[1])
        check(1, ctx.test_wait())
        ctx.test_async(flags)
        check(2, ctx.test_wait())
