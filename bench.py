#!/usr/bin/env python3
"""Throughput of the clause test on one MI355X, at the paper's scale.

Workload (default): 4,000,000 clauses over 1,000,000 variables with the length
mix 50% in [2,10], 40% in [11,50], 10% in [51,300]; 1024 assignment slots (16
words) with an assigned fraction uniform in [0.3, 0.9] per slot; planted hits at
rate 1e-5; between rounds 5% of the variables flip (T <-> F in every slot).

One step = one round of the hot path: the round's delta (new values of the
flipped variables, already resident in HBM) is packed into the bitplanes, then
every live clause is tested against every active slot and the reports are
compacted in HBM (count read back).  value = clauses x slots tested per second.

The JSON line also carries the roofline of the test kernel (algorithmic bytes per
launch over its HIP-event duration, against 8 TB/s) and the oracle's rate on the
host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_test_paper_4Mx1024_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    from paper_2012_03119_amd.profile_summary import kernel_hash as h
    return h()


def make_workload(args):
    from paper_2012_03119_amd import gen
    if args.workload == "tiny":
        return gen.tiny(args.seed), "plain test, tiny: 20k clauses x 2k vars, 64 assignments"
    shuffle = args.seed + 77 if args.zipf_shuffle else None
    weights = gen.zipf_weights(args.vars, args.zipf, shuffle) if args.zipf else None
    w = gen.paper(args.seed, n_clauses=args.clauses, n_vars=args.vars, n_slots=args.slots, var_weights=weights)
    desc = (f"plain test, paper scale: {args.clauses} clauses x {args.vars} vars, {args.slots} assignments, "
            f"length mix 50%[2,10] 40%[11,50] 10%[51,300], 5% variable flips per round")
    if args.zipf:
        desc += (f", Zipf({args.zipf}) variable frequencies "
                 + ("over shuffled variable numbers" if args.zipf_shuffle else "(variable 1 most frequent)"))
    return w, desc


def stage_rounds(w, n_rounds, seed, torch):
    """Per round, the flipped variables and their new values (var-major), on the
    GPU: n_rounds distinct rounds, each applied on top of the previous one."""
    from paper_2012_03119_amd import gen
    vm = np.ascontiguousarray(w.values.T)  # var-major: a round's delta is a set of rows
    rounds = []
    for flip in gen.flip_rounds(seed + 1000, w.n_vars, n_rounds + 1):  # rounds 1..n_rounds
        vm[flip - 1] = -vm[flip - 1]
        rounds.append((flip.astype(np.uint32), torch.from_numpy(np.ascontiguousarray(vm[flip - 1])).cuda()))
    return rounds


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, seconds):
    """The oracle, untuned, over a bounded sample of clauses: on all the host
    threads OpenMP uses (the reported value), then on one thread (about a fifth
    of the time budget, on a smaller sample)."""
    import oracle
    vm = oracle.transpose(w.values)

    def run(n):
        lits = w.lits[: w.offsets[n]]
        offs = w.offsets[: n + 1]
        t0 = time.perf_counter()
        oracle.masks(lits, offs, values_vm=vm)
        return time.perf_counter() - t0

    def sample(budget):
        n = min(w.n_clauses, 2000)
        t = run(n)
        n2 = int(min(w.n_clauses, max(n, n * budget / max(t, 1e-6))))
        if n2 > n:
            n, t = n2, run(n2)
        return n, t

    cores = oracle.max_threads()
    n, t = sample(seconds)
    try:
        oracle.set_threads(1)
        n1, t1 = sample(seconds / 5)
    finally:
        oracle.set_threads(cores)
    rate = n * w.n_slots / t
    return {"value": rate, "unit": "tests/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {w.n_clauses} clauses x {w.n_slots} assignments (round 0), "
                      f"{t:.1f} s; var-major transpose of the values not timed",
            "single_core": {"value": n1 * w.n_slots / t1, "unit": "tests/s",
                            "sample": f"first {n1} clauses, {t1:.1f} s on 1 thread"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


#: the batched workload: (clauses, variables, assignment slots) of 8 independent
#: databases, sizes uneven and variable counts deliberately mismatched to them
BATCHED_STORES = ((100_000, 2_000_000, 1024), (250_000, 50_000, 64), (500_000, 1_180_000, 512),
                  (1_000_000, 85_000, 128), (1_500_000, 698_000, 768), (2_000_000, 144_000, 256),
                  (2_500_000, 412_000, 384), (3_000_000, 243_000, 192))


def bench_batched(args, torch, gss):
    """8 databases in one persistent launch (autotuned schedule, hipGraph replay)
    against the same rounds run database by database with gss_test."""
    from paper_2012_03119_amd import autotune, gen
    t0 = time.perf_counter()
    stream = torch.cuda.Stream()
    stores = []
    n_rounds = min(max(args.warmup, 8) + 2 * args.steps + 1, 40)
    for i, (n, v, a) in enumerate(BATCHED_STORES):
        w = gen.paper(300 + i, n_clauses=n, n_vars=v, n_slots=a)
        ctx = gss.Context(v, a, stream=stream, report_capacity=1 << 22)
        ctx.add_clauses(w.lits, w.offsets)
        ctx.set_assignments(0, w.values)
        rounds = stage_rounds(w, n_rounds, 300 + i, torch)
        stores.append((w, ctx, rounds))
        del w
    log(f"batched workload ready in {time.perf_counter() - t0:.1f} s")
    batch = gss.Batch([s[1] for s in stores])
    shapes = [(n, v, a) for n, v, a in BATCHED_STORES]
    tune = autotune.autotune(batch, shapes, torch.cuda.get_device_name(0), reps=2, use_cache=False)
    log(f"autotuned schedule: order {tune['order']} chunk {tune['chunk_tiles']} blocks/CU {tune['blocks_per_cu']} "
        f"({tune['ms']:.3f} ms)")

    def deltas(i):  # queued: checked on the device, reported by the test that follows
        for w, ctx, rounds in stores:
            vs, delta = rounds[i % len(rounds)]
            ctx.set_var_values_async(0, vs, delta)

    # warm-up rounds cover every slot of each context's upload ring, which grows to
    # the size of a store's delta on first use
    warm = max(args.warmup, 8)

    def store_delta(s, i):
        _, ctx, rounds = stores[s]
        vs, delta = rounds[i % len(rounds)]
        ctx.set_var_values_async(0, vs, delta)

    # A round is every store's delta and test.  Both forms pipeline the rounds the
    # same way: the next round's deltas are queued behind the test in flight, so
    # their host work overlaps the kernels (batched: gss_batch_test_async, the 8
    # deltas, gss_batch_wait; plain: per store gss_test_async, its next delta,
    # gss_test_wait).
    def round_batched(i, last):
        batch.test_async(gss.GSS_TEST_GRAPH)
        if not last:
            deltas(i + 1)
        batch.wait()

    def round_plain(i, last):
        for s, (_, ctx, _) in enumerate(stores):
            ctx.test_async()
            if not last:
                store_delta(s, i + 1)
            ctx.test_wait()

    def run(round_fn, tests_fn):
        """(ms per round with the deltas, ms per round of the tests alone)"""
        deltas(0)
        for i in range(warm):
            round_fn(i, False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(warm, warm + args.steps):
            round_fn(i, i == warm + args.steps - 1)
        torch.cuda.synchronize()
        t_round = (time.perf_counter() - t) / args.steps
        t_test = 0.0  # the tests alone: each round's deltas applied, untimed, first
        for i in range(args.steps):
            deltas(warm + args.steps + i)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tests_fn()
            torch.cuda.synchronize()
            t_test += time.perf_counter() - t1
        return t_round, t_test / args.steps

    def batched_tests():
        batch.test(gss.GSS_TEST_GRAPH)

    def plain_tests():
        for _, ctx, _ in stores:
            ctx.test()

    t_batch, t_batch_test = run(round_batched, batched_tests)
    graph_ms = batch.info()["last_ms"]
    t_plain, t_plain_test = run(round_plain, plain_tests)
    pairs = sum(ctx.stats()["last_pairs"] for _, ctx, _ in stores)
    out = {
        "metric": "clause x assignment tests/sec (batched: 8 databases, one persistent launch)",
        "value": pairs / t_batch, "unit": "tests/s", "n_gpus": 1, "steps": args.steps, "warmup": warm,
        "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched: 8 databases of 0.1M-3M clauses over 50k-2M variables, 64-1024 "
                               "assignments, length mix, 5% flips per round",
                   "stores": [list(x) for x in BATCHED_STORES], "schedule": {k: tune[k] for k in
                   ("order", "chunk_tiles", "blocks_per_cu")}, "graph_launch_ms": graph_ms},
        "tests_ms_per_round": t_batch_test * 1e3,
        "plain": {"value": pairs / t_plain, "ms_per_step": t_plain * 1e3, "tests_ms_per_round": t_plain_test * 1e3,
                  "how": "the same rounds, one gss_test_async/gss_test_wait per database, each database's next "
                         "delta queued behind its test"},
        "how": "rounds pipelined: gss_batch_test_async, the next round's 8 queued deltas, gss_batch_wait",
        "speedup_vs_plain": t_plain / t_batch,
        "tests_speedup_vs_plain": t_plain_test / t_batch_test,
    }
    log(f"batched {t_batch * 1e3:.3f} ms/step vs plain {t_plain * 1e3:.3f} ms/step; tests alone "
        f"{t_batch_test * 1e3:.3f} vs {t_plain_test * 1e3:.3f} ms")
    batch.close()
    for _, ctx, _ in stores:
        ctx.close()
    print(json.dumps(out), flush=True)


def bench_served(args, torch, gss):
    """The served configuration: 32 simulated solver threads, each sending a
    Poisson stream of 64-assignment snapshots (200/s, 5% of the variables redrawn
    per snapshot, Table 1 values) and inserting 20,000 clauses/s, 2% of the live
    store removed per second, over a resident 8M-clause store on 2M variables
    under a 64 GB budget.  Reports tests/s and notify latency, then the plain test
    of the final store with every word active on the same GPU."""
    from paper_2012_03119_amd import gen
    V, P, n0 = 2_000_000, 32, args.serve_clauses
    t0 = time.perf_counter()
    rng = np.random.default_rng(args.seed + 400)
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n0), V)
    log(f"served store generated in {time.perf_counter() - t0:.1f} s: {n0} clauses, {len(lits)} literals")
    budget = int(args.serve_budget_gb * 2**30)
    ctx = gss.Context(V, P * 64, hbm_budget_bytes=budget, report_capacity=1 << 22)
    ctx.add_clauses(lits, offs)
    del lits, offs
    log(f"store resident ({ctx.store_info()['device_bytes'] / 2**30:.2f} GiB); serving for {args.serve_seconds:.0f} s")
    res = ctx.serve_simulate(n_threads=P, duration_s=args.serve_seconds, snapshot_rate=200.0, redraw_fraction=0.05,
                             insert_rate=20_000.0, delete_fraction=0.02, seed=args.seed + 401,
                             test_flags=gss.GSS_TEST_AGGREGATE if args.aggregate else 0,
                             evict_keep=args.evict_keep)
    log(f"served: {res['runs']} runs, {res['tested']} snapshots tested, {res['dropped']} dropped, "
        f"p50 {res['p50_ms']:.2f} ms p99 {res['p99_ms']:.2f} ms, {res['live_end']} live clauses, "
        f"{res['evictions']} evictions ({res['evicted']} clauses)")
    # the plain test on the final store, every word active
    ctx.set_active(np.full(P, 2**64 - 1, dtype=np.uint64))
    flags = gss.GSS_TEST_AGGREGATE if args.aggregate else 0
    for _ in range(2):
        ctx.test(flags)
    ctx.reset_stats()
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = 10
    for _ in range(reps):
        ctx.test(flags)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t) / reps
    st = ctx.stats()
    ctx.close()
    value = res["pairs"] / res["wall_s"]
    out = {
        "metric": "clause x assignment tests/sec (served: continuous batching, notify latency)",
        "value": value, "unit": "tests/s", "n_gpus": 1, "steps": res["runs"], "warmup": 0,
        "ms_per_step": res["wall_s"] * 1e3 / max(res["runs"], 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "served: 32 solver threads x 200 snapshots/s of 64 assignments (5% of 2M variables "
                               "redrawn per snapshot, Table 1 values), 20k inserts/s/thread (length mix), 2%/s "
                               "removals, 8M-clause resident store, 64 GB budget",
                   "seconds": args.serve_seconds, "initial_clauses": n0, "budget_bytes": budget,
                   "evict_keep": args.evict_keep},
        "latency_ms": {k: res[k + "_ms"] for k in ("p50", "p99", "mean", "max")},
        "served": {k: res[k] for k in ("snapshots", "tested", "dropped", "runs", "overflowed_runs", "inserted",
                                       "refused", "deleted", "reports", "live_end", "delta_bytes", "gpu_ms",
                                       "evictions", "evicted", "device_bytes_end")},
        "manager_ms": {k: round(res[k + "_ms"], 1) for k in ("admit", "wait", "fetch", "route", "store", "launch")},
        "dropped_ratio": res["dropped"] / max(res["snapshots"], 1),
        "gpu_busy": res["gpu_ms"] / (res["wall_s"] * 1e3),
        "plain": {"value": st["last_pairs"] / t_plain, "ms_per_test": t_plain * 1e3,
                  "kernel_ms": st["total_kernel_ms"] / max(st["timed_launches"], 1),
                  "how": "gss_test of the final store, all 2048 slots active", "flags": flags},
    }
    print(json.dumps(out), flush=True)


def table1_words(rng, n):
    """(F, T) words of n variables in one 64-slot word: each variable draws a value
    subset with the Table 1 ratios, then every slot a value inside the subset."""
    from paper_2012_03119_amd import gen
    subsets = [sub for sub, _ in gen.TABLE1_SUBSETS]
    p = np.array([w for _, w in gen.TABLE1_SUBSETS], dtype=np.float64)
    pick = rng.choice(len(subsets), size=n, p=p / p.sum())
    x = rng.integers(0, 2**63, size=n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=n, dtype=np.int64).astype(np.uint64)
    y = rng.integers(0, 2**63, size=n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=n, dtype=np.int64).astype(np.uint64)
    f = np.zeros(n, dtype=np.uint64)
    t = np.zeros(n, dtype=np.uint64)
    for k, sub in enumerate(subsets):
        m = pick == k
        vals = set(sub)
        if vals == {1}:
            t[m] = ~np.uint64(0)
        elif vals == {-1}:
            f[m] = ~np.uint64(0)
        elif vals == {1, -1}:
            f[m], t[m] = x[m], ~x[m]
        elif vals == {1, 0}:
            t[m] = x[m]
        elif vals == {-1, 0}:
            f[m] = x[m]
        elif vals == {1, -1, 0}:  # two random bits per slot, redrawn where both are set
            a, b = x[m].copy(), y[m].copy()
            both = a & b
            while both.any():
                a = np.where(both != 0, (a & ~both) | (rng.integers(0, 2**63, size=len(a), dtype=np.int64)
                             .astype(np.uint64) & both), a)
                b = np.where(both != 0, (b & ~both) | (rng.integers(0, 2**63, size=len(b), dtype=np.int64)
                             .astype(np.uint64) & both), b)
                both = a & b
            f[m], t[m] = a, b
    return f, t


def bench_wide(args, torch, gss):
    """Rows wider than 4096 slots and the aggregate of aggregates (Section 7): a
    store tested against 16384 assignments (256 words in 4 super-groups of 4096
    slots).  Assignments are hierarchical: per super-group each variable draws a
    Table 1 value subset, each word keeps part of it, each slot draws inside its
    word's subset.  Times the test kernel without and with the aggregate pre-test
    (super-groups, then words, then slots), in both modes, and reports how many
    (clause, super-group) and (clause, word) aggregate tests are negative (numpy,
    from the definition, on a sample of clauses) and what the kernel's pre-test
    settled (GSS_TEST_COUNT)."""
    from paper_2012_03119_amd import gen
    V, N, S = args.wide_vars, args.wide_clauses, args.wide_slots
    n_super, n_words = S // 4096, S // 64
    rng = np.random.default_rng(args.seed + 700)
    t0 = time.perf_counter()
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, N), V)
    vals = gen.assignments_hierarchical(rng, n_super, V)
    log(f"wide workload ready in {time.perf_counter() - t0:.1f} s: {N} clauses over {V} variables, {S} slots")
    ctx = gss.Context(V, S, report_capacity=1 << 22)
    ctx.add_clauses(lits, offs)
    ctx.set_assignments(0, vals)
    AGG, TRIG = gss.GSS_TEST_AGGREGATE, gss.GSS_TEST_TRIGGER
    forms = {}
    for name, flags in (("falsified", 0), ("falsified_aggregate", AGG), ("trigger", TRIG),
                        ("trigger_aggregate", TRIG | AGG)):
        for _ in range(2):
            ctx.test(flags)
        torch.cuda.synchronize()
        ctx.reset_stats()
        for _ in range(args.steps):
            n = ctx.test(flags)
        st = ctx.stats()
        forms[name] = {"kernel_ms": st["total_kernel_ms"] / max(1, st["timed_launches"]), "reports": int(n)}
    settled = {}
    for name, flags in (("falsified", AGG), ("trigger", TRIG | AGG)):
        ctx.test(flags | gss.GSS_TEST_COUNT)
        st = ctx.stats()
        settled[name] = st["last_agg_settled"] / (st["live_clauses"] * n_words)
    pairs = ctx.stats()["last_pairs"]
    ctx.close()
    # Definition 7, falsified: an aggregate test is negative when some literal of the
    # clause is F in no slot of the group.  F-anywhere per (variable, group, sign).
    slots_f, slots_t = (vals == -1), (vals == 1)
    f_word = slots_f.reshape(n_words, 64, V).any(axis=1)    # [word][var]: v is F in some slot
    t_word = slots_t.reshape(n_words, 64, V).any(axis=1)
    f_sup = f_word.reshape(n_super, 64, V).any(axis=1)      # [super-group][var]
    t_sup = t_word.reshape(n_super, 64, V).any(axis=1)
    n_s = min(N, 20_000)
    neg_sup = neg_word = neg_word_in_pos_sup = pos_sup = 0
    for c in range(n_s):
        cl = lits[offs[c]:offs[c + 1]]
        v = np.abs(cl) - 1
        pos = cl > 0  # a positive literal is F where its variable is F
        sup_ok = np.where(pos[None, :], f_sup[:, v], t_sup[:, v]).all(axis=1)     # [n_super]
        word_ok = np.where(pos[None, :], f_word[:, v], t_word[:, v]).all(axis=1)  # [n_words]
        neg_sup += int((~sup_ok).sum())
        neg_word += int((~word_ok).sum())
        ok_rows = np.repeat(sup_ok, 64)
        pos_sup += int(ok_rows.sum())
        neg_word_in_pos_sup += int((~word_ok & ok_rows).sum())
    ratios = {"super_group_negative": neg_sup / (n_s * n_super), "word_negative": neg_word / (n_s * n_words),
              "word_negative_where_super_group_positive": neg_word_in_pos_sup / max(pos_sup, 1),
              "sample_clauses": n_s}
    plain_ms = forms["falsified"]["kernel_ms"]
    agg_ms = forms["falsified_aggregate"]["kernel_ms"]
    # the same algorithmic model as the plain workload: every literal and the table read once
    alg = 4 * int(offs[-1]) + 8 * N + 2 * (V + 1) * n_words * 8 + 16 * forms["falsified_aggregate"]["reports"]
    achieved = alg / (agg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "gss::k_test (wide rows, three-level aggregate pre-test)", "kernel_ms": round(agg_ms, 4),
                "alg_bytes_per_launch": alg,
                "alg_bytes": "4 B per stored literal + 8 B per clause + plane table once + 16 B per report"}
    out = {
        "metric": "clause x assignment tests/sec (wide rows: aggregate of aggregates, falsified)",
        "value": pairs / (agg_ms * 1e-3), "unit": "tests/s", "n_gpus": 1, "steps": args.steps, "warmup": 2,
        "ms_per_step": agg_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"wide rows: {N} clauses (length mix) over {V} variables x {S} hierarchical "
                               f"assignments ({n_super} super-groups of 64 words, Table 1 subsets, each word "
                               f"keeping 70% of its super-group's values)"},
        "forms": forms, "aggregate_speedup": plain_ms / agg_ms,
        "aggregate_speedup_trigger": forms["trigger"]["kernel_ms"] / forms["trigger_aggregate"]["kernel_ms"],
        "negative_ratios": ratios, "kernel_pretest_settled_ratio": settled, "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        import types
        log("timing the oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(types.SimpleNamespace(values=vals, lits=lits, offsets=offs, n_clauses=N,
                                                                 n_slots=S), args.cpu_seconds)
    log(f"wide: plain {plain_ms:.3f} ms, aggregate {agg_ms:.3f} ms ({plain_ms / agg_ms:.2f}x); trigger "
        f"{forms['trigger']['kernel_ms']:.3f} / {forms['trigger_aggregate']['kernel_ms']:.3f} ms; negative: super "
        f"{ratios['super_group_negative']:.4f}, word {ratios['word_negative']:.4f}; settled {settled}")
    print(json.dumps(out), flush=True)


def recency_params():
    """Hit recency as a network: any hit in the last 8 tested runs scores ~1, none
    scores 0.27 (weights set by hand)."""
    from paper_2012_03119_amd import gss
    recency = np.zeros(gss.MLP_PARAMS, dtype=np.float32)
    recency[4 * 64:12 * 64:64] = 1.0      # W1[4..11][0] = 1
    recency[832] = 1.0                    # W2[0][0] = 1
    recency[4992] = 100.0                 # w3[0]
    recency[5056] = -1.0                  # b3
    return recency


def bench_learned(args, torch, gss):
    """The learned schedule against the plain test on one stream: 32 words of
    Table 1 snapshots, 5% of the variables of each word redrawn per run, over an
    8M-clause store on 2M variables.  The network trains on the hit logs of the
    first runs; its threshold is the score under which at most 0.4% of the
    training positives fall.  On later runs each schedule (learned, hit recency,
    random with the learned one's budget) runs beside the plain test, which judges
    the hits each one misses."""
    from paper_2012_03119_amd import gen
    V, P, n0 = args.learn_vars, 32, args.learn_clauses
    rng = np.random.default_rng(args.seed + 500)
    t0 = time.perf_counter()
    lits, offs = gen.random_clauses(rng, gen.lengths_mix(rng, n0), V)
    lens = np.diff(offs)
    ctx = gss.Context(V, P * 64, hbm_budget_bytes=64 << 30, report_capacity=1 << 22)
    ids = ctx.add_clauses(lits, offs)
    n_s = min(n0, 200_000)  # clause sample for the aggregate-negative ratio
    s_lits, s_offs = lits[: offs[n_s]].copy(), offs[: n_s + 1].copy()
    del lits, offs
    ctx.priority_enable(n_sources=P, sample_period=args.learn_sample_period, sample_capacity=1 << 22,
                        seed=args.seed + 501)
    ctx.priority_set_clause_info(ids, (2 + rng.random(n0) * (np.maximum(lens, 2) - 2)).astype(np.float32),
                                 rng.integers(0, P, n0).astype(np.uint32))
    all_vars = np.arange(1, V + 1, dtype=np.uint32)
    # Section 4: a (clause, word) pair whose aggregate test is negative (some
    # literal is F in no slot of the word) cannot be falsified in that word
    # (falsified); trigger mode runs the recurrence of Section 4.3 over canBeFalse
    # and canBeUndef of the clause's literals, position by position
    s_var = np.abs(s_lits).astype(np.int64) - 1
    s_pos = s_lits > 0
    s_len = np.diff(s_offs)
    s_clause = np.repeat(np.arange(n_s), s_len)
    s_k = np.arange(len(s_lits)) - np.repeat(s_offs[:-1], s_len)  # position in the clause
    by_k = np.argsort(s_k, kind="stable")  # literal entries grouped by position
    k_start = np.searchsorted(s_k[by_k], np.arange(int(s_len.max()) + 1))
    agg_negative = agg_negative_trigger = 0
    for w in range(P):
        f, t = table1_words(rng, V)
        ctx.update_words(w, all_vars, f, t)
        cbf = np.where(s_pos, f[s_var] != 0, t[s_var] != 0)
        cbu = (f[s_var] | t[s_var]) != ~np.uint64(0)
        agg_negative += int(np.count_nonzero(np.bincount(s_clause[~cbf], minlength=n_s)))
        af = np.ones(n_s, dtype=bool)
        ou = np.zeros(n_s, dtype=bool)
        for k in range(int(s_len.max())):
            at = by_k[k_start[k]:k_start[k + 1]]
            c, lf, lu = s_clause[at], cbf[at], cbu[at]
            ou[c] = (af[c] & lu) | (ou[c] & lf)
            af[c] &= lf
        agg_negative_trigger += int(np.count_nonzero(~(af | ou)))
    agg_negative_ratio = agg_negative / (n_s * P)
    agg_negative_trigger_ratio = agg_negative_trigger / (n_s * P)
    del s_var, s_pos, s_clause, s_k
    ctx.set_active(np.full(P, 2**64 - 1, dtype=np.uint64))
    # what the test kernel's pre-test itself settled on the whole store (GSS_TEST_COUNT)
    settled = {}
    for name, fl in (("falsified", 0), ("trigger", gss.GSS_TEST_TRIGGER)):
        ctx.test(fl | gss.GSS_TEST_AGGREGATE | gss.GSS_TEST_COUNT)
        st = ctx.stats()
        settled[name] = st["last_agg_settled"] / (st["live_clauses"] * P)
    log(f"learned: store and snapshots ready in {time.perf_counter() - t0:.1f} s; aggregate-negative ratio "
        f"{agg_negative_ratio:.4f} (trigger {agg_negative_trigger_ratio:.4f}) over {n_s} clauses x {P} words; "
        f"the kernel's pre-test settled {settled['falsified']:.4f} (trigger {settled['trigger']:.4f}) of all "
        f"(clause, word) pairs")
    blocks = (V + 63) // 64

    def advance():  # every word redraws 5% of its variables, in runs of 64
        for w in range(P):
            b = rng.choice(blocks, size=max(1, int(0.05 * blocks)), replace=False)
            vs = (b[:, None] * 64 + np.arange(1, 65)[None, :]).ravel()
            vs = vs[vs <= V].astype(np.uint32)
            f, t = table1_words(rng, len(vs))
            ctx.update_words(w, vs, f, t)

    agg = gss.GSS_TEST_AGGREGATE if args.aggregate else 0

    wall = {}  # per schedule: wall time of the whole test call (list building included)

    def run_test(flags, name=None):
        torch.cuda.synchronize()
        t = time.perf_counter()
        n = ctx.test(flags | agg)
        if name:
            wall[name] = wall.get(name, 0.0) + time.perf_counter() - t
        r = ctx.fetch_reports(n)
        st = ctx.stats()
        bits = int(np.unpackbits(np.ascontiguousarray(r["mask"]).view(np.uint8)).sum()) if len(r) else 0
        return bits, st["last_kernel_ms"], st["last_pairs"]

    for r in range(args.learn_train_runs):
        run_test(0)
        ctx.priority_observe()
        advance()
    t1 = time.perf_counter()
    ctx.priority_set_sampling(0)  # the network is trained once: no samples while it schedules
    loss = ctx.priority_train(args.learn_epochs, batch=4096, lr=args.learn_lr, seed=args.seed + 502)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    info = ctx.priority_info()
    sx, sy = ctx.priority_samples(1 << 22)
    learned = ctx.priority_params()
    p = gss.gss_mlp_forward(ctx.ctx, learned, sx)
    pos = np.sort(p[sy > 0.5])
    tau = float(pos[int(args.learn_quantile * len(pos))]) if len(pos) else 0.5
    log(f"learned: {info['samples']} samples ({sy.mean():.3f} positive), trained in {t_train:.2f} s "
        f"(loss {loss:.4f}), threshold {tau:.4f}")
    recency = recency_params()
    sums = {k: [0, 0.0, 0] for k in ("plain", "learned", "recency", "random")}  # hit bits, kernel ms, runs
    plain_bits = {}
    low_frac, recency_low = [], []
    overhead = 0.0  # the learned schedule's own work per run: scoring (every K runs) and observing
    K = args.learn_rescore
    n_low_learned = None
    for r in range(args.learn_eval_runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        if r % K == 0:  # a full scoring every K runs, the changed clauses every U runs in between
            ctx.priority_params(set_to=learned)
            n_low_learned = ctx.priority_score(tau)
        elif r % args.learn_update == 0:
            n_low_learned = ctx.priority_update()
        torch.cuda.synchronize()
        overhead += time.perf_counter() - t
        low_frac.append(n_low_learned / n0)
        b, ms, _ = run_test(gss.GSS_TEST_SCHEDULED, "learned")
        sums["learned"][0] += b
        sums["learned"][1] += ms
        sums["learned"][2] += 1
        t = time.perf_counter()
        ctx.priority_observe()
        torch.cuda.synchronize()
        overhead += time.perf_counter() - t
        b, ms, pairs = run_test(0, "plain")
        plain_bits[r] = b
        sums["plain"][0] += b
        sums["plain"][1] += ms
        sums["plain"][2] += 1
        if r % K == K - 1:  # baselines on the same run (the next run scores everything again)
            ctx.priority_params(set_to=recency)
            recency_low.append(ctx.priority_score(0.5) / n0)
            b, ms, _ = run_test(gss.GSS_TEST_SCHEDULED)
            sums["recency"][0] += b
            sums["recency"][1] += ms
            sums["recency"][2] += 1
            low = np.zeros(n0, dtype=np.uint8)
            low[rng.choice(n0, size=n_low_learned, replace=False)] = 1
            ctx.priority_mark(low)
            b, ms, _ = run_test(gss.GSS_TEST_SCHEDULED)
            sums["random"][0] += b
            sums["random"][1] += ms
            sums["random"][2] += 1
            sums.setdefault("plain_at_baselines", [0, 0.0, 0])
            sums["plain_at_baselines"][0] += plain_bits[r]
        advance()
    R = args.learn_eval_runs
    plain_ms = sums["plain"][1] / R
    out_sched = {}
    for k in ("learned", "recency", "random"):
        runs = sums[k][2]
        if not runs:  # fewer evaluated runs than one rescoring cycle: no baseline run
            continue
        hits_plain = sums["plain"][0] if k == "learned" else sums["plain_at_baselines"][0]
        ms = sums[k][1] / max(runs, 1)
        out_sched[k] = {"kernel_ms": ms, "runs": runs, "speedup_vs_plain": plain_ms / ms if ms else None,
                        "missed_hit_rate": 1 - sums[k][0] / hits_plain if hits_plain else None}
    overhead_ms = overhead * 1e3 / R
    # end to end on the wall clock: each test call whole (host work, the scheduled
    # test's list building, the kernel, the wait), plus the schedule's upkeep
    plain_wall_ms = wall["plain"] * 1e3 / R
    sched_wall_ms = wall["learned"] * 1e3 / R
    out_sched["learned"]["overhead_ms_per_run"] = overhead_ms
    out_sched["learned"]["test_call_ms"] = sched_wall_ms
    out_sched["learned"]["plain_test_call_ms"] = plain_wall_ms
    out_sched["learned"]["end_to_end_speedup"] = plain_wall_ms / (sched_wall_ms + overhead_ms)
    out_sched["learned"]["end_to_end_speedup_kernels"] = plain_ms / (out_sched["learned"]["kernel_ms"] + overhead_ms)
    ctx.close()
    step_ms = sched_wall_ms + overhead_ms  # the whole scheduled test call plus the schedule's own work
    value = pairs / (step_ms * 1e-3)
    out = {
        "metric": "clause x assignment tests/sec (learned schedule; missed-hit rate judged by the plain test)",
        "value": value, "unit": "tests/s", "n_gpus": 1, "steps": R, "warmup": args.learn_train_runs,
        "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64+f32", "data": "synthetic",
        "config": {"workload": f"learned: {n0} clauses (length mix) over {V} variables, 32 words of Table 1 "
                               f"snapshots, 5% redrawn per run; MLP 12-64-64-1 fp32 trained on "
                               f"{args.learn_train_runs} runs of hit logs", "threshold": tau,
                   "low_fraction": float(np.mean(low_frac)),
                   "recency_low_fraction": float(np.mean(recency_low)) if recency_low else None,
                   "train_s": t_train, "samples": info["samples"],
                   "rescore_every": K, "update_every": args.learn_update, "aggregate": bool(args.aggregate),
                   "aggregate_negative_ratio": agg_negative_ratio,
                   "aggregate_negative_ratio_trigger": agg_negative_trigger_ratio,
                   "aggregate_negative_how": f"falsified aggregate test of {n_s} clauses x {P} words, first snapshot",
                   "kernel_pretest_settled_ratio": settled["falsified"],
                   "kernel_pretest_settled_ratio_trigger": settled["trigger"],
                   "kernel_pretest_how": "GSS_TEST_COUNT on the whole store, first snapshot: (clause, word) pairs "
                                         "the test kernel's aggregate pre-test settled before any gather killed "
                                         "them, over live clauses x words"},
        "plain_kernel_ms": plain_ms, "schedules": out_sched,
        "missed_hit_rate": out_sched["learned"]["missed_hit_rate"],
        "speedup_vs_plain": out_sched["learned"]["speedup_vs_plain"],
    }
    log(f"learned: plain {plain_ms:.3f} ms, " + ", ".join(
        f"{k} {v['kernel_ms']:.3f} ms missed {v['missed_hit_rate']:.4f}" for k, v in out_sched.items()) +
        f"; learned overhead {overhead_ms:.3f} ms/run, test calls {sched_wall_ms:.3f} against {plain_wall_ms:.3f} ms, "
        f"end to end {out_sched['learned']['end_to_end_speedup']:.2f}x"
        f"; low fraction learned {np.mean(low_frac):.3f}"
        + (f", recency {np.mean(recency_low):.3f}" if recency_low else ""))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--timing-interval", type=int, default=4,
                    help="plain workloads: time every n-th test kernel launch with HIP events (1: every one)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["paper", "tiny", "batched", "served", "learned", "wide"], default="paper")
    ap.add_argument("--wide-clauses", type=int, default=1_000_000)
    ap.add_argument("--wide-vars", type=int, default=50_000)
    ap.add_argument("--wide-slots", type=int, default=16384, help="a multiple of 4096")
    ap.add_argument("--learn-clauses", type=int, default=8_000_000)
    ap.add_argument("--learn-vars", type=int, default=2_000_000)
    ap.add_argument("--learn-train-runs", type=int, default=24)
    ap.add_argument("--learn-eval-runs", type=int, default=128)
    ap.add_argument("--learn-epochs", type=int, default=2)
    ap.add_argument("--learn-sample-period", type=int, default=64)
    ap.add_argument("--learn-rescore", type=int, default=128,
                    help="score every clause every K runs (only the changed ones in between)")
    ap.add_argument("--learn-update", type=int, default=16, help="rescore the changed clauses every U runs")
    ap.add_argument("--learn-lr", type=float, default=3e-3)
    ap.add_argument("--learn-quantile", type=float, default=0.004,
                    help="threshold: the score under which this fraction of the training positives fall")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-clauses", type=int, default=8_000_000)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0, help="HBM admission budget of the served store")
    ap.add_argument("--evict-keep", type=float, default=0.0,
                    help="served: when an insert does not fit the budget, evict the least active clauses down to "
                         "this fraction (0 = inserts wait)")
    ap.add_argument("--clauses", type=int, default=4_000_000)
    ap.add_argument("--vars", type=int, default=1_000_000)
    ap.add_argument("--slots", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--hot-vars", type=int, default=0, help="variables whose plane rows are staged in LDS")
    ap.add_argument("--zipf", type=float, default=0.0,
                    help="Zipf exponent of the variable frequencies (0: uniform, as in the paper-scale workload)")
    ap.add_argument("--stitch-steps", type=int, default=5,
                    help="extra steps that also stitch the records into one device list (timed apart)")
    ap.add_argument("--zipf-shuffle", action="store_true",
                    help="deal the Zipf frequencies to the variables in a random order")
    ap.add_argument("--report-capacity", type=int, default=1 << 20)
    ap.add_argument("--no-early-exit", action="store_true")
    ap.add_argument("--trigger", action="store_true")
    ap.add_argument("--aggregate", action="store_true",
                    help="aggregate pre-test of each 64-assignment word before reading plane rows")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration for profiles)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (a multi-GPU clause test "
              f"would shard the store by clause, which is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2012_03119_amd import gss

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {n} bytes 3 times")
        return

    if args.workload == "batched":
        bench_batched(args, torch, gss)
        return
    if args.workload == "served":
        bench_served(args, torch, gss)
        return
    if args.workload == "wide":
        bench_wide(args, torch, gss)
        return
    if args.workload == "learned":
        bench_learned(args, torch, gss)
        return

    t0 = time.perf_counter()
    w, desc = make_workload(args)
    log(f"workload ready in {time.perf_counter() - t0:.1f} s: {w.n_clauses} clauses, {len(w.lits)} literals")
    need_rounds = args.warmup + args.steps + args.stitch_steps if args.workload == "paper" else 0
    # every step applies a round of its own: nothing is recycled
    rounds = stage_rounds(w, need_rounds, args.seed, torch) if need_rounds else []

    flags = 0
    if args.no_early_exit:
        flags |= gss.GSS_TEST_NO_EARLY_EXIT
    if args.trigger:
        flags |= gss.GSS_TEST_TRIGGER
    if args.aggregate:
        flags |= gss.GSS_TEST_AGGREGATE
    # the context works on torch's current stream: inputs made there need no extra wait
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    # the test kernel is timed with HIP events on every timing_interval-th launch:
    # each event leaves the stream idle for a few microseconds per step
    ctx = gss.Context(w.n_vars, w.n_slots, hot_vars=args.hot_vars, report_capacity=args.report_capacity,
                      stream=stream, timing_interval=args.timing_interval)
    t0 = time.perf_counter()
    ctx.add_clauses(w.lits, w.offsets)
    log(f"clauses stored in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    ctx.set_assignments(0, w.values)
    log(f"assignments packed in {time.perf_counter() - t0:.1f} s")

    # A step applies one round's delta and tests the store.  Steps are pipelined:
    # round i+1's delta is queued on the device behind test i, so the device
    # applies it while the host collects test i's count and queues test i+1.
    def queue_delta(i):
        if rounds:
            vs, delta = rounds[i]
            ctx.set_var_values_async(0, vs, delta)

    def run_steps(first, n):
        if n <= 0:
            return 0
        queue_delta(first)
        ctx.test_async(flags)
        for i in range(first + 1, first + n):
            queue_delta(i)
            ctx.test_wait()
            ctx.test_async(flags)
        return ctx.test_wait()

    # one synchronous test first sizes the report segments (a pipelined test that
    # overflows is not repeated, since the next delta is already queued)
    n_rep = ctx.test(flags)
    n_rep = run_steps(0, args.warmup) or n_rep
    log(f"warmup done ({args.warmup} steps), {n_rep} reports per test")
    torch.cuda.synchronize()
    ctx.reset_stats()
    t0 = time.perf_counter()
    n_rep = run_steps(args.warmup, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ctx.stats()
    ms_per_step = elapsed * 1e3 / args.steps
    pairs = st["last_pairs"]
    value = pairs / (elapsed / args.steps)
    kernel_ms = st["total_kernel_ms"] / max(1, st["timed_launches"])

    # the same steps with each test's records also stitched into one device
    # list (the fetch the timed steps leave for the caller): not pipelined, so
    # this measures the step plus the stitch and the extra synchronisation
    stitch_ms = None
    if args.workload == "paper" and args.stitch_steps:
        k = min(args.stitch_steps, len(rounds) - args.warmup - args.steps) if rounds else 0
        dev = torch.empty((max(n_rep, 1) * 5 // 4 + 4096) * 2, dtype=torch.int64, device="cuda")
        if k > 0:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.warmup + args.steps, args.warmup + args.steps + k):
                queue_delta(i)
                n_i = ctx.test(flags)
                gss.gss_fetch_reports_into(ctx.ctx, dev.data_ptr(), min(n_i, dev.numel() // 2))
            torch.cuda.synchronize()
            stitch_ms = (time.perf_counter() - t0) * 1e3 / k
            log(f"{k} steps with the records stitched into one device list: {stitch_ms:.3f} ms/step")
    hot_share = None
    if args.hot_vars:
        hot, stored = ctx.rank_vars()
        hot_share = hot / stored if stored else None

    W = w.n_slots // 64
    table_bytes = 2 * (w.n_vars + 1) * W * 8
    alg_bytes = 4 * st["last_literals"] + 8 * st["live_clauses"] + table_bytes + 16 * st["last_reports"]
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_sha256_16") == kernel_hash() and tr.get("config") == desc:
            traffic = tr.get("hbm_bytes_per_launch")
    # the counters' bytes over the same kernel time: how close the real traffic runs to the peak
    traffic_gbs = traffic / (kernel_ms * 1e-3) / 1e9 if traffic else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_GBps": round(traffic_gbs, 1) if traffic_gbs else None,
                "traffic_frac": round(traffic_gbs / HBM_PEAK_GBS, 4) if traffic_gbs else None,
                "kernel": "gss::k_test", "kernel_ms": round(kernel_ms, 4), "alg_bytes_per_launch": alg_bytes,
                "timed_launches": st["timed_launches"], "launches": st["kernel_launches"],
                "alg_bytes": "4 B per stored literal + 8 B per clause (length, id) + plane table once "
                             "(2 rows x W words x 8 B per variable) + 16 B per report"}
    log(f"{args.steps} steps: {ms_per_step:.3f} ms/step, test kernel {kernel_ms:.3f} ms, "
        f"{value / 1e12:.2f} T tests/s, {achieved:.0f} GB/s algorithmic, {n_rep} reports")

    out = {
        "metric": "clause x assignment tests/sec", "value": value, "unit": "tests/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": desc, "clauses": w.n_clauses, "vars": w.n_vars, "assignments": w.n_slots,
                   "seed": args.seed, "flags": flags, "hot_vars": args.hot_vars,
                   "reports_per_test": n_rep, "gpu": torch.cuda.get_device_name(0)},
        "roofline": roofline,
        "ms_per_step_with_stitch": round(stitch_ms, 4) if stitch_ms else None,
    }
    if hot_share is not None:
        out["config"]["hot_literal_share"] = round(hot_share, 4)
    ctx.close()
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
