"""Hot-variable ranking (GPU): the library counts variable occurrences in the
stored clauses and renumbers its variables internally so that the most frequent
own the LDS-staged rows (Section 7, Conclusion).  The renumbering must be
invisible: every output equals the oracle's, with staging on and off, through
full sets, var-major deltas, packed word updates, removals, inserts and a served
session; and the staged variables must be the most frequent ones whatever
numbers the caller gave them (Zipf frequencies over shuffled variable ids)."""
import numpy as np
import pytest

from gpu_helpers import full_values, gpu_dense, mismatch_summary, new_context, oracle_dense
from paper_2012_03119_amd import gen, gss

pytestmark = pytest.mark.gpu


def _check(got, want):
    assert got.shape == want.shape
    assert np.array_equal(got, want), mismatch_summary(got, want)


def _shuffled_zipf_store(seed, n_clauses, n_vars, s=1.1):
    """Clauses whose variables follow Zipf(s) frequencies, with the variable
    numbers shuffled: the most frequent variable is not variable 1."""
    rng = np.random.default_rng(seed)
    lengths = rng.integers(1, 40, n_clauses)
    lits, offs = gen.random_clauses(rng, lengths, n_vars, gen.zipf_weights(n_vars, s))
    rename = np.concatenate([[0], 1 + rng.permutation(n_vars)]).astype(np.int64)
    lits = (np.sign(lits) * rename[np.abs(lits)]).astype(np.int32)
    return lits, offs


def _top_share(lits, n_vars, H):
    counts = np.bincount(np.abs(lits), minlength=n_vars + 1)[1:]
    return int(np.sort(counts)[::-1][:H].sum())


@pytest.mark.parametrize("max_slots,mode", [(64, "falsified"), (1024, "falsified"), (1024, "trigger")])
def test_ranked_staging_equals_oracle_on_shuffled_zipf(max_slots, mode):
    n_vars, H = 4000, 63
    lits, offs = _shuffled_zipf_store(5, 6000, n_vars)
    rng = np.random.default_rng(6)
    vals_n = gen.assignments_bernoulli(rng, max_slots, n_vars, rng.uniform(0.5, 0.95, max_slots))
    vals, active = full_values(vals_n, max_slots)
    flags = gss.GSS_TEST_TRIGGER if mode == "trigger" else 0
    n = len(offs) - 1
    with new_context(n_vars, max_slots, hot_vars=H) as ctx:
        ctx.add_clauses(lits, offs)
        ctx.set_assignments(0, vals_n)
        print(f"rank: first test ranks ({max_slots} slots, {mode})", flush=True)
        _check(gpu_dense(ctx, n, flags), oracle_dense(lits, offs, vals, active, mode))
        hot, stored = ctx.rank_vars()  # already ranked: the same counts, nothing moves
        assert stored == len(lits)
        assert hot == _top_share(lits, n_vars, H), "the staged variables are not the most frequent"
        assert hot > 0.1 * stored  # Zipf(1.1): the 63 most frequent carry a large share
        _check(gpu_dense(ctx, n, flags | gss.GSS_TEST_NO_HOT), oracle_dense(lits, offs, vals, active, mode))
        # deltas by external variable number: var-major values, then packed words
        flip = 1 + rng.choice(n_vars, n_vars // 5, replace=False).astype(np.uint32)
        vals[:, flip - 1] = -vals[:, flip - 1]
        ctx.set_var_values(0, flip, np.ascontiguousarray(vals[:, flip - 1].T))
        _check(gpu_dense(ctx, n, flags), oracle_dense(lits, offs, vals, active, mode))
        w = max_slots // 64 - 1
        some = 1 + rng.choice(n_vars, 300, replace=False).astype(np.uint32)
        new_vals = rng.choice(np.array([-1, 0, 1], dtype=np.int8), size=(64, len(some)))
        vals[64 * w:64 * w + 64][:, some - 1] = new_vals
        bits = np.uint64(1) << np.arange(64, dtype=np.uint64)
        f = ((new_vals == -1).astype(np.uint64) * bits[:, None]).sum(axis=0).astype(np.uint64)
        t = ((new_vals == 1).astype(np.uint64) * bits[:, None]).sum(axis=0).astype(np.uint64)
        ctx.update_words(w, some, f, t)
        _check(gpu_dense(ctx, n, flags), oracle_dense(lits, offs, vals, active, mode))
        _check(gpu_dense(ctx, n, flags | gss.GSS_TEST_AGGREGATE), oracle_dense(lits, offs, vals, active, mode))


def test_store_growth_reranks_and_inserts_use_the_new_numbers():
    n_vars, H, max_slots = 3000, 40, 256
    lits1, offs1 = _shuffled_zipf_store(11, 3000, n_vars)
    lits2, offs2 = _shuffled_zipf_store(12, 9000, n_vars)  # other hot variables, three times as many clauses
    rng = np.random.default_rng(13)
    vals_n = gen.assignments_bernoulli(rng, max_slots, n_vars, 0.8)
    vals, active = full_values(vals_n, max_slots)
    with new_context(n_vars, max_slots, hot_vars=H) as ctx:
        ids1 = ctx.add_clauses(lits1, offs1)
        ctx.set_assignments(0, vals_n)
        gpu_dense(ctx, len(ids1))
        hot1, _ = ctx.rank_vars()
        assert hot1 == _top_share(lits1, n_vars, H)
        ctx.add_clauses(lits2, offs2)  # encoded with the first ranking's numbers
        lits = np.concatenate([lits1, lits2])
        offs = np.concatenate([offs1, offs1[-1] + offs2[1:]])
        n = len(offs) - 1
        print("rank: the store tripled; the next test ranks again", flush=True)
        _check(gpu_dense(ctx, n), oracle_dense(lits, offs, vals, active))
        hot, stored = ctx.rank_vars()
        assert stored == len(lits) and hot == _top_share(lits, n_vars, H)
        # removals and a test with staging off
        gone = rng.choice(n, n // 3, replace=False).astype(np.uint32)
        ctx.remove_clauses(gone)
        keep = np.ones(n, dtype=bool)
        keep[gone] = False
        want = oracle_dense(lits, offs, vals, active)
        want[~keep] = 0
        _check(gpu_dense(ctx, n), want)
        _check(gpu_dense(ctx, n, gss.GSS_TEST_NO_HOT), want)


def test_served_session_on_a_ranked_context(tmp_path):
    from test_gpu_serve import replay
    W, P, n_vars = 4, 4, 3000
    lits, offs = _shuffled_zipf_store(21, 15_000, n_vars)
    ctx = gss.Context(n_vars, W * 64, hot_vars=60)
    ctx.add_clauses(lits, offs)
    hot, stored = ctx.rank_vars()
    assert hot == _top_share(lits, n_vars, 60) and stored == len(lits)
    log = tmp_path / "serve.log"
    print("rank: served session over renumbered variables", flush=True)
    res = ctx.serve_simulate(n_threads=P, duration_s=1.0, snapshot_rate=25.0, redraw_fraction=0.05,
                             insert_rate=400.0, delete_fraction=0.1, seed=8, log_path=str(log))
    counts, clauses, F, T = replay(str(log), lits, offs, n_vars, W)
    assert counts["E"] >= 5 and res["inserted"] == counts["A"] > 0
    ctx.close()


def test_rank_errors():
    with new_context(100, 64, hot_vars=10) as ctx:
        assert ctx.rank_vars() == (0, 0)  # an empty store: nothing to rank
        ctx.add_clauses(np.array([1, 2, -3], dtype=np.int32), np.array([0, 3], dtype=np.int64))
        ctx.set_active(np.full(1, 2**64 - 1, dtype=np.uint64))
        ctx.test_async()
        with pytest.raises(gss.GssError) as e:
            ctx.rank_vars()
        assert e.value.code == gss.GSS_ERR_STATE
        ctx.test_wait()
    with new_context(100, 64) as ctx:  # no staging: no ranking
        ctx.add_clauses(np.array([1, 2, -3], dtype=np.int32), np.array([0, 3], dtype=np.int64))
        assert ctx.rank_vars() == (0, 0)
