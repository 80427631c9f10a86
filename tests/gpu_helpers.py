"""Shared helpers of the GPU tests: run the HIP path through the C ABI and turn
its reports into dense masks that compare element by element with the oracle."""
import numpy as np

import oracle
from paper_2012_03119_amd import gss


def new_context(num_vars, max_slots, **kw):
    return gss.Context(num_vars, max_slots, **kw)


def reports_to_dense(r, n_ids, n_words):
    """Dense uint64 [n_ids][n_words] from report records; checks that records are
    unique per (clause, word) and never carry an empty mask."""
    key = r["clause_id"].astype(np.uint64) * np.uint64(n_words) + r["word"].astype(np.uint64)
    assert len(np.unique(key)) == len(r), "duplicate (clause, word) records"
    assert (r["mask"] != 0).all(), "record with an empty mask"
    assert (r["word"] < n_words).all()
    assert (r["clause_id"] < n_ids).all()
    dense = np.zeros((n_ids, n_words), dtype=np.uint64)
    dense[r["clause_id"], r["word"]] = r["mask"]
    return dense


def gpu_dense(ctx, n_ids, flags=0):
    n = ctx.test(flags)
    r = ctx.fetch_reports(n)
    assert len(r) == n
    return reports_to_dense(r, n_ids, ctx.n_words)


def full_values(values_by_slot, max_slots, first_slot=0):
    """Embeds [n][V] values at first_slot into [max_slots][V] with an active mask."""
    n, V = values_by_slot.shape
    vals = np.zeros((max_slots, V), dtype=np.int8)
    vals[first_slot:first_slot + n] = values_by_slot
    active = np.zeros(max_slots, dtype=bool)
    active[first_slot:first_slot + n] = True
    return vals, active


def oracle_dense(lits, offsets, vals, active, mode="falsified"):
    return oracle.masks(lits, offsets, vals, mode=mode, active=active)


def csr(clauses):
    offsets = np.zeros(len(clauses) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(c) for c in clauses])
    lits = np.array([l for c in clauses for l in c], dtype=np.int32)
    return lits, offsets


def mismatch_summary(got, want, limit=5):
    bad = np.argwhere(got != want)
    rows = [f"clause {i} word {w}: gpu {int(got[i, w]):#018x} oracle {int(want[i, w]):#018x}" for i, w in bad[:limit]]
    return f"{len(bad)} mismatching words; " + "; ".join(rows)
