"""Seeded synthetic workloads shaped like the paper's: clause databases and
partial assignments.

This module only draws inputs.  It holds none of the clause test's arithmetic:
no bitplanes, no masks.  Both the HIP library's tests and the oracle read what it
produces, so it is the one module the two sides share.

Shapes follow the paper's facts about its workload (millions of learned clauses,
many of them long, up to 1024 assignments per GPU run, per-thread snapshots with
the value-subset ratios of Table 1); the paper's own SAT-competition instances are
not used, and these inputs stand in for them.

Encodings: literals are DIMACS int32 (variable v in 1..n_vars, -v its negation),
clause c is ``lits[offsets[c]:offsets[c+1]]``, truth values are int8 (+1 T, -1 F,
0 U) in slot-major arrays ``values[slot][var-1]``.  Every draw comes from
``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

T, F, U = 1, -1, 0


@dataclass
class Workload:
    """A clause database plus one set of assignments."""
    name: str
    n_vars: int
    lits: np.ndarray          # int32, DIMACS literals, concatenated clauses
    offsets: np.ndarray       # int64 [n_clauses + 1]
    values: np.ndarray        # int8 [n_slots][n_vars]
    planted: np.ndarray       # int64 [n_planted][2]: (clause index, slot) made falsified
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n_clauses(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_slots(self) -> int:
        return self.values.shape[0]

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def clause(self, c: int) -> np.ndarray:
        return self.lits[self.offsets[c]:self.offsets[c + 1]]


# ---------------------------------------------------------------------------
# clause lengths
# ---------------------------------------------------------------------------

def lengths_geometric(rng, n: int, p: float = 1.0 / 8.0, lo: int = 2, hi: int = 64) -> np.ndarray:
    """Geometric on {1, 2, ...} with success probability p (mean 1/p), clamped to [lo, hi]."""
    return np.clip(rng.geometric(p, size=n), lo, hi).astype(np.int64)


#: (probability, lo, hi) of the three length classes of the large workloads
LENGTH_MIX = ((0.5, 2, 10), (0.4, 11, 50), (0.1, 51, 300))


def lengths_mix(rng, n: int, mix=LENGTH_MIX) -> np.ndarray:
    """Each clause picks a class with the given probability, then a uniform integer
    length inside the class's inclusive range."""
    u = rng.random(n)
    out = np.empty(n, dtype=np.int64)
    edge = 0.0
    for k, (p, lo, hi) in enumerate(mix):
        sel = (u >= edge) & (u < edge + p) if k < len(mix) - 1 else (u >= edge)
        out[sel] = rng.integers(lo, hi + 1, size=int(sel.sum()))
        edge += p
    return out


# ---------------------------------------------------------------------------
# clause bodies
# ---------------------------------------------------------------------------

def _distinct_rows(rng, n_rows: int, length: int, n_vars: int, var_weights=None) -> np.ndarray:
    """n_rows rows of `length` distinct variables in 1..n_vars (uniform, or drawn
    from the cumulative weights `var_weights` when given).  Entries that repeat an
    earlier entry of their row are redrawn until every row is distinct."""
    if length > n_vars:
        raise ValueError("more distinct variables requested than exist")

    def draw(shape):
        if var_weights is None:
            return rng.integers(1, n_vars + 1, size=shape, dtype=np.int64)
        return np.searchsorted(var_weights, rng.random(shape), side="right").astype(np.int64) + 1

    rows = draw((n_rows, length))
    if length == 1:
        return rows
    todo = np.arange(n_rows)
    while len(todo):
        # rows that still hold a repeat (a plain sort is the cheap test)
        srt = np.sort(rows[todo], axis=1)
        todo = todo[(srt[:, 1:] == srt[:, :-1]).any(axis=1)]
        if len(todo) == 0:
            break
        sub = rows[todo]
        order = np.argsort(sub, axis=1, kind="stable")
        srt = np.take_along_axis(sub, order, axis=1)
        dup_sorted = np.zeros_like(srt, dtype=bool)
        dup_sorted[:, 1:] = srt[:, 1:] == srt[:, :-1]
        if not dup_sorted.any():
            break
        dup = np.zeros_like(dup_sorted)
        np.put_along_axis(dup, order, dup_sorted, axis=1)   # later copies of a value
        r_idx, c_idx = np.nonzero(dup)
        sub[r_idx, c_idx] = draw(len(r_idx))
        rows[todo] = sub
        todo = todo[np.unique(r_idx)]
    return rows


def random_clauses(rng, lengths: np.ndarray, n_vars: int, var_weights=None):
    """Clauses with the given lengths; variables distinct within a clause, in random
    order; each sign uniform.  Returns (lits int32, offsets int64).  Each distinct
    length draws from its own child generator, so the result does not depend on
    how many threads fill it."""
    n = len(lengths)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    lits = np.empty(int(offsets[-1]), dtype=np.int32)
    uniq = np.unique(lengths)
    if len(uniq) and uniq[-1] > n_vars:
        raise ValueError(f"clause length {uniq[-1]} exceeds the number of variables {n_vars}")
    seeds = rng.integers(0, 1 << 63, size=len(uniq))

    def fill(k):
        L = int(uniq[k])
        r = np.random.default_rng(int(seeds[k]))
        idx = np.flatnonzero(lengths == L)
        rows = _distinct_rows(r, len(idx), L, n_vars, var_weights)
        signs = r.integers(0, 2, size=rows.shape, dtype=np.int64) * 2 - 1
        pos = offsets[idx][:, None] + np.arange(L)[None, :]
        lits[pos] = (rows * signs).astype(np.int32)

    _parallel(fill, len(uniq))
    return lits, offsets


def _parallel(fn, n: int) -> None:
    """Runs fn(0..n-1) on a small thread pool (numpy releases the GIL in bulk ops)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1, n))
    if workers == 1:
        for k in range(n):
            fn(k)
        return
    with ThreadPoolExecutor(workers) as ex:
        for _ in ex.map(fn, range(n)):
            pass


# ---------------------------------------------------------------------------
# assignments
# ---------------------------------------------------------------------------

def assignments_bernoulli(rng, n_slots: int, n_vars: int, assigned_fraction, chunk: int = 16) -> np.ndarray:
    """Slot-major int8 [n_slots][n_vars].  In slot s each variable is assigned with
    probability assigned_fraction[s] (a scalar applies to all slots; resolution
    2^-16) and then T or F with probability 1/2 each; otherwise it is U.  Each
    chunk of slots draws from its own child generator."""
    frac = np.broadcast_to(np.asarray(assigned_fraction, dtype=np.float64), (n_slots,))
    thresh = np.floor(frac * 65536.0).astype(np.uint32)
    out = np.empty((n_slots, n_vars), dtype=np.int8)
    n_chunks = (n_slots + chunk - 1) // chunk
    seeds = rng.integers(0, 1 << 63, size=n_chunks)

    def fill(k):
        s0, s1 = k * chunk, min(n_slots, (k + 1) * chunk)
        r = np.random.default_rng(int(seeds[k]))
        raw = r.integers(0, 1 << 32, size=(s1 - s0, n_vars), dtype=np.uint32)
        assigned = (raw & np.uint32(0xFFFF)) < thresh[s0:s1, None]
        sign = (raw >> np.uint32(31)).astype(np.int8) * np.int8(2) - np.int8(1)
        np.multiply(sign, assigned, out=out[s0:s1])

    _parallel(fill, n_chunks)
    return out


#: Table 1 of the paper: how often each subset of {T, F, U} is the set of values a
#: variable takes over 32 successive assignments of one solver thread.
TABLE1_SUBSETS = (
    ((T,), 0.127), ((F,), 0.064), ((T, F), 0.000), ((U,), 0.660),
    ((T, U), 0.060), ((F, U), 0.068), ((T, F, U), 0.021),
)


def assignments_table1(rng, n_slots: int, n_vars: int) -> np.ndarray:
    """A group of n_slots correlated assignments, as one solver thread's successive
    snapshots: each variable draws a value subset with the Table 1 ratios
    (renormalised), then every slot draws its value uniformly inside the subset."""
    subsets = [s for s, _ in TABLE1_SUBSETS]
    p = np.array([w for _, w in TABLE1_SUBSETS], dtype=np.float64)
    p /= p.sum()
    pick = rng.choice(len(subsets), size=n_vars, p=p)
    out = np.empty((n_slots, n_vars), dtype=np.int8)
    r = rng.random((n_slots, n_vars))
    for k, sub in enumerate(subsets):
        cols = np.flatnonzero(pick == k)
        if len(cols) == 0:
            continue
        idx = np.minimum((r[:, cols] * len(sub)).astype(np.int64), len(sub) - 1)
        out[:, cols] = np.asarray(sub, dtype=np.int8)[idx]
    return out


def assignments_hierarchical(rng, n_super: int, n_vars: int, words_per_super: int = 64,
                             keep: float = 0.7) -> np.ndarray:
    """Assignments for aggregates of aggregates: n_super super-groups of
    words_per_super 64-slot groups.  Each variable draws a value subset per
    super-group with the Table 1 ratios; each group keeps every value of it with
    probability `keep` (at least one); each slot draws its value uniformly in its
    group's subset.  Returns int8 [n_super * words_per_super * 64][n_vars]."""
    vals_of = {m: np.array([v for bit, v in ((1, T), (2, F), (4, U)) if m & bit], dtype=np.int8) for m in range(1, 8)}
    sub_mask = np.array([sum({T: 1, F: 2, U: 4}[x] for x in sub) for sub, _ in TABLE1_SUBSETS], dtype=np.int64)
    p = np.array([w for _, w in TABLE1_SUBSETS], dtype=np.float64)
    p /= p.sum()
    out = np.empty((n_super * words_per_super * 64, n_vars), dtype=np.int8)
    for s in range(n_super):
        base = sub_mask[rng.choice(len(p), size=n_vars, p=p)]
        for w in range(words_per_super):
            kept = np.zeros(n_vars, dtype=np.int64)
            for bit in (1, 2, 4):
                kept |= np.where(rng.random(n_vars) < keep, bit, 0)
            mask = base & kept
            lowest = base & -base
            mask = np.where(mask == 0, lowest, mask)
            r = rng.random((64, n_vars))
            block = out[(s * words_per_super + w) * 64:(s * words_per_super + w + 1) * 64]
            for m, vals in vals_of.items():
                cols = np.flatnonzero(mask == m)
                if len(cols):
                    idx = np.minimum((r[:, cols] * len(vals)).astype(np.int64), len(vals) - 1)
                    block[:, cols] = vals[idx]
    return out


# ---------------------------------------------------------------------------
# planting
# ---------------------------------------------------------------------------

def plant(rng, lits: np.ndarray, offsets: np.ndarray, values: np.ndarray, n_planted: int) -> np.ndarray:
    """Rewrites n_planted distinct clauses so that each is falsified by one uniformly
    chosen slot: the clause keeps its length, its variables are redrawn without
    replacement among the variables assigned in that slot, and each sign is chosen
    so the literal is F there.  Returns [n_planted][2] (clause, slot)."""
    n = len(offsets) - 1
    n_slots, n_vars = values.shape
    clauses = rng.choice(n, size=n_planted, replace=False) if n_planted else np.zeros(0, np.int64)
    slots = rng.integers(0, n_slots, size=n_planted)
    for c, s in zip(clauses, slots):
        L = int(offsets[c + 1] - offsets[c])
        row = values[s]
        if n_vars <= 65536 and int(np.count_nonzero(row)) < L:
            raise ValueError("slot has fewer assigned variables than the clause length")
        pick = np.zeros(0, dtype=np.int64)
        while len(pick) < L:
            # rejection sampling: uniform candidates; keep assigned, distinct, new ones
            cand = rng.integers(0, n_vars, size=4 * L + 16)
            cand = cand[row[cand] != 0]
            _, first = np.unique(cand, return_index=True)
            cand = cand[np.sort(first)]
            cand = cand[~np.isin(cand, pick)]
            pick = np.concatenate([pick, cand[:L - len(pick)]])
        vals = row[pick].astype(np.int64)          # +1 or -1
        # the literal v is F when A(v) = F; the literal -v is F when A(v) = T
        lits[offsets[c]:offsets[c + 1]] = (-(pick + 1) * vals).astype(np.int32)
    return np.stack([clauses.astype(np.int64), slots.astype(np.int64)], axis=1)


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def tiny(seed: int = 1, n_clauses: int = 20_000, n_vars: int = 2_000, n_slots: int = 64,
         assigned: float = 0.6, planted_fraction: float = 0.02) -> Workload:
    """Plain test, tiny: 20,000 clauses over 2,000 variables, lengths geometric with
    mean 8 clamped to [2, 64], 64 assignments with each variable assigned with
    probability 0.6, 2% of the clauses planted to be falsified by one assignment."""
    rng = np.random.default_rng(seed)
    lengths = lengths_geometric(rng, n_clauses)
    lits, offsets = random_clauses(rng, lengths, n_vars)
    values = assignments_bernoulli(rng, n_slots, n_vars, assigned)
    planted = plant(rng, lits, offsets, values, int(round(planted_fraction * n_clauses)))
    return Workload("tiny", n_vars, lits, offsets, values, planted, seed,
                    meta=dict(assigned=assigned, planted_fraction=planted_fraction))


def paper(seed: int = 2, n_clauses: int = 4_000_000, n_vars: int = 1_000_000, n_slots: int = 1024,
          frac_lo: float = 0.3, frac_hi: float = 0.9, planted_rate: float = 1e-5,
          var_weights=None) -> Workload:
    """Plain test at the paper's scale: 4M clauses over 1M variables with the length
    mix (50% in [2,10], 40% in [11,50], 10% in [51,300]), 1024 assignments whose
    assigned fraction is uniform in [0.3, 0.9] per assignment, and planted
    (clause, assignment) pairs at rate 1e-5 of all pairs (distinct clauses).

    ``var_weights`` (a cumulative distribution over the variables) replaces the
    uniform choice of variables, e.g. with ``zipf_weights``."""
    rng = np.random.default_rng(seed)
    lengths = lengths_mix(rng, n_clauses)
    lits, offsets = random_clauses(rng, lengths, n_vars, var_weights)
    frac = rng.uniform(frac_lo, frac_hi, size=n_slots)
    values = assignments_bernoulli(rng, n_slots, n_vars, frac)
    n_planted = min(n_clauses, int(round(planted_rate * n_clauses * n_slots)))
    planted = plant(rng, lits, offsets, values, n_planted)
    return Workload("paper", n_vars, lits, offsets, values, planted, seed,
                    meta=dict(assigned_fraction=frac, planted_rate=planted_rate))


def zipf_weights(n_vars: int, s: float = 1.1, shuffle_seed=None) -> np.ndarray:
    """Cumulative Zipf(s) distribution over variables 1..n_vars: variable 1 most
    frequent, or, with ``shuffle_seed``, the same frequencies dealt to the
    variables in a seeded random order."""
    w = 1.0 / np.arange(1, n_vars + 1, dtype=np.float64) ** s
    if shuffle_seed is not None:
        w = w[np.random.default_rng(shuffle_seed).permutation(n_vars)]
    c = np.cumsum(w)
    return c / c[-1]


def flip_rounds(seed: int, n_vars: int, n_rounds: int, fraction: float = 0.05) -> List[np.ndarray]:
    """Per round r >= 1, the variables (1-based) whose values flip between round r-1
    and round r: a fraction of the variables drawn without replacement.  A flip
    swaps T and F in every slot where the variable is assigned; U stays U."""
    rng = np.random.default_rng(seed)
    k = int(round(fraction * n_vars))
    return [np.sort(rng.choice(n_vars, size=k, replace=False)).astype(np.int64) + 1
            for _ in range(max(0, n_rounds - 1))]


def apply_flips(values: np.ndarray, flipped_vars: np.ndarray) -> None:
    """Swaps T and F of the given variables in every slot, in place."""
    cols = np.asarray(flipped_vars, dtype=np.int64) - 1
    values[:, cols] = -values[:, cols]
