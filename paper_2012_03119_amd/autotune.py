"""Autotuner of the batched test's schedule.

Times every candidate schedule (tile order, chunk size, persistent workgroups
per compute unit) on the batch as it stands, keeps the fastest and records it in
a JSON cache keyed by the device and the stores' shapes, so a later run with the
same shapes starts from the cached choice.  Every schedule gives the same
results; only the time differs.
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Iterable, Optional, Sequence, Tuple

from . import gss

#: (order, chunk_tiles, blocks_per_cu) candidates
CANDIDATES: Tuple[Tuple[int, int, int], ...] = (
    (gss.GSS_ORDER_STORE, 0, 0),
    (gss.GSS_ORDER_INTERLEAVE, 16, 0),
    (gss.GSS_ORDER_INTERLEAVE, 64, 0),
    (gss.GSS_ORDER_INTERLEAVE, 256, 0),
    (gss.GSS_ORDER_LONGEST_FIRST, 64, 0),
    (gss.GSS_ORDER_LONGEST_FIRST, 256, 0),
    (gss.GSS_ORDER_INTERLEAVE, 64, 4),
    (gss.GSS_ORDER_LONGEST_FIRST, 64, 4),
)


def default_cache_path() -> str:
    return os.environ.get("GSS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gss", "autotune.json"))


def cache_key(device_name: str, shapes: Iterable[Tuple[int, int, int]]) -> str:
    """Device plus (clauses, variables, slots) of every store, in batch order."""
    return device_name + "|" + ";".join(f"{n}x{v}x{a}" for n, v, a in shapes)


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def autotune(batch: "gss.Batch", shapes: Sequence[Tuple[int, int, int]], device_name: str, *, flags: int = 0,
             reps: int = 3, candidates=CANDIDATES, cache_path: Optional[str] = None, use_cache: bool = True) -> dict:
    """Picks the fastest schedule for `batch` and leaves it set.  Returns
    {"order", "chunk_tiles", "blocks_per_cu", "ms", "source", "trials"}."""
    path = cache_path or default_cache_path()
    key = cache_key(device_name, shapes)
    cache = _load(path)
    if use_cache and key in cache:
        c = cache[key]
        batch.set_schedule(c["order"], c["chunk_tiles"], c["blocks_per_cu"])
        return dict(c, source="cache", trials=[])
    trials = []
    for order, chunk, bpc in candidates:
        batch.set_schedule(order, chunk, bpc)
        batch.test(flags)  # settles report segments; not timed
        times = []
        for _ in range(reps):
            batch.test(flags)
            times.append(batch.info()["last_ms"])
        trials.append(dict(order=order, chunk_tiles=chunk, blocks_per_cu=bpc, ms=statistics.median(times)))
    best = min(trials, key=lambda t: t["ms"])
    batch.set_schedule(best["order"], best["chunk_tiles"], best["blocks_per_cu"])
    cache[key] = best
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass
    return dict(best, source="measured", trials=trials)
