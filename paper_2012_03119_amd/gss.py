"""Python binding of libgss (the C ABI in include/gss.h), by ctypes.

Argument marshalling only: every step of the clause test runs in the HIP library.
The module-level functions carry the ABI's names; ``Context`` wraps them for
convenience.  PyTorch, when present, provides device memory (the caching
allocator, through the allocator hooks) and the stream; nothing else.

The library must be built first (``python -m paper_2012_03119_amd.build``); if it
is missing, loading raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgss.so")

GSS_OK = 0
GSS_ERR_INVALID_ARG = -1
GSS_ERR_BAD_LITERAL = -2
GSS_ERR_UNKNOWN_ID = -3
GSS_ERR_CAPACITY = -4
GSS_ERR_REPORT_OVERFLOW = -5
GSS_ERR_DEVICE = -6
GSS_ERR_STATE = -7

GSS_TEST_FALSIFIED = 0
GSS_TEST_TRIGGER = 1
GSS_TEST_NO_EARLY_EXIT = 2
GSS_TEST_SORTED = 4
GSS_NOT_READY = 1  # gss_poll: the test is still running
GSS_TEST_DENSE = 8
GSS_TEST_NO_REGROW = 16
GSS_TEST_NO_HOT = 32
GSS_TEST_GRAPH = 64

GSS_ORDER_STORE = 0
GSS_ORDER_INTERLEAVE = 1
GSS_ORDER_LONGEST_FIRST = 2

REPORT_DTYPE = np.dtype([("clause_id", "<u4"), ("word", "<u4"), ("mask", "<u8")])

_ERR_NAMES = {
    GSS_ERR_INVALID_ARG: "GSS_ERR_INVALID_ARG", GSS_ERR_BAD_LITERAL: "GSS_ERR_BAD_LITERAL",
    GSS_ERR_UNKNOWN_ID: "GSS_ERR_UNKNOWN_ID", GSS_ERR_CAPACITY: "GSS_ERR_CAPACITY",
    GSS_ERR_REPORT_OVERFLOW: "GSS_ERR_REPORT_OVERFLOW", GSS_ERR_DEVICE: "GSS_ERR_DEVICE",
    GSS_ERR_STATE: "GSS_ERR_STATE",
}


class GssError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {message}")
        self.code = code


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class gss_config(ctypes.Structure):
    _fields_ = [
        ("num_vars", ctypes.c_uint32),
        ("max_slots", ctypes.c_uint32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("report_capacity", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
        ("dev_alloc", ALLOC_FN),
        ("dev_free", FREE_FN),
        ("alloc_user", ctypes.c_void_p),
        ("hot_vars", ctypes.c_uint32),
        ("timing_interval", ctypes.c_uint32),
    ]


class gss_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "tests_run", "last_pairs", "last_reports", "last_literals", "live_clauses", "active_slots",
        "device_bytes", "compactions", "regrows", "kernel_launches")] + [
        ("last_kernel_ms", ctypes.c_double), ("total_kernel_ms", ctypes.c_double),
        ("timed_launches", ctypes.c_uint64), ("last_gathers", ctypes.c_uint64),
        ("last_gather_bytes", ctypes.c_uint64), ("last_agg_settled", ctypes.c_uint64)]


class gss_schedule(ctypes.Structure):
    _fields_ = [("order", ctypes.c_uint32), ("chunk_tiles", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class gss_adam_config(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("batch", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 3)]


class gss_priority_config(ctypes.Structure):
    _fields_ = [("n_sources", ctypes.c_uint32), ("sample_period", ctypes.c_uint32),
                ("sample_capacity", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("activity_decay", ctypes.c_double),
                ("reserved", ctypes.c_uint64 * 3)]


MLP_FEATURES = 12
MLP_PARAMS = 5057
GSS_TEST_SCHEDULED = 128
GSS_TEST_AGGREGATE = 256
GSS_TEST_COUNT = 512


class gss_server_config(ctypes.Structure):
    _fields_ = [("n_producers", ctypes.c_uint32), ("test_flags", ctypes.c_uint32),
                ("delete_fraction", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("log_path", ctypes.c_char_p), ("max_queued_lits", ctypes.c_uint64),
                ("evict_keep", ctypes.c_double), ("reserved", ctypes.c_uint64 * 2)]


SERVE_RESULT_COUNTS = ("snapshots", "tested", "dropped", "runs", "overflowed_runs", "inserted", "refused",
                       "deleted", "reports", "pairs", "live_end", "device_bytes_end", "delta_bytes", "evicted",
                       "evictions")
SERVE_RESULT_TIMES = ("wall_s", "gpu_ms", "mean_ms", "p50_ms", "p99_ms", "max_ms", "admit_ms", "wait_ms",
                      "fetch_ms", "route_ms", "store_ms", "launch_ms")


class gss_serve_result(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in SERVE_RESULT_COUNTS] + [(n, ctypes.c_double) for n in SERVE_RESULT_TIMES]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class gss_sim_config(ctypes.Structure):
    _fields_ = [("n_threads", ctypes.c_uint32), ("test_flags", ctypes.c_uint32),
                ("duration_s", ctypes.c_double), ("snapshot_rate", ctypes.c_double),
                ("redraw_fraction", ctypes.c_double), ("insert_rate", ctypes.c_double),
                ("delete_fraction", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("log_path", ctypes.c_char_p), ("evict_keep", ctypes.c_double), ("reserved", ctypes.c_uint64 * 3)]


_lib = None


def load_library(path: Optional[str] = None):
    """Loads libgss.so (or the build named by $GSS_LIBRARY) and declares its
    signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("GSS_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2012_03119_amd.build`")
    lib = ctypes.CDLL(path)
    P, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "gss_create": ([ctypes.POINTER(gss_config), ctypes.POINTER(P)], ctypes.c_int32),
        "gss_destroy": ([P], None),
        "gss_last_error": ([P], ctypes.c_char_p),
        "gss_add_clauses": ([P, P, P, u32, P], ctypes.c_int32),
        "gss_remove_clauses": ([P, P, u32], ctypes.c_int32),
        "gss_store_info": ([P, P, P, P], ctypes.c_int32),
        "gss_set_assignments": ([P, u32, u32, P], ctypes.c_int32),
        "gss_set_var_values": ([P, u32, u32, u32, P, P], ctypes.c_int32),
        "gss_set_var_values_async": ([P, u32, u32, u32, P, P], ctypes.c_int32),
        "gss_clear_slots": ([P, u32, u32], ctypes.c_int32),
        "gss_test": ([P, u32, P], ctypes.c_int32),
        "gss_test_noalloc": ([P, u32, P, u64, P], ctypes.c_int32),
        "gss_rank_vars": ([P, P, P], ctypes.c_int32),
        "gss_fetch_reports": ([P, P, u64, P], ctypes.c_int32),
        "gss_fetch_masks": ([P, P, u32, P], ctypes.c_int32),
        "gss_get_stats": ([P, ctypes.POINTER(gss_stats)], ctypes.c_int32),
        "gss_reset_stats": ([P], ctypes.c_int32),
        "gss_get_stream": ([P, ctypes.POINTER(P)], ctypes.c_int32),
        "gss_update_words": ([P, u32, u32, P, P, P], ctypes.c_int32),
        "gss_update_vars": ([P, u32, u32, P, P, P], ctypes.c_int32),
        "gss_set_active": ([P, P], ctypes.c_int32),
        "gss_test_async": ([P, u32], ctypes.c_int32),
        "gss_test_query": ([P, P], ctypes.c_int32),
        "gss_poll": ([P, P], ctypes.c_int32),
        "gss_test_wait": ([P, P], ctypes.c_int32),
        "gss_batch_create": ([P, u32, ctypes.POINTER(P)], ctypes.c_int32),
        "gss_batch_destroy": ([P], None),
        "gss_batch_last_error": ([P], ctypes.c_char_p),
        "gss_batch_set_schedule": ([P, ctypes.POINTER(gss_schedule)], ctypes.c_int32),
        "gss_batch_test": ([P, u32, P], ctypes.c_int32),
        "gss_batch_test_async": ([P, u32], ctypes.c_int32),
        "gss_batch_wait": ([P, P], ctypes.c_int32),
        "gss_batch_info": ([P, P, P, P, P], ctypes.c_int32),
        "gss_mlp_forward": ([P, P, P, u32, P], ctypes.c_int32),
        "gss_mlp_loss_grad": ([P, P, P, P, u32, P, P], ctypes.c_int32),
        "gss_mlp_train": ([P, P, P, P, u32, P, u64, ctypes.POINTER(gss_adam_config), P], ctypes.c_int32),
        "gss_priority_enable": ([P, ctypes.POINTER(gss_priority_config)], ctypes.c_int32),
        "gss_priority_set_clause_info": ([P, P, u32, P, P], ctypes.c_int32),
        "gss_priority_observe": ([P], ctypes.c_int32),
        "gss_priority_train": ([P, u32, ctypes.POINTER(gss_adam_config), u64, P], ctypes.c_int32),
        "gss_priority_clear_samples": ([P], ctypes.c_int32),
        "gss_priority_score": ([P, ctypes.c_float, P], ctypes.c_int32),
        "gss_priority_params": ([P, P, P], ctypes.c_int32),
        "gss_priority_mark": ([P, P, u64], ctypes.c_int32),
        "gss_priority_update": ([P, P], ctypes.c_int32),
        "gss_priority_set_sampling": ([P, u32], ctypes.c_int32),
        "gss_priority_reduce": ([P, u64, P], ctypes.c_int32),
        "gss_priority_activity": ([P, P, u32, P], ctypes.c_int32),
        "gss_priority_fetch": ([P, P, u32, P, P, P], ctypes.c_int32),
        "gss_priority_samples": ([P, P, P, u64, P], ctypes.c_int32),
        "gss_priority_info": ([P, P, P, P], ctypes.c_int32),
        "gss_server_start": ([P, ctypes.POINTER(gss_server_config), ctypes.POINTER(P)], ctypes.c_int32),
        "gss_server_send": ([P, u32, u32, P, P, P], ctypes.c_int32),
        "gss_server_insert": ([P, u32, P, P, u32], ctypes.c_int32),
        "gss_server_poll": ([P, u32, P, u64, P, P], ctypes.c_int32),
        "gss_server_stop": ([P, ctypes.POINTER(gss_serve_result)], ctypes.c_int32),
        "gss_server_last_error": ([P], ctypes.c_char_p),
        "gss_serve_simulate": ([P, ctypes.POINTER(gss_sim_config), ctypes.POINTER(gss_serve_result)], ctypes.c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(ctx, rc: int):
    if rc != GSS_OK:
        msg = load_library().gss_last_error(ctx)
        raise GssError(rc, msg.decode() if msg else "")


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _data_ptr(x, dtype):
    """(pointer, keep-alive, n_elements) for a numpy array or a torch tensor
    (host or device), converted to the dtype if needed."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            tdt = {np.int8: torch.int8, np.uint32: torch.int32, np.int32: torch.int32}[dtype]
            t = x.contiguous()
            if t.dtype != tdt:
                t = t.to(tdt)
            return ctypes.c_void_p(t.data_ptr()), t, t.numel()
    except ImportError:  # pragma: no cover
        pass
    a = np.ascontiguousarray(x, dtype=dtype)
    return _np_ptr(a), a, a.size


# ---------------------------------------------------------------------------
# ABI-named functions
# ---------------------------------------------------------------------------

def gss_create(cfg: gss_config):
    lib = load_library()
    ctx = ctypes.c_void_p()
    rc = lib.gss_create(ctypes.byref(cfg), ctypes.byref(ctx))
    if rc != GSS_OK:
        msg = lib.gss_last_error(None)
        raise GssError(rc, msg.decode() if msg else "")
    return ctx


def gss_destroy(ctx) -> None:
    load_library().gss_destroy(ctx)


def gss_add_clauses(ctx, lits, offsets) -> np.ndarray:
    lits = np.ascontiguousarray(lits, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(offsets) - 1
    ids = np.empty(max(n, 0), dtype=np.uint32)
    if n <= 0:
        return ids
    _check(ctx, load_library().gss_add_clauses(ctx, _np_ptr(lits), _np_ptr(offsets), n, _np_ptr(ids)))
    return ids


def gss_remove_clauses(ctx, ids) -> None:
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    _check(ctx, load_library().gss_remove_clauses(ctx, _np_ptr(ids), len(ids)))


def gss_store_info(ctx):
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, load_library().gss_store_info(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return dict(live_clauses=a.value, next_id=b.value, device_bytes=c.value)


def gss_set_assignments(ctx, first_slot: int, values) -> None:
    """values: int8 [n_slots][num_vars], numpy or torch (host or device)."""
    n_slots = int(values.shape[0]) if len(values.shape) == 2 else 0
    ptr, keep, _ = _data_ptr(values, np.int8)
    _check(ctx, load_library().gss_set_assignments(ctx, first_slot, n_slots, ptr))
    del keep


def gss_set_var_values(ctx, first_slot: int, vars_, values) -> None:
    """vars_: distinct variables (host); values: int8 [len(vars_)][n_slots] (host or device)."""
    vars_ = np.ascontiguousarray(vars_, dtype=np.uint32)
    n_slots = int(values.shape[1])
    ptr, keep, _ = _data_ptr(values, np.int8)
    _check(ctx, load_library().gss_set_var_values(ctx, first_slot, n_slots, len(vars_), _np_ptr(vars_), ptr))
    del keep


def gss_set_var_values_async(ctx, first_slot: int, vars_, values) -> None:
    """Queued form of gss_set_var_values: values must be device memory that stays
    unchanged until the next gss_test / gss_test_wait returns (the caller keeps it
    alive); a failed device-side check is reported by that call."""
    vars_ = np.ascontiguousarray(vars_, dtype=np.uint32)
    n_slots = int(values.shape[1])
    ptr, keep, _ = _data_ptr(values, np.int8)
    _check(ctx, load_library().gss_set_var_values_async(ctx, first_slot, n_slots, len(vars_), _np_ptr(vars_), ptr))
    del keep


def gss_update_words(ctx, word: int, vars_, f_words, t_words) -> None:
    """Packed delta of one 64-slot word: f/t words per listed variable."""
    vars_ = np.ascontiguousarray(vars_, dtype=np.uint32)
    f = np.ascontiguousarray(f_words, dtype=np.uint64)
    t = np.ascontiguousarray(t_words, dtype=np.uint64)
    if not (len(vars_) == len(f) == len(t)):
        raise ValueError("vars, f_words and t_words differ in length")
    _check(ctx, load_library().gss_update_words(ctx, word, len(vars_), _np_ptr(vars_), _np_ptr(f), _np_ptr(t)))


def gss_set_active(ctx, active) -> None:
    a = np.ascontiguousarray(active, dtype=np.uint64)
    _check(ctx, load_library().gss_set_active(ctx, _np_ptr(a)))


def gss_test_async(ctx, flags: int = 0) -> None:
    _check(ctx, load_library().gss_test_async(ctx, flags))


def gss_poll(ctx) -> Optional[int]:
    """None while the test in flight runs; once it has completed, its record count
    (the test is then complete, as after gss_test_wait)."""
    n = ctypes.c_uint64()
    rc = load_library().gss_poll(ctx, ctypes.byref(n))
    if rc == GSS_NOT_READY:
        return None
    _check(ctx, rc)
    return n.value


def gss_test_query(ctx) -> bool:
    d = ctypes.c_int()
    _check(ctx, load_library().gss_test_query(ctx, ctypes.byref(d)))
    return bool(d.value)


def gss_test_wait(ctx) -> int:
    n = ctypes.c_uint64()
    _check(ctx, load_library().gss_test_wait(ctx, ctypes.byref(n)))
    return n.value


def gss_clear_slots(ctx, first_slot: int, n_slots: int) -> None:
    _check(ctx, load_library().gss_clear_slots(ctx, first_slot, n_slots))


def gss_test(ctx, flags: int = 0) -> int:
    n = ctypes.c_uint64()
    _check(ctx, load_library().gss_test(ctx, flags, ctypes.byref(n)))
    return n.value


def gss_rank_vars(ctx):
    """Ranks the variables for LDS staging now; returns (literal occurrences on
    the staged variables, literals stored) at that ranking."""
    hot, lits = ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, load_library().gss_rank_vars(ctx, ctypes.byref(hot), ctypes.byref(lits)))
    return hot.value, lits.value


def gss_test_noalloc(ctx, flags: int, ptr: int, cap: int) -> int:
    """The test with its records stitched into device memory at address ptr
    (room for cap 16-byte records); returns the exact number of records."""
    n = ctypes.c_uint64()
    _check(ctx, load_library().gss_test_noalloc(ctx, flags, ctypes.c_void_p(ptr) if cap else None, cap,
                                                ctypes.byref(n)))
    return n.value


def gss_fetch_reports(ctx, cap: int) -> np.ndarray:
    out = np.empty(cap, dtype=REPORT_DTYPE)
    n = ctypes.c_uint64()
    _check(ctx, load_library().gss_fetch_reports(ctx, _np_ptr(out) if cap else None, cap, ctypes.byref(n)))
    return out[:n.value]


def gss_fetch_reports_into(ctx, ptr: int, cap: int) -> int:
    """Copies up to cap records into memory at address ptr (device or host, room
    for cap 16-byte records); returns how many were copied."""
    n = ctypes.c_uint64()
    _check(ctx, load_library().gss_fetch_reports(ctx, ctypes.c_void_p(ptr), cap, ctypes.byref(n)))
    return n.value


def gss_fetch_masks(ctx, ids, n_words: int) -> np.ndarray:
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.zeros((len(ids), n_words), dtype=np.uint64)
    if len(ids):
        _check(ctx, load_library().gss_fetch_masks(ctx, _np_ptr(ids), len(ids), _np_ptr(out)))
    return out


def gss_get_stats(ctx) -> dict:
    s = gss_stats()
    _check(ctx, load_library().gss_get_stats(ctx, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in gss_stats._fields_}


def gss_reset_stats(ctx) -> None:
    _check(ctx, load_library().gss_reset_stats(ctx))


def gss_get_stream(ctx) -> int:
    p = ctypes.c_void_p()
    _check(ctx, load_library().gss_get_stream(ctx, ctypes.byref(p)))
    return p.value or 0


def gss_batch_create(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    b = ctypes.c_void_p()
    rc = load_library().gss_batch_create(arr, len(ctxs), ctypes.byref(b))
    if rc != GSS_OK:
        raise GssError(rc, "gss_batch_create failed")
    return b


def gss_batch_destroy(b) -> None:
    load_library().gss_batch_destroy(b)


def _check_batch(b, rc: int):
    if rc != GSS_OK:
        msg = load_library().gss_batch_last_error(b)
        raise GssError(rc, msg.decode() if msg else "")


def gss_batch_set_schedule(b, order: int, chunk_tiles: int = 0, blocks_per_cu: int = 0) -> None:
    s = gss_schedule(order, chunk_tiles, blocks_per_cu, 0)
    _check_batch(b, load_library().gss_batch_set_schedule(b, ctypes.byref(s)))


def gss_batch_test(b, n: int, flags: int = 0) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    _check_batch(b, load_library().gss_batch_test(b, flags, _np_ptr(out)))
    return out


def gss_batch_test_async(b, flags: int = 0) -> None:
    _check_batch(b, load_library().gss_batch_test_async(b, flags))


def gss_batch_wait(b, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    _check_batch(b, load_library().gss_batch_wait(b, _np_ptr(out)))
    return out


def gss_batch_info(b) -> dict:
    ms, la, ca, ti = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check_batch(b, load_library().gss_batch_info(b, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(ca),
                                                 ctypes.byref(ti)))
    return dict(last_ms=ms.value, launches=la.value, captures=ca.value, tiles=ti.value)


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def gss_mlp_forward(ctx, params, x) -> np.ndarray:
    p = _f32(params, (MLP_PARAMS,))
    x = _f32(x)
    n = x.shape[0]
    if x.shape != (n, MLP_FEATURES):
        raise ValueError("x must be [n][12]")
    out = np.zeros(n, dtype=np.float32)
    _check(ctx, load_library().gss_mlp_forward(ctx, _np_ptr(p), _np_ptr(x), n, _np_ptr(out)))
    return out


def gss_mlp_loss_grad(ctx, params, x, y):
    p = _f32(params, (MLP_PARAMS,))
    x, y = _f32(x), _f32(y)
    n = x.shape[0]
    if x.shape != (n, MLP_FEATURES) or y.shape != (n,):
        raise ValueError("x must be [n][12] and y [n]")
    loss = ctypes.c_float()
    g = np.zeros(MLP_PARAMS, dtype=np.float32)
    _check(ctx, load_library().gss_mlp_loss_grad(ctx, _np_ptr(p), _np_ptr(x), _np_ptr(y), n, ctypes.byref(loss),
                                                 _np_ptr(g)))
    return loss.value, g


def _adam(lr, beta1, beta2, eps, batch):
    return gss_adam_config(lr, beta1, beta2, eps, batch)


def gss_mlp_train(ctx, params, x, y, order, *, batch: int, lr: float = 1e-3, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-8):
    """(trained parameters, per-step losses)."""
    p = _f32(params, (MLP_PARAMS,)).copy()
    x, y = _f32(x), _f32(y)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    cfg = _adam(lr, beta1, beta2, eps, batch)
    steps = (order.size + batch - 1) // batch
    losses = np.zeros(max(steps, 1), dtype=np.float32)
    _check(ctx, load_library().gss_mlp_train(ctx, _np_ptr(p), _np_ptr(x), _np_ptr(y), x.shape[0], _np_ptr(order),
                                             order.size, ctypes.byref(cfg), _np_ptr(losses)))
    return p, losses[:steps]


def gss_server_start(ctx, n_producers: int, *, test_flags: int = 0, delete_fraction: float = 0.0, seed: int = 0,
                     log_path: Optional[str] = None, max_queued_lits: int = 0, evict_keep: float = 0.0):
    cfg = gss_server_config(n_producers, test_flags, delete_fraction, seed,
                            log_path.encode() if log_path else None, max_queued_lits, evict_keep)
    srv = ctypes.c_void_p()
    _check(ctx, load_library().gss_server_start(ctx, ctypes.byref(cfg), ctypes.byref(srv)))
    return srv


def _check_server(srv, rc: int):
    if rc != GSS_OK:
        msg = load_library().gss_server_last_error(srv)
        raise GssError(rc, msg.decode() if msg else "")


def gss_server_send(srv, producer: int, vars_, f_words, t_words) -> None:
    v = np.ascontiguousarray(vars_, dtype=np.uint32)
    f = np.ascontiguousarray(f_words, dtype=np.uint64)
    t = np.ascontiguousarray(t_words, dtype=np.uint64)
    if not (v.size == f.size == t.size):
        raise ValueError("vars, f_words and t_words differ in length")
    _check_server(srv, load_library().gss_server_send(srv, producer, v.size, _np_ptr(v), _np_ptr(f), _np_ptr(t)))


def gss_server_insert(srv, producer: int, lits, offsets) -> None:
    lits = np.ascontiguousarray(lits, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    _check_server(srv, load_library().gss_server_insert(srv, producer, _np_ptr(lits), _np_ptr(offsets),
                                                        offsets.size - 1))


def gss_server_poll(srv, producer: int, cap: int = 1 << 20):
    """(records, last run routed to the producer or None)."""
    out = np.zeros(max(cap, 1), dtype=REPORT_DTYPE)
    n, run = ctypes.c_uint64(), ctypes.c_uint64()
    _check_server(srv, load_library().gss_server_poll(srv, producer, _np_ptr(out), cap, ctypes.byref(n),
                                                      ctypes.byref(run)))
    return out[:n.value].copy(), (None if run.value == 2**64 - 1 else run.value)


def gss_server_stop(ctx, srv) -> dict:
    r = gss_serve_result()
    _check(ctx, load_library().gss_server_stop(srv, ctypes.byref(r)))
    return r.as_dict()


def gss_serve_simulate(ctx, *, n_threads: int, duration_s: float, snapshot_rate: float, redraw_fraction: float,
                       insert_rate: float, delete_fraction: float, seed: int, test_flags: int = 0,
                       log_path: Optional[str] = None, evict_keep: float = 0.0) -> dict:
    cfg = gss_sim_config(n_threads, test_flags, duration_s, snapshot_rate, redraw_fraction, insert_rate,
                         delete_fraction, seed, log_path.encode() if log_path else None, evict_keep)
    r = gss_serve_result()
    _check(ctx, load_library().gss_serve_simulate(ctx, ctypes.byref(cfg), ctypes.byref(r)))
    return r.as_dict()


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

class Context:
    """One clause store plus one set of assignment slots on the current GPU."""

    def __init__(self, num_vars: int, max_slots: int = 64, *, hbm_budget_bytes: int = 0,
                 report_capacity: int = 1 << 16, hot_vars: int = 0, use_torch: bool = True, stream=None,
                 timing_interval: int = 0):
        self.num_vars = int(num_vars)
        self.max_slots = int(max_slots)
        self.n_words = self.max_slots // 64
        self._keep = []
        cfg = gss_config()
        cfg.num_vars = self.num_vars
        cfg.max_slots = self.max_slots
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.report_capacity = report_capacity
        cfg.hot_vars = hot_vars
        cfg.timing_interval = timing_interval
        self.torch_stream = None
        self._held, self._held_by_test = [], []  # device inputs of queued updates, kept alive
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible to torch")
            dev = torch.cuda.current_device()
            # a shared stream (batches need one) or a stream of its own; default priority
            self.torch_stream = stream if stream is not None else torch.cuda.Stream(device=dev)
            cfg.stream = self.torch_stream.cuda_stream

            def _alloc(size, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(size, dev, stream)
                except Exception:
                    return None

            def _free(ptr, stream, user):
                torch.cuda.caching_allocator_delete(ptr)

            cfg.dev_alloc = ALLOC_FN(_alloc)
            cfg.dev_free = FREE_FN(_free)
            self._keep += [cfg.dev_alloc, cfg.dev_free]
        self._cfg = cfg
        self.ctx = gss_create(cfg)

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            gss_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _sync_inputs(self, *xs):
        # device inputs produced on torch's current stream must be ready for ours
        if self.torch_stream is None:
            return
        import torch
        if any(isinstance(x, torch.Tensor) and x.is_cuda for x in xs):
            cur = torch.cuda.current_stream()
            if cur != self.torch_stream:  # on the same stream the order already holds
                self.torch_stream.wait_stream(cur)

    # -- ABI calls
    def add_clauses(self, lits, offsets) -> np.ndarray:
        return gss_add_clauses(self.ctx, lits, offsets)

    def remove_clauses(self, ids) -> None:
        gss_remove_clauses(self.ctx, ids)

    def store_info(self) -> dict:
        return gss_store_info(self.ctx)

    def set_assignments(self, first_slot: int, values) -> None:
        self._sync_inputs(values)
        gss_set_assignments(self.ctx, first_slot, values)

    def set_var_values(self, first_slot: int, vars_, values) -> None:
        self._sync_inputs(values)
        gss_set_var_values(self.ctx, first_slot, vars_, values)

    def set_var_values_async(self, first_slot: int, vars_, values) -> None:
        """values (a device tensor) is held until the next test has completed."""
        self._sync_inputs(values)
        gss_set_var_values_async(self.ctx, first_slot, vars_, values)
        self._held.append(values)  # until the next test begun after this call completes

    def clear_slots(self, first_slot: int, n_slots: int) -> None:
        gss_clear_slots(self.ctx, first_slot, n_slots)

    def update_words(self, word: int, vars_, f_words, t_words) -> None:
        gss_update_words(self.ctx, word, vars_, f_words, t_words)

    def set_active(self, active) -> None:
        gss_set_active(self.ctx, active)

    def test_async(self, flags: int = 0) -> None:
        gss_test_async(self.ctx, flags)
        self._held_by_test, self._held = self._held, []

    def poll(self) -> Optional[int]:
        try:
            n = gss_poll(self.ctx)
        except GssError:
            self._held_by_test = []  # the test completed with an error
            raise
        if n is not None:
            self._held_by_test = []
        return n

    def test_query(self) -> bool:
        return gss_test_query(self.ctx)

    def test_wait(self) -> int:
        try:
            return gss_test_wait(self.ctx)
        finally:
            self._held_by_test = []

    def test(self, flags: int = 0) -> int:
        n = gss_test(self.ctx, flags)  # on an error the queued inputs stay held (harmless if applied)
        self._held = []
        return n

    def rank_vars(self):
        return gss_rank_vars(self.ctx)

    def test_noalloc(self, flags: int, out) -> int:
        """gss_test_noalloc into `out`, a contiguous CUDA tensor whose bytes hold
        len(out bytes) // 16 records; returns the exact number of records."""
        if not (out.is_cuda and out.is_contiguous()):
            raise ValueError("out must be a contiguous CUDA tensor")
        cap = out.numel() * out.element_size() // 16
        n = gss_test_noalloc(self.ctx, flags, out.data_ptr(), cap)
        self._held = []
        return n

    def fetch_reports(self, cap: Optional[int] = None) -> np.ndarray:
        if cap is None:
            cap = self.stats()["last_reports"]
        return gss_fetch_reports(self.ctx, int(cap))

    def fetch_masks(self, ids) -> np.ndarray:
        return gss_fetch_masks(self.ctx, ids, self.n_words)

    def stats(self) -> dict:
        return gss_get_stats(self.ctx)

    def reset_stats(self) -> None:
        gss_reset_stats(self.ctx)

    @property
    def stream(self) -> int:
        return gss_get_stream(self.ctx)

    # -- learned priority
    def priority_enable(self, *, n_sources: int = 1, sample_period: int = 0, sample_capacity: int = 0,
                        seed: int = 0, activity_decay: float = 0.0) -> None:
        cfg = gss_priority_config(n_sources, sample_period, sample_capacity, seed, activity_decay)
        _check(self.ctx, load_library().gss_priority_enable(self.ctx, ctypes.byref(cfg)))

    def priority_set_clause_info(self, ids, lbd, source) -> None:
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        lbd = _f32(lbd, ids.shape)
        source = np.ascontiguousarray(source, dtype=np.uint32)
        _check(self.ctx, load_library().gss_priority_set_clause_info(self.ctx, _np_ptr(ids), ids.size, _np_ptr(lbd),
                                                                     _np_ptr(source)))

    def priority_observe(self) -> None:
        _check(self.ctx, load_library().gss_priority_observe(self.ctx))

    def priority_train(self, epochs: int, *, batch: int = 1024, lr: float = 1e-3, beta1: float = 0.9,
                       beta2: float = 0.999, eps: float = 1e-8, seed: int = 0) -> float:
        cfg = _adam(lr, beta1, beta2, eps, batch)
        loss = ctypes.c_float()
        _check(self.ctx, load_library().gss_priority_train(self.ctx, epochs, ctypes.byref(cfg), seed,
                                                           ctypes.byref(loss)))
        return loss.value

    def priority_set_sampling(self, period: int) -> None:
        _check(self.ctx, load_library().gss_priority_set_sampling(self.ctx, period))

    def priority_clear_samples(self) -> None:
        _check(self.ctx, load_library().gss_priority_clear_samples(self.ctx))

    def priority_score(self, threshold: float) -> int:
        n = ctypes.c_uint64()
        _check(self.ctx, load_library().gss_priority_score(self.ctx, ctypes.c_float(threshold), ctypes.byref(n)))
        return n.value

    def priority_update(self) -> int:
        n = ctypes.c_uint64()
        _check(self.ctx, load_library().gss_priority_update(self.ctx, ctypes.byref(n)))
        return n.value

    def priority_reduce(self, keep: int) -> int:
        n = ctypes.c_uint64()
        _check(self.ctx, load_library().gss_priority_reduce(self.ctx, keep, ctypes.byref(n)))
        return n.value

    def priority_activity(self, ids) -> np.ndarray:
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        out = np.zeros(ids.size, dtype=np.float32)
        _check(self.ctx, load_library().gss_priority_activity(self.ctx, _np_ptr(ids), ids.size, _np_ptr(out)))
        return out

    def priority_mark(self, low) -> None:
        low = np.ascontiguousarray(low, dtype=np.uint8)
        _check(self.ctx, load_library().gss_priority_mark(self.ctx, _np_ptr(low), low.size))

    def priority_params(self, set_to=None) -> np.ndarray:
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        src = _f32(set_to, (MLP_PARAMS,)) if set_to is not None else None
        _check(self.ctx, load_library().gss_priority_params(self.ctx, _np_ptr(out),
                                                            _np_ptr(src) if src is not None else None))
        return out

    def priority_fetch(self, ids):
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        x = np.zeros((ids.size, MLP_FEATURES), dtype=np.float32)
        sc = np.zeros(ids.size, dtype=np.float32)
        low = np.zeros(ids.size, dtype=np.uint8)
        _check(self.ctx, load_library().gss_priority_fetch(self.ctx, _np_ptr(ids), ids.size, _np_ptr(x), _np_ptr(sc),
                                                           _np_ptr(low)))
        return x, sc, low.astype(bool)

    def priority_samples(self, cap: int):
        x = np.zeros((max(cap, 1), MLP_FEATURES), dtype=np.float32)
        y = np.zeros(max(cap, 1), dtype=np.float32)
        n = ctypes.c_uint64()
        _check(self.ctx, load_library().gss_priority_samples(self.ctx, _np_ptr(x), _np_ptr(y), cap, ctypes.byref(n)))
        return x[:n.value], y[:n.value]

    def priority_info(self) -> dict:
        r, s_, lo = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.ctx, load_library().gss_priority_info(self.ctx, ctypes.byref(r), ctypes.byref(s_),
                                                          ctypes.byref(lo)))
        return dict(run=r.value, samples=s_.value, n_low=lo.value)

    def serve_simulate(self, **kw) -> dict:
        """Runs the served workload generator on this context (gss_serve_simulate)."""
        return gss_serve_simulate(self.ctx, **kw)


class Server:
    """A manager thread serving producers on one context (gss_server_*).  The
    context must not be used directly until stop()."""

    def __init__(self, context: "Context", n_producers: int, **kw):
        self.context = context
        self.srv = gss_server_start(context.ctx, n_producers, **kw)

    def send(self, producer: int, vars_, f_words, t_words) -> None:
        gss_server_send(self.srv, producer, vars_, f_words, t_words)

    def insert(self, producer: int, lits, offsets) -> None:
        gss_server_insert(self.srv, producer, lits, offsets)

    def poll(self, producer: int, cap: int = 1 << 20):
        return gss_server_poll(self.srv, producer, cap)

    def stop(self) -> dict:
        srv, self.srv = self.srv, None
        return gss_server_stop(self.context.ctx, srv)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        if self.srv is not None:
            self.stop()


def sort_reports(r: np.ndarray) -> np.ndarray:
    """Orders records by (clause_id, word), the canonical order for comparisons."""
    return np.sort(r, order=["clause_id", "word"])


class Batch:
    """Several contexts (sharing one stream) tested in one persistent launch."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        self.b = gss_batch_create([c.ctx for c in self.contexts])

    def set_schedule(self, order: int, chunk_tiles: int = 0, blocks_per_cu: int = 0) -> None:
        gss_batch_set_schedule(self.b, order, chunk_tiles, blocks_per_cu)

    def test(self, flags: int = 0) -> np.ndarray:
        counts = gss_batch_test(self.b, len(self.contexts), flags)
        for c in self.contexts:  # their queued updates have been read
            c._held = []
        return counts

    def test_async(self, flags: int = 0) -> None:
        """Queues the batched test; updates queued on the members afterwards stay
        held until the next test."""
        gss_batch_test_async(self.b, flags)
        for c in self.contexts:
            c._held_by_test, c._held = c._held, []

    def wait(self) -> np.ndarray:
        try:
            return gss_batch_wait(self.b, len(self.contexts))
        finally:
            for c in self.contexts:
                c._held_by_test = []

    def info(self) -> dict:
        return gss_batch_info(self.b)

    def close(self):
        if getattr(self, "b", None):
            gss_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
