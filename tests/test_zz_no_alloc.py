"""GPU tests of gss_test_noalloc, the test whose report segments live in the
library's per-GPU scratch array: its records equal those of gss_test followed by
gss_fetch_reports on the same context, on two calls in a row (the second on a
smaller input, so stale scratch contents would show), and its errors."""
import numpy as np
import pytest

import oracle
from gpu_helpers import reports_to_dense
from paper_2012_03119_amd import gen, gss

pytestmark = pytest.mark.gpu


def _records(buf, n):
    return buf[:n].cpu().numpy().view(gss.REPORT_DTYPE).reshape(-1)


def _sorted(r):
    return np.sort(r, order=["clause_id", "word"])


def _both(ctx, flags, cap):
    """(records of gss_test + gss_fetch_reports, records of gss_test_noalloc)."""
    import torch
    n_ref = ctx.test(flags)
    ref = ctx.fetch_reports(n_ref)
    buf = torch.full((cap, 2), -1, dtype=torch.int64, device="cuda")
    print(f"noalloc flags={flags} cap={cap}", flush=True)
    n = ctx.test_noalloc(flags, buf)
    assert n == n_ref
    return ref, _records(buf, n)


@pytest.mark.parametrize("flags", [0, gss.GSS_TEST_TRIGGER, gss.GSS_TEST_NO_EARLY_EXIT | gss.GSS_TEST_NO_HOT])
def test_noalloc_equals_test_then_fetch_twice(flags):
    mode = "trigger" if flags & gss.GSS_TEST_TRIGGER else "falsified"
    # first call: the tiny workload, 64 slots
    w = gen.tiny(1)
    with gss.Context(w.n_vars, 64, hot_vars=50) as ctx:
        ctx.add_clauses(w.lits, w.offsets)
        ctx.set_assignments(0, w.values)
        ref, got = _both(ctx, flags, 1 << 18)
        assert len(got) > 5000
        assert np.array_equal(_sorted(got), _sorted(ref))
        want = oracle.masks(w.lits, w.offsets, w.values, mode=mode)
        assert np.array_equal(reports_to_dense(got, w.n_clauses, 1), want)
    # second call, on another context: a smaller store with 1024 slots and fewer records
    w2 = gen.tiny(7, n_clauses=3000, n_vars=300, n_slots=1024, assigned=0.5)
    with gss.Context(w2.n_vars, 1024) as ctx:
        ctx.add_clauses(w2.lits, w2.offsets)
        ctx.set_assignments(0, w2.values)
        ref, got = _both(ctx, flags, 1 << 16)
        assert len(got) > 0
        assert np.array_equal(_sorted(got), _sorted(ref))
        want = oracle.masks(w2.lits, w2.offsets, w2.values, mode=mode)
        assert np.array_equal(reports_to_dense(got, w2.n_clauses, 16), want)


def test_noalloc_aggregate_and_wide_rows():
    w = gen.tiny(3, n_clauses=4000, n_vars=200, n_slots=8192, assigned=0.7)
    with gss.Context(w.n_vars, 8192) as ctx:
        ctx.add_clauses(w.lits, w.offsets)
        ctx.set_assignments(0, w.values)
        for flags in (gss.GSS_TEST_AGGREGATE, 0):
            ref, got = _both(ctx, flags, 1 << 18)
            assert np.array_equal(_sorted(got), _sorted(ref))
        # the trigger form of the pre-test needs bits a gss_test allocates first
        import torch
        buf = torch.zeros((16, 2), dtype=torch.int64, device="cuda")
        flags = gss.GSS_TEST_AGGREGATE | gss.GSS_TEST_TRIGGER
        with pytest.raises(gss.GssError) as e:
            ctx.test_noalloc(flags, buf)
        assert e.value.code == gss.GSS_ERR_STATE
        ref, got = _both(ctx, flags, 1 << 20)
        assert np.array_equal(_sorted(got), _sorted(ref))
        want = oracle.masks(w.lits, w.offsets, w.values, mode="trigger")
        assert np.array_equal(reports_to_dense(got, w.n_clauses, 128), want)


def test_noalloc_errors_and_short_output():
    import torch
    w = gen.tiny(2, n_clauses=5000, n_vars=500)
    with gss.Context(w.n_vars, 64) as ctx:
        ctx.add_clauses(w.lits, w.offsets)
        ctx.set_assignments(0, w.values)
        n_ref = ctx.test()
        ref = ctx.fetch_reports(n_ref)
        buf = torch.zeros((64, 2), dtype=torch.int64, device="cuda")
        for bad in (gss.GSS_TEST_SORTED, gss.GSS_TEST_DENSE, gss.GSS_TEST_SCHEDULED, 1 << 20):
            with pytest.raises(gss.GssError) as e:
                ctx.test_noalloc(bad, buf)
            assert e.value.code == gss.GSS_ERR_INVALID_ARG
        # host memory is refused
        lib = gss.load_library()
        host = np.zeros(64, dtype=gss.REPORT_DTYPE)
        import ctypes
        n = ctypes.c_uint64()
        rc = lib.gss_test_noalloc(ctx.ctx, 0, host.ctypes.data_as(ctypes.c_void_p), 64, ctypes.byref(n))
        assert rc == gss.GSS_ERR_INVALID_ARG
        # the records before the failed calls are still fetchable
        assert np.array_equal(ctx.fetch_reports(n_ref), ref)
        # fewer places than records: the exact count, and cap records of the full set
        rc = lib.gss_test_noalloc(ctx.ctx, 0, ctypes.c_void_p(buf.data_ptr()), 64, ctypes.byref(n))
        assert rc == gss.GSS_ERR_REPORT_OVERFLOW
        assert n.value == n_ref
        part = _records(buf, 64)
        key = lambda r: set(zip(r["clause_id"].tolist(), r["word"].tolist(), r["mask"].tolist()))
        assert key(part) <= key(ref) and len(key(part)) == 64
        # the context's records are no longer the last test's
        with pytest.raises(gss.GssError) as e:
            ctx.fetch_reports(n_ref)
        assert e.value.code == gss.GSS_ERR_STATE
    # an empty store: no records, no launch
    with gss.Context(10, 64) as ctx:
        assert ctx.test_noalloc(0, torch.zeros((1, 2), dtype=torch.int64, device="cuda")) == 0
