// Host side of the single-store clause test: launch shape, the entry points
// gss_test, gss_test_async / query / wait, gss_fetch_reports and gss_fetch_masks.
// The kernels are in test_kernels.h.
#include "test_kernels.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>

namespace gss {


using KernelFn = void (*)(const BucketDesc *, const TestArgs, uint32_t, uint32_t);

// row words RW (power of two) -> lanes per clause and words per lane (a lane
// takes one 32-byte sector: 4 words, or the whole row when it is shorter)
template <int MODE, bool HOT, bool AGG>
static KernelFn pick_rw(uint32_t rw) {
    switch (rw) {
    case 1: return k_test<1, 1, MODE, HOT, AGG>;
    case 2: return k_test<1, 2, MODE, HOT, AGG>;
    case 4: return k_test<1, 4, MODE, HOT, AGG>;
    case 8: return k_test<2, 4, MODE, HOT, AGG>;
    case 16: return k_test<4, 4, MODE, HOT, AGG>;
    case 32: return k_test<8, 4, MODE, HOT, AGG>;
    default: return k_test<16, 4, MODE, HOT, AGG>;
    }
}

template <bool AGG>
static KernelFn pick_mode(uint32_t rw, int mode, bool hot) {
    if (mode == 0) return hot ? pick_rw<0, true, AGG>(rw) : pick_rw<0, false, AGG>(rw);
    return hot ? pick_rw<1, true, AGG>(rw) : pick_rw<1, false, AGG>(rw);
}

// the scheduled test's kernel, which walks the list of the slots a run tests
template <int MODE, bool HOT, bool AGG>
static KernelFn pick_rw_list(uint32_t rw) {
    switch (rw) {
    case 1: return k_test_list<1, 1, MODE, HOT, AGG>;
    case 2: return k_test_list<1, 2, MODE, HOT, AGG>;
    case 4: return k_test_list<1, 4, MODE, HOT, AGG>;
    case 8: return k_test_list<2, 4, MODE, HOT, AGG>;
    case 16: return k_test_list<4, 4, MODE, HOT, AGG>;
    case 32: return k_test_list<8, 4, MODE, HOT, AGG>;
    default: return k_test_list<16, 4, MODE, HOT, AGG>;
    }
}

template <bool AGG>
static KernelFn pick_mode_list(uint32_t rw, int mode, bool hot) {
    if (mode == 0) return hot ? pick_rw_list<0, true, AGG>(rw) : pick_rw_list<0, false, AGG>(rw);
    return hot ? pick_rw_list<1, true, AGG>(rw) : pick_rw_list<1, false, AGG>(rw);
}

// rw: words of a row in one chunk; wide: more than one chunk (no LDS staging then);
// listed: a scheduled test that walks the list of the slots it tests
static KernelFn pick_kernel(uint32_t rw, int mode, bool hot, bool agg, bool wide, bool listed = false) {
    if (listed) return agg ? pick_mode_list<true>(rw, mode, hot) : pick_mode_list<false>(rw, mode, hot);
    if (wide) {
        if (mode == 0) return agg ? k_test<16, 4, 0, false, true, true> : k_test<16, 4, 0, false, false, true>;
        return agg ? k_test<16, 4, 1, false, true, true> : k_test<16, 4, 1, false, false, true>;
    }
    return agg ? pick_mode<true>(rw, mode, hot) : pick_mode<false>(rw, mode, hot);
}

struct Launch {
    TestArgs args{};
    const BucketDesc *descs = nullptr;
    KernelFn fn = nullptr;
    unsigned grid = 0;
    size_t lds = 0;
};

// Builds the descriptors of the non-empty length classes, uploads them and picks
// the launch shape.
static Launch prepare(Ctx &c, uint32_t flags) {
    Launch L;
    TestArgs &a = L.args;
    BucketDesc *h = (BucketDesc *)c.hsmall_desc;
    uint32_t nb = 0, tiles = 0;
    const bool sched = (flags & GSS_TEST_SCHEDULED) != 0;
    a.sched_run = sched ? priority_schedule(c) : 0u;
    // a scheduled test lists the slots it tests (on the device, behind the
    // schedule bits) so that the clauses sitting out the run take no lanes
    const bool listed = sched && c.G == 1;
    uint64_t list_off = 0;
    if (listed) {
        uint64_t slots = 0;
        for (const Bucket &B : c.buckets) slots += B.n_slots;
        if (slots > c.sched_list_cap) {
            const uint64_t want = std::max<uint64_t>(slots, c.sched_list_cap + c.sched_list_cap / 2);
            uint32_t *p = (uint32_t *)c.dalloc(want * 4);
            c.defer_free(c.sched_list);  // a test queued before may still read it
            c.sched_list = p;
            c.sched_list_cap = want;
        }
        if (!c.sched_counts) c.sched_counts = (uint32_t *)c.dalloc(kMaxBuckets * 4);
        launch_fill_u32(c, c.sched_counts, kMaxBuckets, 0);
    }
    SchedTable st{};
    uint32_t sched_blocks = 0;
    for (int b = 0; b < kMaxBuckets; ++b) {
        const Bucket &B = c.buckets[b];
        if (B.n_slots == 0 || B.n_dead == B.n_slots) continue;
        BucketDesc d{};
        d.lits = B.lits;
        d.meta = B.meta;
        d.lits_bytes = B.cap_slots << B.stride_log2 << 2;
        d.meta_bytes = B.cap_slots * 8;
        d.stride_log2 = B.stride_log2;
        d.tile_begin = tiles;
        if (sched) {
            d.low = B.low;
            d.low_bytes = B.low_words * 4;
        }
        if (listed) {
            d.list = c.sched_list + list_off;
            d.list_count = c.sched_counts + nb;
            st.cls[st.n++] = SchedClass{B.meta, B.low, c.sched_list + list_off, c.sched_counts + nb, (uint32_t)B.n_slots,
                                        sched_blocks};
            sched_blocks += (uint32_t)((B.n_slots + kSchedSlots - 1) / kSchedSlots);
            list_off += B.n_slots;
        }
        h[nb++] = d;
        tiles += (uint32_t)((B.n_slots + c.T - 1) / c.T);
    }
    if (listed && sched_blocks) {  // every class's list in one launch
        hipLaunchKernelGGL(k_sched_list, dim3(sched_blocks), dim3(kSchedThreads), 0, c.stream, st, a.sched_run);
        GSS_HIP(hipGetLastError());
    }
    a.n_buckets = nb;
    a.n_tiles = tiles;
    a.planes = c.planes;
    a.active = c.active;
    a.W = c.W;
    a.G = c.G;
    a.chunk_elems = c.chunk_elems;
    a.n_rows = c.n_rows;
    a.gmask = 0;
    for (uint32_t w = 0; w < c.W; ++w)
        if (c.h_active[w]) a.gmask |= 1ull << (w / kChunkWords);
    a.sagg = nullptr;
    a.saggu = nullptr;
    const bool hot = c.hot_rows > 0 && !(flags & GSS_TEST_NO_HOT);
    a.hot_rows = hot ? c.hot_rows : 0;
    a.reports = c.reports;
    a.seg_counts = c.seg_counts;
    a.seg_cap = c.seg_cap;
    a.dense = c.dense;
    a.agg = nullptr;
    a.aggu = nullptr;
    a.wave_stats = (flags & GSS_TEST_COUNT) ? c.wave_stats : nullptr;
    if (flags & GSS_TEST_AGGREGATE) {
        if (!c.agg_valid) {
            agg_rebuild(c, 0, 2ull * ((uint64_t)c.cfg.num_vars + 1));
            c.agg_valid = true;
        }
        a.agg = c.agg;
        if (flags & GSS_TEST_TRIGGER) {
            if (!c.aggu_valid) aggu_rebuild(c);
            a.aggu = c.aggu;
        }
        if (c.G > 1) {  // the super-group bits above the word bits
            super_rebuild(c, (flags & GSS_TEST_TRIGGER) != 0);
            a.sagg = c.sagg;
            a.saggu = c.saggu;
        }
    }
    // the device copy is uploaded again only when the descriptors changed (a
    // growth, compaction or new schedule arrays; not a removal or a delta)
    if (nb && (c.desc_shadow.size() != nb || std::memcmp(c.desc_shadow.data(), h, nb * sizeof(BucketDesc)) != 0)) {
        GSS_HIP(hipMemcpyAsync(c.d_desc, h, nb * sizeof(BucketDesc), hipMemcpyHostToDevice, c.stream));
        c.desc_shadow.assign(h, h + nb);
    }
    L.descs = (const BucketDesc *)c.d_desc;
    L.fn = pick_kernel(c.RWc, (flags & GSS_TEST_TRIGGER) ? 1 : 0, hot, a.agg != nullptr, c.G > 1, listed);
    if (hot) L.lds = (size_t)a.hot_rows * c.RW * 8;
    // persistent: exactly as many workgroups as fit on the device at once
    if (c.occ_fn != (const void *)L.fn || c.occ_lds != L.lds) {  // the query costs host time: cache it
        GSS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&c.occ_fit, L.fn, kTestWavesPerBlock * 64, L.lds));
        c.occ_fn = (const void *)L.fn;
        c.occ_lds = L.lds;
    }
    const int fit = c.occ_fit;
    const uint64_t per_cu = std::max<int>(1, std::min<int>(fit, (int)kTestBlocksPerCU));
    const uint64_t one_tile_each = (tiles + kTestWavesPerBlock - 1) / kTestWavesPerBlock;
    L.grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(one_tile_each, per_cu * c.n_cu));
    return L;
}

// Report segments of one launch: the records of each wavefront, their counts and
// the exclusive prefix of the kept records.  The context's own buffers, or the
// scratch array of gss_test_noalloc.
struct Segments {
    gss_report *reports;
    uint32_t *counts;
    uint64_t *offsets;
    uint32_t cap;
};

static Segments context_segments(Ctx &c) { return Segments{c.reports, c.seg_counts, c.seg_offsets, c.seg_cap}; }

// Queues the test kernel and the finalize kernel, which writes the summary and
// the test's serial into pinned host memory.
static void launch(Ctx &c, const Launch &L, uint32_t flags, const Segments &sg) {
    const uint64_t serial = c.tests_launched + 1;
    // timing events around the kernel on every timing_interval-th launch (each
    // event leaves the stream idle for a few microseconds; attaching them to the
    // dispatch instead, with hipExtLaunchKernel, measured slower: 24 against 10 us
    // of host time per launch, on the path between two tests)
    c.timed = serial % std::max<uint32_t>(1u, c.cfg.timing_interval) == 0;
    if (c.timed) GSS_HIP(hipEventRecord(c.ev_start, c.stream));
    hipLaunchKernelGGL(L.fn, dim3(L.grid), dim3(kTestWavesPerBlock * 64), L.lds, c.stream, L.descs, L.args,
                       (flags & GSS_TEST_NO_EARLY_EXIT) ? 0u : 1u, (flags & GSS_TEST_DENSE) ? 1u : 0u);
    GSS_HIP(hipGetLastError());
    if (c.timed) GSS_HIP(hipEventRecord(c.ev_stop, c.stream));
    const uint32_t n_waves = L.grid * kTestWavesPerBlock;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, c.stream, sg.counts, n_waves, sg.cap, sg.offsets,
                       c.d_summary, deferred_flag(c), c.hd_summary, (unsigned long long)serial);
    GSS_HIP(hipGetLastError());
    c.tests_launched = serial;
    c.last_waves = n_waves;
    c.launch_mutations = c.mutations;
}

// True once the last launched test's finalize kernel has written its serial to
// the host; a device error on the stream is raised.
static bool summary_arrived(Ctx &c, bool check_stream) {
    const volatile unsigned long long *hs = c.h_summary;
    if (hs[4] == c.tests_launched) {
        std::atomic_thread_fence(std::memory_order_acquire);  // the summary words were written before it
        return true;
    }
    if (check_stream) {
        const hipError_t e = hipStreamQuery(c.stream);
        if (e != hipErrorNotReady) {
            GSS_HIP(e);
            // the stream is idle: the serial must be there now
            GSS_REQUIRE(hs[4] == c.tests_launched, GSS_ERR_DEVICE, "the test summary did not arrive");
            std::atomic_thread_fence(std::memory_order_acquire);
            return true;
        }
    }
    return false;
}

// Waits for a launched test and records its kernel time.  The wait polls the
// serial in pinned memory rather than blocking in the runtime: the caller is
// about to queue the next test, and a blocked thread wakes too late to keep the
// device busy.  The stream is queried now and then for device errors.
static void complete(Ctx &c) {
    for (uint32_t spins = 1; !summary_arrived(c, (spins & 1023) == 0); ++spins) {
    }
    c.tests_completed = c.tests_launched;
    c.release_deferred();
    c.stats.kernel_launches++;
    if (!c.timed) return;
    GSS_HIP(hipEventSynchronize(c.ev_stop));  // recorded before the finalize kernel: already complete
    float ms = 0.f;
    GSS_HIP(hipEventElapsedTime(&ms, c.ev_start, c.ev_stop));
    c.stats.last_kernel_ms = ms;
    c.stats.total_kernel_ms += ms;
    c.stats.timed_launches++;
}

// Checks flags and prepares a test; returns false when there is nothing to launch.
static bool begin_test(Ctx &c, uint32_t flags, Launch &L) {
    const uint32_t known = GSS_TEST_TRIGGER | GSS_TEST_NO_EARLY_EXIT | GSS_TEST_SORTED | GSS_TEST_DENSE |
                           GSS_TEST_NO_REGROW | GSS_TEST_NO_HOT | GSS_TEST_SCHEDULED | GSS_TEST_AGGREGATE |
                           GSS_TEST_COUNT;
    GSS_REQUIRE((flags & ~known) == 0, GSS_ERR_INVALID_ARG, "unknown gss_test flag");
    GSS_REQUIRE(!((flags & GSS_TEST_SORTED) && (flags & GSS_TEST_DENSE)), GSS_ERR_INVALID_ARG,
                "GSS_TEST_SORTED orders records; GSS_TEST_DENSE produces none");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is already in flight (call gss_test_wait)");
    if (flags & GSS_TEST_DENSE) {
        const uint64_t rows = std::max<uint64_t>(c.id_loc.size(), 1);
        if (rows > c.dense_rows) {
            uint64_t want = std::max<uint64_t>(rows, c.dense_rows + c.dense_rows / 2);
            uint64_t *p = (uint64_t *)c.dalloc(want * c.W * 8);
            c.dfree(c.dense);
            c.dense = p;
            c.dense_rows = want;
        }
        launch_fill_u64(c, c.dense, c.dense_rows * c.W, 0);
        c.dense_ids = c.id_loc.size();
    }
    if ((flags & GSS_TEST_COUNT) && !c.wave_stats) c.wave_stats = (uint32_t *)c.dalloc((uint64_t)c.max_waves * 8);
    uint64_t act = 0;
    for (uint64_t x : c.h_active) act += __builtin_popcountll(x);
    uint64_t lits = 0;
    for (const auto &B : c.buckets) lits += B.n_lits;
    // hot rows: ranked by occurrences the first time, and again whenever the
    // store has doubled since (never while a server owns the context)
    if (c.hot_rows && !(flags & GSS_TEST_NO_HOT) && !c.serving && lits > 2 * c.ranked_lits) rank_vars(c);
    c.stats.last_pairs = c.live * act;
    c.stats.last_literals = lits;
    c.tested = false;
    L = prepare(c, flags);
    if (L.args.n_tiles == 0) {
        c.last_waves = 0;
        return false;
    }
    launch(c, L, flags, context_segments(c));
    return true;
}

// Completes a test begun by begin_test: waits, grows the report segments and
// repeats the test once if they overflowed (unless GSS_TEST_NO_REGROW), and
// publishes the counts.  Throws GSS_ERR_REPORT_OVERFLOW when records were lost.
static uint64_t end_test(Ctx &c, uint32_t flags, bool launched) {
    uint64_t n = 0, kept = 0;
    if (launched) {
        complete(c);
        n = c.h_summary[0];
        kept = c.h_summary[2];
        const uint64_t largest = c.h_summary[1];
        if (!(flags & GSS_TEST_DENSE) && largest > c.seg_cap && !(flags & GSS_TEST_NO_REGROW)) {
            const uint64_t want = largest + largest / 8 + kMinSegment;
            bool grown = false;
            try {
                gss_report *p = (gss_report *)c.dalloc((uint64_t)c.max_waves * want * sizeof(gss_report));
                c.dfree(c.reports);
                c.reports = p;
                c.seg_cap = (uint32_t)want;
                c.version++;
                grown = true;
            } catch (const Error &e) {
                if (e.code != GSS_ERR_CAPACITY) throw;
            }
            // Repeating the test is only right while the state it saw is unchanged:
            // changes queued behind an asynchronous test would be in the rerun.
            if (grown && c.mutations == c.launch_mutations) {
                c.stats.regrows++;
                Launch L = prepare(c, flags);
                launch(c, L, flags, context_segments(c));
                complete(c);
                n = c.h_summary[0];
                kept = c.h_summary[2];
            }
        }
    }
    c.stats.last_gathers = c.stats.last_gather_bytes = c.stats.last_agg_settled = 0;
    if (launched && (flags & GSS_TEST_COUNT)) {  // the kernel's own counts, summed over its wavefronts
        std::vector<uint32_t> ws(2ull * c.last_waves);
        GSS_HIP(hipMemcpyAsync(ws.data(), c.wave_stats, ws.size() * 4, hipMemcpyDeviceToHost, c.stream));
        c.sync();
        for (size_t i = 0; i < ws.size(); i += 2) {
            c.stats.last_gathers += ws[i];
            c.stats.last_agg_settled += ws[i + 1];
        }
        // a lane reads min(row words, 4) words of a row per gather; trigger mode two rows
        const uint64_t per = 8ull * std::min<uint32_t>(c.RWc, 4) * ((flags & GSS_TEST_TRIGGER) ? 2 : 1);
        c.stats.last_gather_bytes = c.stats.last_gathers * per;
    }
    c.stats.tests_run++;
    c.test_serial++;
    c.tested = true;
    c.last_flags = flags;
    if (flags & GSS_TEST_DENSE) n = kept = 0;
    c.n_reports = n;
    c.n_kept = kept;
    c.stats.last_reports = n;
    // a failed asynchronous update is reported here; the test itself ran on the
    // state without it, and its records stay available
    report_deferred(c, launched ? (uint32_t)c.h_summary[3] : read_deferred(c));
    GSS_REQUIRE(kept == n, GSS_ERR_REPORT_OVERFLOW,
                "report segments of " + std::to_string(c.seg_cap) + " records kept " + std::to_string(kept) + " of " +
                    std::to_string(n) + " records");
    return n;
}

static void queue_stitch(Ctx &c, const Segments &sg, gss_report *dst, uint64_t n) {
    if (!n) return;
    const unsigned grid = std::max<uint32_t>(1, std::min<uint32_t>(c.last_waves, 65535));
    hipLaunchKernelGGL(k_stitch, dim3(grid), dim3(256), 0, c.stream, sg.reports, sg.counts, sg.offsets, sg.cap,
                       c.last_waves, n, dst);
    GSS_HIP(hipGetLastError());
}

void queue_stitch(Ctx &c, gss_report *dst, uint64_t n) { queue_stitch(c, context_segments(c), dst, n); }

}  // namespace gss

using namespace gss;

extern "C" gss_status gss_test(gss_ctx *ctx, uint32_t flags, uint64_t *out_n_reports) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    if (out_n_reports) *out_n_reports = 0;
    Launch L;
    const bool launched = begin_test(c, flags, L);
    try {
        const uint64_t n = end_test(c, flags, launched);
        if (out_n_reports) *out_n_reports = n;
    } catch (const Error &e) {
        if (out_n_reports) *out_n_reports = c.n_reports;
        throw;
    }
    GSS_API_END
}

extern "C" gss_status gss_test_async(gss_ctx *ctx, uint32_t flags) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Launch L;
    c.pending_launched = begin_test(c, flags, L);
    c.pending = true;
    c.pending_flags = flags;
    GSS_API_END
}

extern "C" gss_status gss_test_wait(gss_ctx *ctx, uint64_t *out_n_reports) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(c.pending, GSS_ERR_STATE, "no test in flight");
    GSS_REQUIRE(!c.batch_pending, GSS_ERR_STATE, "the test in flight is a batch's (call gss_batch_wait)");
    c.pending = false;
    if (out_n_reports) *out_n_reports = 0;
    try {
        const uint64_t n = end_test(c, c.pending_flags, c.pending_launched);
        if (out_n_reports) *out_n_reports = n;
    } catch (const Error &e) {
        if (out_n_reports) *out_n_reports = c.n_reports;
        throw;
    }
    GSS_API_END
}

extern "C" gss_status gss_poll(gss_ctx *ctx, uint64_t *out_n_reports) {
    int done = 0;
    const gss_status q = gss_test_query(ctx, &done);
    if (q != GSS_OK) return q;
    if (!done) return GSS_NOT_READY;
    return gss_test_wait(ctx, out_n_reports);
}

extern "C" gss_status gss_test_query(gss_ctx *ctx, int *done) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(done != nullptr, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(c.pending, GSS_ERR_STATE, "no test in flight");
    GSS_REQUIRE(!c.batch_pending, GSS_ERR_STATE, "the test in flight is a batch's (call gss_batch_wait)");
    if (!c.pending_launched) {
        *done = 1;
    } else {
        *done = summary_arrived(c, true) ? 1 : 0;
    }
    GSS_API_END
}

extern "C" gss_status gss_fetch_reports(gss_ctx *ctx, gss_report *out, uint64_t cap, uint64_t *out_n) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight (call gss_test_wait)");
    GSS_REQUIRE(c.tested, GSS_ERR_STATE, "no test has run yet");
    GSS_REQUIRE(out_n != nullptr, GSS_ERR_INVALID_ARG, "null argument");
    const uint64_t n = std::min(c.n_kept, cap);
    *out_n = 0;
    if (n) {
        GSS_REQUIRE(out != nullptr, GSS_ERR_INVALID_ARG, "null argument");
        const bool dev = is_device_pointer(out);
        gss_report *dst = dev ? out : (gss_report *)c.device_stage(n * sizeof(gss_report));
        if (c.last_flags & GSS_TEST_SORTED) {
            // every kept record takes part in the order; the first n of it are returned
            const uint64_t all = c.n_kept;
            gss_report *st = (gss_report *)c.dalloc(all * sizeof(gss_report));
            gss_report *so = (dev && n == all) ? dst : (gss_report *)c.dalloc(all * sizeof(gss_report));
            try {
                queue_stitch(c, st, all);
                sort_records(c, st, all, so);
                if (so != dst)
                    GSS_HIP(hipMemcpyAsync(dst, so, n * sizeof(gss_report), hipMemcpyDeviceToDevice, c.stream));
                c.sync();
            } catch (...) {
                (void)hipStreamSynchronize(c.stream);
                c.dfree(st);
                if (so != dst) c.dfree(so);
                throw;
            }
            c.dfree(st);
            if (so != dst) c.dfree(so);
        } else {
            queue_stitch(c, dst, n);
        }
        if (!dev) GSS_HIP(hipMemcpyAsync(out, dst, n * sizeof(gss_report), hipMemcpyDeviceToHost, c.stream));
        c.sync();
    }
    *out_n = n;
    GSS_API_END
}

extern "C" gss_status gss_fetch_masks(gss_ctx *ctx, const uint32_t *ids, uint32_t n, uint64_t *out) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(c.tested && (c.last_flags & GSS_TEST_DENSE), GSS_ERR_STATE, "no dense test has run");
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(ids && out, GSS_ERR_INVALID_ARG, "null argument");
    std::vector<uint32_t> q(n);
    for (uint32_t i = 0; i < n; ++i) {
        GSS_REQUIRE(ids[i] < c.id_loc.size(), GSS_ERR_UNKNOWN_ID, "clause id " + std::to_string(ids[i]) + " never issued");
        // the dense rows cover the ids issued when the test ran; a clause added
        // since has no row (and may lie beyond the buffer)
        GSS_REQUIRE(ids[i] < c.dense_ids, GSS_ERR_STATE,
                    "clause id " + std::to_string(ids[i]) + " was added after the last dense test");
        q[i] = c.id_loc[ids[i]] == kNoLoc ? kDeadId : ids[i];
    }
    const size_t ids_bytes = ((size_t)n * 4 + 255) / 256 * 256;
    const size_t out_bytes = (size_t)n * c.W * 8;
    char *d = (char *)c.device_stage(ids_bytes + out_bytes);
    GSS_HIP(hipMemcpyAsync(d, q.data(), (size_t)n * 4, hipMemcpyHostToDevice, c.stream));
    const uint64_t total = (uint64_t)n * c.W;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((total + 255) / 256, 16384));
    hipLaunchKernelGGL(k_gather_rows, dim3(grid), dim3(256), 0, c.stream, (uint64_t *)(d + ids_bytes), c.dense,
                       (const uint32_t *)d, n, c.W);
    GSS_HIP(hipGetLastError());
    GSS_HIP(hipMemcpyAsync(out, d + ids_bytes, out_bytes, hipMemcpyDefault, c.stream));
    c.sync();
    GSS_API_END
}

// ---------------------------------------------------------------------------
// A test that allocates nothing, for callers that cannot allocate device memory.
// Its report segments, their counts and offsets live in a file-scope device
// array: one copy per GPU, held from the library's first context on that GPU
// until the process ends.
// ---------------------------------------------------------------------------

namespace gss {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices] = {};  // device address of `scratch` per GPU

// Called by gss_create with the context's device current.  Host code uses the
// address returned here, never the array's name (a host-side stand-in).
void scratch_setup(int device) {
    GSS_REQUIRE(device >= 0 && device < kMaxDevices, GSS_ERR_DEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        throw Error(GSS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = p;
}

static void *scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < kMaxDevices ? g_scratch[device] : nullptr;
}

// Carves the segments of a launch of n_waves wavefronts out of the scratch array:
// counts, offsets, then records.  Too many wavefronts for kMinSegment records
// each: GSS_ERR_CAPACITY.
static Segments scratch_segments(void *base, uint32_t n_waves) {
    const uint64_t counts_bytes = ((uint64_t)n_waves * 4 + 255) / 256 * 256;
    const uint64_t offsets_bytes = (((uint64_t)n_waves + 1) * 8 + 255) / 256 * 256;
    const uint64_t head = counts_bytes + offsets_bytes;
    const uint64_t per_wave = head < kScratchBytes ? (kScratchBytes - head) / sizeof(gss_report) / n_waves : 0;
    GSS_REQUIRE(per_wave >= kMinSegment, GSS_ERR_CAPACITY,
                "a test of " + std::to_string(n_waves) + " wavefronts needs more than the " +
                    std::to_string(kScratchBytes) + " bytes of scratch memory");
    char *p = static_cast<char *>(base);
    Segments sg;
    sg.counts = reinterpret_cast<uint32_t *>(p);
    sg.offsets = reinterpret_cast<uint64_t *>(p + counts_bytes);
    sg.reports = reinterpret_cast<gss_report *>(p + head);
    sg.cap = (uint32_t)std::min<uint64_t>(per_wave, 0xFFFFFFFFull);
    return sg;
}

}  // namespace gss

extern "C" gss_status gss_test_noalloc(gss_ctx *ctx, uint32_t flags, gss_report *out, uint64_t cap,
                                       uint64_t *out_n_reports) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    if (out_n_reports) *out_n_reports = 0;
    const uint32_t known = GSS_TEST_TRIGGER | GSS_TEST_NO_EARLY_EXIT | GSS_TEST_NO_REGROW | GSS_TEST_NO_HOT |
                           GSS_TEST_AGGREGATE;
    GSS_REQUIRE((flags & ~known) == 0, GSS_ERR_INVALID_ARG,
                "gss_test_noalloc takes GSS_TEST_TRIGGER, NO_EARLY_EXIT, NO_REGROW, NO_HOT and AGGREGATE only");
    GSS_REQUIRE(out_n_reports != nullptr, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(cap == 0 || (out != nullptr && is_device_pointer(out)), GSS_ERR_INVALID_ARG,
                "out must be device memory with room for cap records");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is already in flight (call gss_test_wait)");
    // the trigger form of the aggregate pre-test needs bits the context allocates
    // on its first use
    if ((flags & GSS_TEST_AGGREGATE) && (flags & GSS_TEST_TRIGGER))
        GSS_REQUIRE(c.aggu != nullptr && (c.G == 1 || c.saggu != nullptr), GSS_ERR_STATE,
                    "run one gss_test with GSS_TEST_TRIGGER | GSS_TEST_AGGREGATE first (it allocates the "
                    "canBeUndef bits)");
    void *base = scratch_of(c.device);
    GSS_REQUIRE(base != nullptr, GSS_ERR_STATE, "scratch memory was not set up on this device");
    uint64_t act = 0;
    for (uint64_t x : c.h_active) act += __builtin_popcountll(x);
    uint64_t lits = 0;
    for (const auto &B : c.buckets) lits += B.n_lits;
    c.stats.last_pairs = c.live * act;
    c.stats.last_literals = lits;

    Launch L = prepare(c, flags);
    uint64_t n = 0, kept = 0;
    if (L.args.n_tiles) {
        const Segments sg = scratch_segments(base, L.grid * kTestWavesPerBlock);
        L.args.reports = sg.reports;
        L.args.seg_counts = sg.counts;
        L.args.seg_cap = sg.cap;
        // the context's records of an earlier test are not touched; they are no
        // longer the last test's
        c.tested = false;
        launch(c, L, flags, sg);
        complete(c);
        n = c.h_summary[0];
        kept = c.h_summary[2];
        const uint64_t m = std::min(kept, cap);
        queue_stitch(c, sg, out, m);
        c.sync();
        report_deferred(c, (uint32_t)c.h_summary[3]);
    } else {
        c.last_waves = 0;
        c.tested = false;
        report_deferred(c, read_deferred(c));
    }
    c.stats.tests_run++;
    c.stats.last_reports = n;
    c.test_serial++;
    *out_n_reports = n;
    GSS_REQUIRE(kept == n, GSS_ERR_REPORT_OVERFLOW,
                "the scratch segments kept " + std::to_string(kept) + " of " + std::to_string(n) + " records");
    GSS_REQUIRE(n <= cap, GSS_ERR_REPORT_OVERFLOW,
                "out holds " + std::to_string(cap) + " of " + std::to_string(n) + " records");
    GSS_API_END
}
