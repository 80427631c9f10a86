// Batched clause test: several independent stores (each its own clause database,
// variable count and slot width) tested in one persistent launch.  Global tiles
// follow a schedule -- the order in which the stores' tiles are dealt to the
// wavefronts -- and every wavefront keeps, per store, its own report segment in
// that store's context, so each context reads its results exactly as after its
// own gss_test.  The launch sequence can be captured in a hipGraph and replayed
// while the stores, the schedule and the flags stay the same.
#include "tester.h"

#include <algorithm>
#include <cstring>

namespace gss {

constexpr uint32_t kMaxBatch = 64;

// One store as the batched kernel sees it.
struct StoreDesc {
    const BucketDesc *descs;
    const uint64_t *planes;
    const uint64_t *active;
    gss_report *reports;
    uint32_t *seg_counts;
    uint64_t *seg_offsets;
    uint32_t n_buckets;
    uint32_t n_tiles;
    uint32_t W;
    uint32_t RW;
    uint32_t seg_cap;
    uint32_t pad;
    const uint32_t *deferred;  // the context's verdict of queued updates (reported after the test)
    const void *agg;           // GSS_TEST_AGGREGATE: the context's aggregate bits (null otherwise)
    const void *aggu;          // and, in trigger mode, its canBeUndef bits
};

// A run of `count` consecutive tiles of one store, starting at its tile `tile0`;
// `begin` is the global index of the run's first tile.
struct SchedSeg {
    uint32_t store;
    uint32_t tile0;
    uint32_t begin;
    uint32_t count;
};

// Lanes per clause of a store whose rows hold RW words: one per 32-byte sector.
__device__ inline uint32_t lanes_per_clause(uint32_t RW) { return RW <= 4 ? 1u : RW / 4; }

template <int LPC, int WPL, int MODE, bool AGG>
__device__ uint32_t batch_run(const StoreDesc &st, const TileRef &cur, gss_report *seg, uint32_t produced,
                              uint32_t early_exit) {
    using Ts = Tester<LPC, WPL, MODE, false, AGG>;
    const Ts ts(threadIdx.x & 63, st.planes, st.active, st.W, 0, nullptr, 0u, st.agg, st.aggu);
    Counts none;
    return ts.run(cur, seg, st.seg_cap, produced, early_exit, nullptr, none);
}

// The store and store-local tile of global tile g: segs[lo].begin <= g < segs[lo + 1].begin.
__device__ inline void locate(const SchedSeg *segs, uint32_t n_segs, uint32_t g, uint32_t &store, uint32_t &tile) {
    uint32_t lo = 0, hi = n_segs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (segs[mid].begin <= g) lo = mid; else hi = mid;
    }
    store = segs[lo].store;
    tile = segs[lo].tile0 + (g - segs[lo].begin);
}

// Each wavefront walks the global tiles g = wave, wave + N, ... and, like the
// single-store kernel, opens the next tile (its store located, its metadata and
// first codes in flight) while it tests the current one.
// The falsified kernel fits 5 wavefronts per SIMD in 96 registers without
// spilling (4 unconstrained); the others would spill, and keep their own count.
template <int MODE, bool AGG>
__global__ __launch_bounds__(kTestWavesPerBlock * 64)
__attribute__((amdgpu_waves_per_eu(MODE == 0 && !AGG ? 5 : 1))) void k_test_batch(const StoreDesc *__restrict__ stores,
                                                                         uint32_t n_stores,
                                                                         const SchedSeg *__restrict__ segs,
                                                                         uint32_t n_segs, uint32_t total,
                                                                         uint32_t early_exit) {
    __shared__ uint32_t counts[kTestWavesPerBlock][kMaxBatch];  // records per (wavefront, store)
    const uint32_t lane = threadIdx.x & 63, wib = threadIdx.x / 64;
    for (uint32_t s = lane; s < n_stores; s += 64) counts[wib][s] = 0;
    __syncthreads();
    const uint32_t n_waves = gridDim.x * kTestWavesPerBlock;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * kTestWavesPerBlock + wib);
    auto open = [&](uint32_t g, uint32_t &store, TileRef &tl) {
        uint32_t tile, bi = 0;
        locate(segs, n_segs, g, store, tile);
        const StoreDesc &st = stores[store];
        const uint32_t lpc = lanes_per_clause(st.RW);
        open_tile(st.descs, st.n_buckets, bi, tile, lane / lpc, 64 / lpc, tl);
    };
    uint32_t g = wave, s_cur = 0;
    TileRef cur;
    if (g < total) open(g, s_cur, cur);
    while (g < total) {
        const uint32_t gn = g + n_waves;
        uint32_t s_nxt = s_cur;
        TileRef nxt = cur;
        if (gn < total) open(gn, s_nxt, nxt);  // in flight while the current tile is tested
        const StoreDesc &st = stores[s_cur];
        gss_report *const seg = st.reports + (uint64_t)wave * st.seg_cap;
        uint32_t produced = counts[wib][s_cur];
        switch (st.RW) {
        case 1: produced = batch_run<1, 1, MODE, AGG>(st, cur, seg, produced, early_exit); break;
        case 2: produced = batch_run<1, 2, MODE, AGG>(st, cur, seg, produced, early_exit); break;
        case 4: produced = batch_run<1, 4, MODE, AGG>(st, cur, seg, produced, early_exit); break;
        case 8: produced = batch_run<2, 4, MODE, AGG>(st, cur, seg, produced, early_exit); break;
        case 16: produced = batch_run<4, 4, MODE, AGG>(st, cur, seg, produced, early_exit); break;
        case 32: produced = batch_run<8, 4, MODE, AGG>(st, cur, seg, produced, early_exit); break;
        default: produced = batch_run<16, 4, MODE, AGG>(st, cur, seg, produced, early_exit); break;
        }
        counts[wib][s_cur] = produced;
        g = gn;
        s_cur = s_nxt;
        cur = nxt;
    }
    for (uint32_t s = lane; s < n_stores; s += 64) stores[s].seg_counts[wave] = counts[wib][s];
}

// One workgroup per store: totals and segment offsets, as k_finalize.
__global__ __launch_bounds__(1024) void k_finalize_batch(const StoreDesc *stores, uint32_t n_waves,
                                                          unsigned long long *summary) {
    const StoreDesc &st = stores[blockIdx.x];
    finalize_segments(st.seg_counts, n_waves, st.seg_cap, st.seg_offsets, summary + 4 * blockIdx.x);
    if (threadIdx.x == 0) summary[4 * blockIdx.x + 3] = *st.deferred;  // the thread that wrote the others
}

}  // namespace gss

using namespace gss;

struct gss_batch {
    std::vector<Ctx *> ctxs;
    hipStream_t stream = nullptr;
    gss_schedule sched{GSS_ORDER_INTERLEAVE, 64, 0, 0};
    // device and pinned host copies of the launch's tables
    StoreDesc *d_stores = nullptr, *h_stores = nullptr;
    BucketDesc *d_descs = nullptr, *h_descs = nullptr;
    SchedSeg *d_segs = nullptr, *h_segs = nullptr;
    uint32_t seg_capacity = 0;
    unsigned long long *d_summary = nullptr, *h_summary = nullptr;
    uint32_t n_segs = 0, total = 0, grid = 0;
    std::vector<uint32_t> n_tiles;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_valid = false;
    std::vector<uint64_t> versions;
    uint32_t graph_flags = 0;
    gss_schedule graph_sched{};
    uint64_t captures = 0, launches = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;
    std::string last_error;
    // gss_batch_test_async issued, gss_batch_wait not yet called
    bool pending = false;
    uint32_t pending_flags = 0;
    std::vector<uint64_t> launch_mutations;  // each member's change count when the test was queued
};

namespace {

void free_graph(gss_batch &b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.graph_valid = false;
}

void destroy_batch(gss_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->pending)  // destroyed with a test in flight: the members are usable again
        for (Ctx *c : b->ctxs) {
            c->pending = false;
            c->batch_pending = false;
            c->mark_idle();
        }
    free_graph(*b);
    Ctx &c0 = *b->ctxs[0];
    c0.dfree(b->d_stores);
    c0.dfree(b->d_descs);
    c0.dfree(b->d_segs);
    c0.dfree(b->d_summary);
    if (b->h_stores) (void)hipHostFree(b->h_stores);
    if (b->h_descs) (void)hipHostFree(b->h_descs);
    if (b->h_segs) (void)hipHostFree(b->h_segs);
    if (b->h_summary) (void)hipHostFree(b->h_summary);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
}

// Tile runs of one store, per non-empty length class: (stride_log2, first tile, count).
struct Run {
    uint32_t s_log2, tile0, count;
};

// Fills the descriptor tables of every store and the schedule of global tiles.
void plan(gss_batch &b, uint32_t flags) {
    const uint32_t n = (uint32_t)b.ctxs.size();
    std::vector<std::vector<Run>> runs(n);
    b.n_tiles.assign(n, 0);
    for (uint32_t s = 0; s < n; ++s) {
        Ctx &c = *b.ctxs[s];
        uint32_t nb = 0, tiles = 0;
        for (int k = 0; k < kMaxBuckets; ++k) {
            const Bucket &B = c.buckets[k];
            if (B.n_slots == 0 || B.n_dead == B.n_slots) continue;
            BucketDesc d{};
            d.lits = B.lits;
            d.meta = B.meta;
            d.lits_bytes = B.cap_slots << B.stride_log2 << 2;
            d.meta_bytes = B.cap_slots * 8;
            d.stride_log2 = B.stride_log2;
            d.tile_begin = tiles;
            b.h_descs[s * kMaxBuckets + nb++] = d;
            const uint32_t nt = (uint32_t)((B.n_slots + c.T - 1) / c.T);
            runs[s].push_back(Run{B.stride_log2, tiles, nt});
            tiles += nt;
        }
        b.n_tiles[s] = tiles;
        StoreDesc &sd = b.h_stores[s];
        sd.descs = b.d_descs + s * kMaxBuckets;
        sd.planes = c.planes;
        sd.active = c.active;
        sd.reports = c.reports;
        sd.seg_counts = c.seg_counts;
        sd.seg_offsets = c.seg_offsets;
        sd.n_buckets = nb;
        sd.n_tiles = tiles;
        sd.W = c.W;
        sd.RW = c.RW;
        sd.seg_cap = c.seg_cap;
        sd.pad = 0;
        sd.deferred = deferred_flag(c);
        sd.agg = (flags & GSS_TEST_AGGREGATE) ? c.agg : nullptr;
        sd.aggu = (flags & GSS_TEST_AGGREGATE) && (flags & GSS_TEST_TRIGGER) ? c.aggu : nullptr;
    }

    std::vector<SchedSeg> segs;
    uint32_t begin = 0;
    auto emit = [&](uint32_t s, uint32_t tile0, uint32_t count) {
        if (!count) return;
        segs.push_back(SchedSeg{s, tile0, begin, count});
        begin += count;
    };
    const uint32_t chunk = b.sched.chunk_tiles ? b.sched.chunk_tiles : 64;
    if (b.sched.order == GSS_ORDER_STORE) {
        for (uint32_t s = 0; s < n; ++s) emit(s, 0, b.n_tiles[s]);
    } else if (b.sched.order == GSS_ORDER_INTERLEAVE) {
        std::vector<uint32_t> done(n, 0);
        for (bool more = true; more;) {
            more = false;
            for (uint32_t s = 0; s < n; ++s) {
                const uint32_t take = std::min(chunk, b.n_tiles[s] - done[s]);
                emit(s, done[s], take);
                done[s] += take;
                more |= done[s] < b.n_tiles[s];
            }
        }
    } else {  // longest clauses first: length classes by decreasing stride, stores interleaved within one
        for (int sl = kMaxBuckets - 1; sl >= 0; --sl) {
            std::vector<Run> cls(n, Run{0, 0, 0});
            for (uint32_t s = 0; s < n; ++s)
                for (const Run &r : runs[s])
                    if ((int)r.s_log2 == sl) cls[s] = r;
            for (bool more = true; more;) {
                more = false;
                for (uint32_t s = 0; s < n; ++s) {
                    const uint32_t take = std::min(chunk, cls[s].count);
                    emit(s, cls[s].tile0, take);
                    cls[s].tile0 += take;
                    cls[s].count -= take;
                    more |= cls[s].count > 0;
                }
            }
        }
    }
    if (segs.empty()) segs.push_back(SchedSeg{0, 0, 0, 0});
    Ctx &c0 = *b.ctxs[0];
    if (segs.size() > b.seg_capacity) {
        c0.sync();
        c0.dfree(b.d_segs);
        if (b.h_segs) (void)hipHostFree(b.h_segs);
        b.seg_capacity = (uint32_t)(segs.size() + segs.size() / 2);
        b.d_segs = (SchedSeg *)c0.dalloc((size_t)b.seg_capacity * sizeof(SchedSeg));
        GSS_HIP(hipHostMalloc(&b.h_segs, (size_t)b.seg_capacity * sizeof(SchedSeg), hipHostMallocDefault));
    }
    std::copy(segs.begin(), segs.end(), b.h_segs);
    b.n_segs = (uint32_t)segs.size();
    b.total = begin;
}

using BatchFn = void (*)(const StoreDesc *, uint32_t, const SchedSeg *, uint32_t, uint32_t, uint32_t);

BatchFn batch_kernel(uint32_t flags) {
    const bool agg = flags & GSS_TEST_AGGREGATE;
    if (flags & GSS_TEST_TRIGGER) return agg ? k_test_batch<1, true> : k_test_batch<1, false>;
    return agg ? k_test_batch<0, true> : k_test_batch<0, false>;
}

// With the aggregate pre-test: each store's bits brought up to date on the shared
// stream before the launch (bulk plane updates leave them stale).  Returns true
// when a store's bits were allocated now (a captured graph holds the old pointers).
bool refresh_aggregates(gss_batch &b, uint32_t flags) {
    if (!(flags & GSS_TEST_AGGREGATE)) return false;
    bool moved = false;
    for (Ctx *c : b.ctxs) {
        if (!c->agg_valid) {
            agg_rebuild(*c, 0, 2ull * ((uint64_t)c->cfg.num_vars + 1));
            c->agg_valid = true;
        }
        if ((flags & GSS_TEST_TRIGGER) && !c->aggu_valid) {
            moved |= c->aggu == nullptr;
            aggu_rebuild(*c);
        }
    }
    return moved;
}

uint32_t grid_for(gss_batch &b, BatchFn fn) {
    Ctx &c0 = *b.ctxs[0];
    int fit = 0;
    GSS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, fn, kTestWavesPerBlock * 64, 0));
    uint32_t per_cu = (uint32_t)std::max(1, std::min(fit, (int)kTestBlocksPerCU));
    if (b.sched.blocks_per_cu) per_cu = std::min(per_cu, b.sched.blocks_per_cu);
    const uint64_t one_tile_each = (b.total + kTestWavesPerBlock - 1) / kTestWavesPerBlock;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(one_tile_each, (uint64_t)per_cu * c0.n_cu));
}

// Queues the table uploads, the batched kernel, the finalize kernel and the copy of
// the summaries on the batch stream (the same sequence is what a graph captures).
void enqueue(gss_batch &b, uint32_t flags) {
    const uint32_t n = (uint32_t)b.ctxs.size();
    GSS_HIP(hipMemcpyAsync(b.d_descs, b.h_descs, (size_t)n * kMaxBuckets * sizeof(BucketDesc), hipMemcpyHostToDevice,
                           b.stream));
    GSS_HIP(hipMemcpyAsync(b.d_stores, b.h_stores, (size_t)n * sizeof(StoreDesc), hipMemcpyHostToDevice, b.stream));
    GSS_HIP(hipMemcpyAsync(b.d_segs, b.h_segs, (size_t)b.n_segs * sizeof(SchedSeg), hipMemcpyHostToDevice, b.stream));
    const BatchFn fn = batch_kernel(flags);
    hipLaunchKernelGGL(fn, dim3(b.grid), dim3(kTestWavesPerBlock * 64), 0, b.stream, b.d_stores, n, b.d_segs, b.n_segs,
                       b.total, (flags & GSS_TEST_NO_EARLY_EXIT) ? 0u : 1u);
    GSS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finalize_batch, dim3(n), dim3(1024), 0, b.stream, b.d_stores, b.grid * kTestWavesPerBlock,
                       b.d_summary);
    GSS_HIP(hipGetLastError());
    GSS_HIP(hipMemcpyAsync(b.h_summary, b.d_summary, (size_t)n * 4 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, b.stream));
}

bool same_schedule(const gss_schedule &x, const gss_schedule &y) {
    return x.order == y.order && x.chunk_tiles == y.chunk_tiles && x.blocks_per_cu == y.blocks_per_cu;
}

// Queues one batched test: plans (unless a valid graph is replayed) and
// launches.  Every member counts it as a test of its own: its serial releases
// the upload slots and deferred frees queued before it once it has completed.
void launch_batch(gss_batch &b, uint32_t flags) {
    const uint32_t n = (uint32_t)b.ctxs.size();
    const bool use_graph = flags & GSS_TEST_GRAPH;
    const bool moved = refresh_aggregates(b, flags);
    bool valid = !moved && use_graph && b.graph_valid && b.graph_flags == flags && same_schedule(b.graph_sched, b.sched);
    for (uint32_t s = 0; valid && s < n; ++s) valid = b.versions[s] == b.ctxs[s]->version;
    if (!valid) {
        plan(b, flags);
        b.grid = grid_for(b, batch_kernel(flags));
    }
    if (use_graph && !valid) {
        free_graph(b);
        GSS_HIP(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
        enqueue(b, flags);
        GSS_HIP(hipStreamEndCapture(b.stream, &b.graph));
        GSS_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
        b.graph_valid = true;
        b.graph_flags = flags;
        b.graph_sched = b.sched;
        b.versions.resize(n);
        for (uint32_t s = 0; s < n; ++s) b.versions[s] = b.ctxs[s]->version;
        b.captures++;
    }
    GSS_HIP(hipEventRecord(b.ev0, b.stream));
    if (use_graph)
        GSS_HIP(hipGraphLaunch(b.exec, b.stream));
    else
        enqueue(b, flags);
    GSS_HIP(hipEventRecord(b.ev1, b.stream));
    b.launch_mutations.resize(n);
    for (uint32_t s = 0; s < n; ++s) {
        Ctx &c = *b.ctxs[s];
        c.tests_launched++;
        b.launch_mutations[s] = c.mutations;
    }
}

// Waits for the queued batched test (work queued after it may still run) and
// publishes every store's counts into its context.  Returns true when some store
// overflowed its report segments.
bool complete_batch(gss_batch &b, uint32_t flags, bool &any_overflow_growable) {
    const uint32_t n = (uint32_t)b.ctxs.size();
    GSS_HIP(hipEventSynchronize(b.ev1));
    float ms = 0.f;
    GSS_HIP(hipEventElapsedTime(&ms, b.ev0, b.ev1));
    b.last_ms = ms;
    b.launches++;

    bool overflow = false;
    any_overflow_growable = false;
    uint64_t act = 0;
    for (uint32_t s = 0; s < n; ++s) {
        Ctx &c = *b.ctxs[s];
        c.tests_completed = c.tests_launched;  // the batch was the member's last queued test
        c.release_deferred();
        const unsigned long long *sum = b.h_summary + 4 * s;
        c.last_waves = b.grid * kTestWavesPerBlock;
        c.n_reports = sum[0];
        c.n_kept = sum[2];
        c.tested = true;
        c.last_flags = flags & ~GSS_TEST_GRAPH;
        c.stats.tests_run++;
        c.stats.last_reports = sum[0];
        act = 0;
        for (uint64_t x : c.h_active) act += __builtin_popcountll(x);
        c.stats.last_pairs = c.live * act;
        uint64_t lits = 0;
        for (const auto &B : c.buckets) lits += B.n_lits;
        c.stats.last_literals = lits;
        if (sum[1] > c.seg_cap) {
            overflow = true;
            if (!(flags & GSS_TEST_NO_REGROW)) {
                const uint64_t want = sum[1] + sum[1] / 8 + kMinSegment;
                try {
                    gss_report *p = (gss_report *)c.dalloc((uint64_t)c.max_waves * want * sizeof(gss_report));
                    c.dfree(c.reports);
                    c.reports = p;
                    c.seg_cap = (uint32_t)want;
                    c.version++;
                    c.stats.regrows++;
                    any_overflow_growable = true;
                } catch (const Error &e) {
                    if (e.code != GSS_ERR_CAPACITY) throw;
                }
            }
        }
    }
    // failed checks of queued updates: every context's verdict is cleared, the first reported
    gss_status bad = GSS_OK;
    std::string why;
    for (uint32_t s = 0; s < n; ++s) {
        try {
            report_deferred(*b.ctxs[s], (uint32_t)b.h_summary[4 * s + 3]);
        } catch (const Error &e) {
            if (bad == GSS_OK) {
                bad = e.code;
                why = std::string("store ") + std::to_string(s) + ": " + e.what();
            }
        }
    }
    GSS_REQUIRE(bad == GSS_OK, bad, why);
    return overflow;
}

// One batched test, waited for.
bool run_once(gss_batch &b, uint32_t flags, bool &any_overflow_growable) {
    launch_batch(b, flags);
    return complete_batch(b, flags, any_overflow_growable);
}

void check_batch_flags(const gss_batch &b, uint32_t flags) {
    const uint32_t known =
        GSS_TEST_TRIGGER | GSS_TEST_NO_EARLY_EXIT | GSS_TEST_NO_REGROW | GSS_TEST_GRAPH | GSS_TEST_AGGREGATE;
    GSS_REQUIRE((flags & ~known) == 0, GSS_ERR_INVALID_ARG, "flag not supported by gss_batch_test");
    GSS_REQUIRE(!b.pending, GSS_ERR_STATE, "the batch has a test in flight (call gss_batch_wait)");
    // a member's asynchronous test would have its report segments overwritten
    for (const Ctx *c : b.ctxs)
        GSS_REQUIRE(!c->pending, GSS_ERR_STATE, "a member context has a test in flight (call gss_test_wait)");
}

}  // namespace

#define GSS_BATCH_BEGIN(bp)                                  \
    gss_batch *b_ = (bp);                                    \
    if (!b_) return GSS_ERR_INVALID_ARG;                     \
    try {                                                    \
        b_->last_error.clear();
#define GSS_BATCH_END                                        \
    }                                                        \
    catch (const ::gss::Error &e) {                          \
        b_->last_error = e.what();                           \
        return e.code;                                       \
    }                                                        \
    catch (const std::exception &e) {                        \
        b_->last_error = e.what();                           \
        return GSS_ERR_DEVICE;                               \
    }                                                        \
    return GSS_OK;

extern "C" gss_status gss_batch_create(gss_ctx *const *ctxs, uint32_t n, gss_batch **out) {
    if (!out) return GSS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctxs || n == 0 || n > kMaxBatch) return GSS_ERR_INVALID_ARG;
    gss_batch *b = new (std::nothrow) gss_batch();
    if (!b) return GSS_ERR_CAPACITY;
    try {
        for (uint32_t i = 0; i < n; ++i) {
            Ctx *c = reinterpret_cast<Ctx *>(ctxs[i]);
            GSS_REQUIRE(c != nullptr, GSS_ERR_INVALID_ARG, "null context");
            for (Ctx *d : b->ctxs) GSS_REQUIRE(d != c, GSS_ERR_INVALID_ARG, "context listed twice");
            b->ctxs.push_back(c);
        }
        Ctx &c0 = *b->ctxs[0];
        b->stream = c0.stream;
        for (Ctx *c : b->ctxs) {
            GSS_REQUIRE(c->device == c0.device, GSS_ERR_INVALID_ARG, "contexts on different devices");
            GSS_REQUIRE(c->stream == c0.stream, GSS_ERR_INVALID_ARG, "contexts on different streams");
            GSS_REQUIRE(c->G == 1, GSS_ERR_INVALID_ARG, "a batch takes contexts of at most 4096 slots");
        }
        b->d_stores = (StoreDesc *)c0.dalloc((size_t)n * sizeof(StoreDesc));
        b->d_descs = (BucketDesc *)c0.dalloc((size_t)n * kMaxBuckets * sizeof(BucketDesc));
        b->d_summary = (unsigned long long *)c0.dalloc((size_t)n * 4 * sizeof(unsigned long long));
        GSS_HIP(hipHostMalloc(&b->h_stores, (size_t)n * sizeof(StoreDesc), hipHostMallocDefault));
        GSS_HIP(hipHostMalloc(&b->h_descs, (size_t)n * kMaxBuckets * sizeof(BucketDesc), hipHostMallocDefault));
        GSS_HIP(hipHostMalloc(&b->h_summary, (size_t)n * 4 * sizeof(unsigned long long), hipHostMallocDefault));
        std::memset(b->h_descs, 0, (size_t)n * kMaxBuckets * sizeof(BucketDesc));
        GSS_HIP(hipEventCreate(&b->ev0));
        GSS_HIP(hipEventCreate(&b->ev1));
    } catch (const std::exception &e) {
        const gss_status code = dynamic_cast<const Error *>(&e) ? static_cast<const Error &>(e).code : GSS_ERR_DEVICE;
        if (b->ctxs.empty()) {
            delete b;
        } else {
            b->ctxs[0]->last_error = e.what();
            destroy_batch(b);
        }
        return code;
    }
    *out = b;
    return GSS_OK;
}

extern "C" void gss_batch_destroy(gss_batch *b) { destroy_batch(b); }

extern "C" const char *gss_batch_last_error(const gss_batch *b) { return b ? b->last_error.c_str() : ""; }

extern "C" gss_status gss_batch_set_schedule(gss_batch *b, const gss_schedule *s) {
    GSS_BATCH_BEGIN(b)
    GSS_REQUIRE(s != nullptr, GSS_ERR_INVALID_ARG, "null schedule");
    GSS_REQUIRE(s->order <= GSS_ORDER_LONGEST_FIRST, GSS_ERR_INVALID_ARG, "unknown schedule order");
    GSS_REQUIRE(s->blocks_per_cu <= kTestBlocksPerCU, GSS_ERR_INVALID_ARG, "blocks_per_cu above 8");
    b_->sched = *s;
    GSS_BATCH_END
}

extern "C" gss_status gss_batch_test(gss_batch *b, uint32_t flags, uint64_t *out_n_reports) {
    GSS_BATCH_BEGIN(b)
    check_batch_flags(*b_, flags);
    bool grown = false;
    bool overflow = run_once(*b_, flags, grown);
    if (overflow && grown) overflow = run_once(*b_, flags, grown);
    const uint32_t n = (uint32_t)b_->ctxs.size();
    if (out_n_reports)
        for (uint32_t s = 0; s < n; ++s) out_n_reports[s] = b_->ctxs[s]->n_reports;
    GSS_REQUIRE(!overflow, GSS_ERR_REPORT_OVERFLOW, "a store's report segments overflowed; its counts are exact");
    GSS_BATCH_END
}

extern "C" gss_status gss_batch_test_async(gss_batch *b, uint32_t flags) {
    GSS_BATCH_BEGIN(b)
    check_batch_flags(*b_, flags);
    launch_batch(*b_, flags);
    b_->pending = true;
    b_->pending_flags = flags;
    for (Ctx *c : b_->ctxs) {
        c->pending = true;
        c->batch_pending = true;
    }
    GSS_BATCH_END
}

extern "C" gss_status gss_batch_wait(gss_batch *b, uint64_t *out_n_reports) {
    GSS_BATCH_BEGIN(b)
    GSS_REQUIRE(b_->pending, GSS_ERR_STATE, "no batched test in flight");
    b_->pending = false;
    for (Ctx *c : b_->ctxs) {
        c->pending = false;
        c->batch_pending = false;
    }
    const uint32_t flags = b_->pending_flags;
    const uint32_t n = (uint32_t)b_->ctxs.size();
    bool grown = false;
    bool overflow = false;
    try {
        overflow = complete_batch(*b_, flags, grown);
        // repeated at once only when no member has changed since the launch (a
        // change queued behind the test would be read by the repeat)
        bool unchanged = true;
        for (uint32_t s = 0; s < n; ++s) unchanged = unchanged && b_->ctxs[s]->mutations == b_->launch_mutations[s];
        if (overflow && grown && unchanged) overflow = run_once(*b_, flags, grown);
    } catch (...) {
        if (out_n_reports)
            for (uint32_t s = 0; s < n; ++s) out_n_reports[s] = b_->ctxs[s]->n_reports;
        throw;
    }
    if (out_n_reports)
        for (uint32_t s = 0; s < n; ++s) out_n_reports[s] = b_->ctxs[s]->n_reports;
    GSS_REQUIRE(!overflow, GSS_ERR_REPORT_OVERFLOW,
                "a store's report segments overflowed (now grown); its counts are exact: test again");
    GSS_BATCH_END
}

extern "C" gss_status gss_batch_info(const gss_batch *b, double *last_ms, uint64_t *launches, uint64_t *captures,
                                     uint64_t *tiles) {
    if (!b) return GSS_ERR_INVALID_ARG;
    if (last_ms) *last_ms = b->last_ms;
    if (launches) *launches = b->launches;
    if (captures) *captures = b->captures;
    if (tiles) *tiles = b->total;
    return GSS_OK;
}
