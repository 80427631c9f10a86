// Device code of the single-store clause test: the persistent test kernel over
// one store's tiles, the finalize kernel that turns per-wavefront record counts
// into totals and segment offsets, the stitch that joins the segments, and the
// dense-mode row gather.  The per-tile work is the Tester of tester.h
// (Sections 3.4-3.5).  Host code lives in test.hip.
#pragma once

#include "tester.h"

namespace gss {

// Each wavefront walks the tiles t = wave, wave + N, ... (N wavefronts in the
// grid) and prefetches the next tile's metadata and first codes while it tests
// the current one.  WIDE: plane rows of more than 64 words (several chunks).
template <int LPC, int WPL, int MODE, bool HOT, bool AGG, bool WIDE = false>
__global__ __launch_bounds__(kTestWavesPerBlock * 64) void k_test(const BucketDesc *__restrict__ descs,
                                                                   const TestArgs a, uint32_t early_exit,
                                                                   uint32_t dense) {
    using Ts = Tester<LPC, WPL, MODE, HOT, AGG, WIDE>;
    extern __shared__ uint64_t lds_rows[];
    if constexpr (HOT) {
        const uint32_t n = a.hot_rows * Ts::RW;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) lds_rows[i] = a.planes[i];
        __syncthreads();
    }
    const uint32_t lane = threadIdx.x & 63;
    const Ts ts(lane, a.planes, a.active, a.W, a.hot_rows, lds_rows, a.sched_run, a.agg, a.aggu, a.G, a.chunk_elems,
                a.n_rows, a.sagg, a.saggu);
    const uint32_t waves_per_block = blockDim.x / 64;
    const uint32_t n_waves = gridDim.x * waves_per_block;
    // wave-uniform by construction; readfirstlane lets the compiler keep it in SGPRs
    const uint32_t wave = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * waves_per_block +
                                                         threadIdx.x / 64);
    gss_report *const seg = a.reports + (uint64_t)wave * a.seg_cap;
    const uint32_t seg_cap = a.seg_cap;
    uint64_t *const dense_out = dense ? a.dense : nullptr;
    uint32_t produced = 0;  // records of this wavefront (uniform)
    uint32_t bi = 0;
    Counts cnt;  // GSS_TEST_COUNT (uniform)
    cnt.on = a.wave_stats != nullptr;

    const uint32_t last = a.n_tiles - 1;
    uint32_t t = wave;
    typename Ts::Tile cur;
    ts.open(descs, a.n_buckets, bi, t < a.n_tiles ? t : last, cur);
    while (t < a.n_tiles) {
        const uint32_t tn = t + n_waves;
        typename Ts::Tile nxt;
        ts.open(descs, a.n_buckets, bi, tn < a.n_tiles ? tn : last, nxt);  // prefetch, unconditionally
        if constexpr (!WIDE) {
            produced = ts.run(cur, seg, seg_cap, produced, early_exit, dense_out, cnt);
        } else {
            // rows of more than 64 words: the tile is tested chunk by chunk, each
            // chunk's 4096 slots a super-group; with the aggregate pre-test, first
            // on the super-groups' aggregates, then only on the chunks where some
            // clause of the tile can still be falsified (or trigger)
            const uint64_t sup = AGG ? ts.super_mask(cur, a.gmask) : a.gmask;
            for (uint32_t g = 0; g < a.G; ++g)
                if (__ballot((sup >> g) & 1u))
                    produced = ts.run(cur, seg, seg_cap, produced, early_exit, dense_out, cnt, g, sup);
        }
        t = tn;
        cur = nxt;
    }
    if (lane == 0) {
        a.seg_counts[wave] = produced;
        if (a.wave_stats) {
            a.wave_stats[2 * wave] = cnt.gathers;
            a.wave_stats[2 * wave + 1] = cnt.settled;
        }
    }
}

// Scheduled test: the wavefronts walk chunks of T listed slots (the clauses this
// run tests, k_sched_list) instead of tiles, so that clauses sitting out the run
// take no lanes.  Otherwise as k_test (no rows of more than 64 words).
template <int LPC, int WPL, int MODE, bool HOT, bool AGG>
__global__ __launch_bounds__(kTestWavesPerBlock * 64) void k_test_list(const BucketDesc *__restrict__ descs,
                                                                        const TestArgs a, uint32_t early_exit,
                                                                        uint32_t dense) {
    using Ts = Tester<LPC, WPL, MODE, HOT, AGG>;
    extern __shared__ uint64_t lds_rows[];
    __shared__ uint32_t chunk_begin[kMaxBuckets + 1], count[kMaxBuckets];
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t b = 0; b < a.n_buckets; ++b) {
            count[b] = *descs[b].list_count;
            chunk_begin[b] = acc;
            acc += (count[b] + Ts::T - 1) / Ts::T;
        }
        chunk_begin[a.n_buckets] = acc;
    }
    if constexpr (HOT) {
        const uint32_t n = a.hot_rows * Ts::RW;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) lds_rows[i] = a.planes[i];
    }
    __syncthreads();
    constexpr uint32_t t_log2 = ilog2<Ts::T>();
    const uint32_t lane = threadIdx.x & 63, j = lane / LPC;
    const Ts ts(lane, a.planes, a.active, a.W, a.hot_rows, lds_rows, 0u, a.agg, a.aggu);
    const uint32_t waves_per_block = blockDim.x / 64;
    const uint32_t n_waves = gridDim.x * waves_per_block;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * waves_per_block +
                                                         threadIdx.x / 64);
    gss_report *const seg = a.reports + (uint64_t)wave * a.seg_cap;
    uint64_t *const dense_out = dense ? a.dense : nullptr;
    uint32_t produced = 0;
    uint32_t bi = 0;
    Counts cnt;
    cnt.on = a.wave_stats != nullptr;
    const uint32_t total = chunk_begin[a.n_buckets];
    uint32_t c = wave;
    TileRef cur;
    if (c < total) open_listed(descs, a.n_buckets, bi, c, chunk_begin, count, j, t_log2, cur);
    while (c < total) {
        const uint32_t cn = c + n_waves;
        TileRef nxt = cur;
        if (cn < total) open_listed(descs, a.n_buckets, bi, cn, chunk_begin, count, j, t_log2, nxt);
        produced = ts.run(cur, seg, a.seg_cap, produced, early_exit, dense_out, cnt);
        c = cn;
        cur = nxt;
    }
    if (lane == 0) {
        a.seg_counts[wave] = produced;
        if (a.wave_stats) {
            a.wave_stats[2 * wave] = cnt.gathers;
            a.wave_stats[2 * wave + 1] = cnt.settled;
        }
    }
}

// The slots that a scheduled run tests (alive, and not a low-priority clause off
// its turn: (run + id) % 4 != 0), one list per length class, built by one launch
// over every class: workgroup g takes kSchedSlots consecutive slots of the class
// whose block range holds g, 32 per thread (one word of schedule bits; their 256
// bytes of metadata are loaded at once), and claims its range of the class's
// list with one atomic on its count (one per 8192 slots: the counters see few
// atomics).  In slot order within a workgroup: the workgroup's part of the list is
// assembled in LDS and written out in whole lines.
constexpr uint32_t kSchedThreads = 256, kSchedSlots = 32 * kSchedThreads;

struct SchedClass {
    const uint2 *meta;
    const uint32_t *low;  // one bit per slot
    uint32_t *list;
    uint32_t *count;
    uint32_t n_slots;
    uint32_t block_begin;  // first workgroup of the class
};

struct SchedTable {
    SchedClass cls[kMaxBuckets];
    uint32_t n;
};

__global__ __launch_bounds__(kSchedThreads) void k_sched_list(const SchedTable tab, uint32_t run) {
    __shared__ uint32_t wave_sum[kSchedThreads / 64];
    __shared__ uint32_t base, total;
    __shared__ uint32_t stage[kSchedSlots];
    uint32_t b = 0;
    while (b + 1 < tab.n && blockIdx.x >= tab.cls[b + 1].block_begin) ++b;
    const SchedClass &C = tab.cls[b];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t s0 = (blockIdx.x - C.block_begin) * kSchedSlots + 32u * t;  // one low word
    uint32_t flags = 0;
    if (s0 < C.n_slots) {
        const uint32_t lw = C.low[s0 >> 5];
        if (s0 + 32 <= C.n_slots) {
            // 32 slots' metadata in sixteen 16-byte loads, all in flight together
            const uint4 *mp = reinterpret_cast<const uint4 *>(C.meta + s0);
            uint4 q[16];
#pragma unroll
            for (uint32_t k = 0; k < 16; ++k) q[k] = mp[k];
#pragma unroll
            for (uint32_t k = 0; k < 16; ++k) {
                const bool t0 = q[k].x != 0 && !(((lw >> (2 * k)) & 1u) && ((run + q[k].y) & 3u) != 0);
                const bool t1 = q[k].z != 0 && !(((lw >> (2 * k + 1)) & 1u) && ((run + q[k].w) & 3u) != 0);
                flags |= (t0 ? 1u : 0u) << (2 * k) | (t1 ? 1u : 0u) << (2 * k + 1);
            }
        } else {
            for (uint32_t k = 0; s0 + k < C.n_slots; ++k) {
                const uint2 m = C.meta[s0 + k];
                const bool tested = m.x != 0 && !(((lw >> k) & 1u) && ((run + m.y) & 3u) != 0);
                flags |= (tested ? 1u : 0u) << k;
            }
        }
    }
    const uint32_t mine = __builtin_popcount(flags);
    uint32_t x = mine;  // inclusive scan: within the wavefront, then across
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wave_sum[wave] = x;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (uint32_t w = 0; w < kSchedThreads / 64; ++w) {
            const uint32_t v = wave_sum[w];
            wave_sum[w] = acc;
            acc += v;
        }
        base = acc ? atomicAdd(C.count, acc) : 0u;
        total = acc;
    }
    __syncthreads();
    uint32_t pos = wave_sum[wave] + x - mine;  // below kSchedSlots: at most 32 per thread
    for (uint32_t f = flags; f; f &= f - 1) stage[pos++] = s0 + (uint32_t)__builtin_ctz(f);
    __syncthreads();
    for (uint32_t i = t; i < total; i += kSchedThreads) C.list[base + i] = stage[i];
}

// summary[3] receives the verdict of the asynchronous updates queued before the
// test.  The summary is also written straight into pinned host memory, followed by
// the test's serial number: the host sees the test complete when the serial
// arrives, with no copy or event queued behind the kernel.
__global__ __launch_bounds__(1024) void k_finalize(const uint32_t *counts, uint32_t n, uint32_t cap,
                                                    uint64_t *offsets, unsigned long long *summary,
                                                    const uint32_t *deferred, unsigned long long *host_summary,
                                                    unsigned long long serial) {
    finalize_segments(counts, n, cap, offsets, summary);
    if (threadIdx.x == 0) {  // the thread that wrote summary[0..2]
        summary[3] = *deferred;
#pragma unroll
        for (int k = 0; k < 4; ++k) host_summary[k] = summary[k];
        __threadfence_system();  // the summary reaches the host before the serial
        host_summary[4] = serial;  // made visible by the kernel's end
    }
}

// Copies the kept records of every segment into one list (segment order), the
// first `limit` records only.  One workgroup per segment.
__global__ void k_stitch(const gss_report *reports, const uint32_t *counts, const uint64_t *offsets, uint32_t seg_cap,
                         uint32_t n_segments, uint64_t limit, gss_report *out) {
    for (uint32_t s = blockIdx.x; s < n_segments; s += gridDim.x) {
        const uint32_t n = min(counts[s], seg_cap);
        const uint64_t base = offsets[s];
        const u32x4 *src = reinterpret_cast<const u32x4 *>(reports) + (uint64_t)s * seg_cap;
        u32x4 *dst = reinterpret_cast<u32x4 *>(out);
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
            if (base + i < limit) dst[base + i] = src[i];
    }
}

// Dense-mode fetch: out[i] = dense row of ids[i], or zeros when ids[i] == kDeadId.
__global__ void k_gather_rows(uint64_t *out, const uint64_t *dense, const uint32_t *ids, uint32_t n, uint32_t W) {
    const uint64_t total = (uint64_t)n * W;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t id = ids[x / W];
        out[x] = id == kDeadId ? 0ull : dense[(uint64_t)id * W + x % W];
    }
}

}  // namespace gss
