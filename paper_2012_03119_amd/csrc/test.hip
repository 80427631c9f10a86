// The clause test (Sections 3.4-3.5) and its report compaction.
//
// Two forms of parallelism, as in Section 3.5: wavefront lanes work on different
// clauses, and each lane tests 64 assignment slots at once with 64-bit bitwise
// operations.  A clause is spread over LPC lanes, one 64-slot word per lane, so a
// wavefront covers T = 64 / LPC clauses and the W words of one plane row are read
// by adjacent lanes as one contiguous access.
//
// Falsified mode: the clause mask is the AND over its literals of the gathered
// plane words (the allFalse half of the bitwise trigger test of Section 3.4).
// Trigger mode (Definition 1): the same loop also carries the oneUndef word, which
// needs the row of the opposite literal as well (isSet = F-row | T-row).
//
// Early exit: after every group of gathers the wavefront votes; once no lane of
// any of its clauses has a live bit left, it stops reading literals.  Hot rows
// (the first `hot_rows` plane rows; variables are kept in code order inside a
// clause, so the first literals land there most often) can be staged in LDS.
//
// The kernel is persistent: each wavefront walks the tiles t = wave, wave + N, ...
// (N wavefronts in the grid) and prefetches the next tile's metadata and first
// literal block while it tests the current one.  Reports need no atomics: every
// wavefront owns one segment of the report buffer and appends its records there,
// at its running count + (records of lower lanes, from mbcnt).  A one-block
// finalize kernel turns the per-wavefront counts into totals and segment offsets;
// fetching stitches the segments into one list.  Counts beyond a segment's
// capacity are still counted, so the exact size needed is always known.
#include "gss_internal.h"

#include <algorithm>
#include <cstring>

namespace gss {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so that a
// contiguous range of logical workgroups (neighbouring tiles, sharing cache lines
// of the literal and metadata streams) runs on one XCD and its L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    constexpr uint32_t X = 8;
    const uint32_t x = b % X, i = b / X, q = nb / X, r = nb % X;
    return x * q + (x < r ? x : r) + i;
}

__device__ inline uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int LPC, int MODE, bool HOT>
__global__ __launch_bounds__(kTestWavesPerBlock * 64) void k_test(const BucketDesc *__restrict__ descs,
                                                                   const TestArgs a, uint32_t early_exit,
                                                                   uint32_t dense) {
    constexpr uint32_t T = 64 / LPC;             // clauses per wavefront (and per tile)
    constexpr uint32_t R = (T == 64) ? 4 : LPC;  // literal rows per block load
    constexpr uint32_t BL = (T == 64) ? R : 1;   // codes per lane per block load
    constexpr uint32_t U = R < 4 ? R : 4;        // gathers in flight per lane between votes
    extern __shared__ uint64_t lds_rows[];

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t W = a.W;
    if constexpr (HOT) {
        const uint32_t n = a.hot_rows * W;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) lds_rows[i] = a.planes[i];
        __syncthreads();
    }
    const uint32_t j = lane / LPC;  // clause of this lane within the tile
    const uint32_t w = lane % LPC;  // word of this lane
    const bool word_ok = w < W;
    const uint64_t act = word_ok ? a.active[w] : 0;
    const uint32_t waves_per_block = blockDim.x / 64;
    const uint32_t n_waves = gridDim.x * waves_per_block;
    const uint32_t wave = xcd_remap(blockIdx.x, gridDim.x) * waves_per_block + threadIdx.x / 64;
    gss_report *const seg = a.reports + (uint64_t)wave * a.seg_cap;
    uint32_t produced = 0;  // records of this wavefront (uniform)
    uint32_t bi = 0;        // bucket of the current tile; tiles are visited in increasing order

    auto fetch = [&](uint32_t code) -> uint64_t {
        if constexpr (HOT) {
            if (code < a.hot_rows) return lds_rows[code * W + w];
        }
        return a.planes[(uint64_t)code * W + w];
    };

    // wave-uniform description of a tile, plus this lane's metadata and first block
    struct Tile {
        const uint32_t *lits;
        uint32_t s_log2;
        uint2 meta;
        uint32_t blk[BL];
    };
    auto load_block = [&](const Tile &tl, uint32_t k, uint32_t *blk) {
        const uint32_t S = 1u << tl.s_log2;
        if constexpr (T == 64) {
#pragma unroll
            for (uint32_t u = 0; u < R; ++u) blk[u] = (k + u < S) ? tl.lits[(uint64_t)(k + u) * 64 + lane] : 0u;
        } else {
            const uint32_t row = k + lane / T;
            blk[0] = row < S ? tl.lits[(uint64_t)row * T + lane % T] : 0u;
        }
    };
    auto open_tile = [&](uint32_t t, Tile &tl) {
        while (bi + 1 < a.n_buckets && t >= descs[bi + 1].tile_begin) ++bi;
        const BucketDesc &d = descs[bi];
        const uint32_t tile = t - d.tile_begin;
        tl.s_log2 = d.stride_log2;
        tl.lits = d.lits + ((uint64_t)tile << d.stride_log2) * T;
        tl.meta = d.meta[(uint64_t)tile * T + j];
        load_block(tl, 0, tl.blk);
    };

    uint32_t t = wave;
    Tile cur;
    if (t < a.n_tiles) open_tile(t, cur);
    while (t < a.n_tiles) {
        const uint32_t tn = t + n_waves;
        Tile nxt{};
        if (tn < a.n_tiles) open_tile(tn, nxt);  // prefetch: loads in flight while this tile runs

        const uint32_t len = cur.meta.x;
        uint64_t af = (len && word_ok) ? act : 0;  // allFalse
        uint64_t ou = 0;                           // oneUndef (trigger mode)
        uint32_t blk[BL];
#pragma unroll
        for (uint32_t u = 0; u < BL; ++u) blk[u] = cur.blk[u];
        for (uint32_t k = 0;; k += R) {
            {
                const bool go = k < len && word_ok && (!early_exit || (af | ou) != 0);
                if (!__ballot(go)) break;
            }
            if (k) load_block(cur, k, blk);
            bool stop = false;
#pragma unroll
            for (uint32_t r = 0; r < R; r += U) {
                if (stop) continue;  // wave-uniform; keeps the loop unrollable
                uint64_t gf[U], gt[U];
#pragma unroll
                for (uint32_t u = 0; u < U; ++u) {
                    const uint32_t kk = k + r + u;
                    uint32_t code;
                    if constexpr (T == 64)
                        code = blk[r + u];
                    else
                        code = (uint32_t)__shfl((int)blk[0], (int)((r + u) * T + j), 64);
                    const bool live = kk < len && word_ok && (!early_exit || (af | ou) != 0);
                    gf[u] = ~0ull;
                    gt[u] = 0;
                    if (live) {
                        gf[u] = fetch(code);
                        if constexpr (MODE == 1) gt[u] = fetch(code ^ 1u);
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < U; ++u) {
                    if constexpr (MODE == 1) {
                        const uint64_t is_set = gf[u] | gt[u];
                        ou = (af & ~is_set) | (ou & gf[u]);
                    }
                    af &= gf[u];
                }
                if (early_exit) {
                    const bool more = (k + r + U) < len && (af | ou) != 0;
                    stop = !__ballot(more);
                }
            }
            if (stop) break;
        }

        const uint64_t res = af | ou;
        if (dense) {
            if (len && word_ok) a.dense[(uint64_t)cur.meta.y * W + w] = res;
        } else {
            const bool has = res != 0;
            const uint64_t bal = __ballot(has);
            if (has) {
                const uint32_t pos = produced + lanes_below(bal);
                if (pos < a.seg_cap) {
                    const u32x4 rec = {cur.meta.y, w, (uint32_t)res, (uint32_t)(res >> 32)};
                    __builtin_nontemporal_store(rec, reinterpret_cast<u32x4 *>(seg) + pos);
                }
            }
            produced += (uint32_t)__builtin_popcountll(bal);
        }
        t = tn;
        cur = nxt;
    }
    if (lane == 0) a.seg_counts[wave] = produced;
}

// One workgroup of 1024 threads: exclusive prefix of the records each segment
// kept (min(count, cap)) into offsets[0..n], and summary = {total count, largest
// count, records kept}.
__global__ __launch_bounds__(1024) void k_finalize(const uint32_t *counts, uint32_t n, uint32_t cap,
                                                    uint64_t *offsets, unsigned long long *summary) {
    __shared__ unsigned long long part[1024];
    __shared__ unsigned long long tot[1024];
    __shared__ unsigned int mx[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t lo = tid * per, hi = min(n, lo + per);
    unsigned long long kept = 0, all = 0;
    unsigned int m = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        kept += min(counts[i], cap);
        all += counts[i];
        m = max(m, counts[i]);
    }
    part[tid] = kept;
    tot[tid] = all;
    mx[tid] = m;
    __syncthreads();
    // inclusive Hillis-Steele scan of part[], reductions of tot[] and mx[]
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        unsigned long long p = tid >= off ? part[tid - off] : 0ull;
        unsigned long long q = (tid + off < 1024) ? tot[tid + off] : 0ull;
        unsigned int r = (tid + off < 1024) ? mx[tid + off] : 0u;
        __syncthreads();
        part[tid] += p;
        if ((tid & (2 * off - 1)) == 0) {
            tot[tid] += q;
            mx[tid] = max(mx[tid], r);
        }
        __syncthreads();
    }
    unsigned long long base = tid ? part[tid - 1] : 0ull;
    for (uint32_t i = lo; i < hi; ++i) {
        offsets[i] = base;
        base += min(counts[i], cap);
    }
    if (tid == 1023) offsets[n] = part[1023];
    if (tid == 0) {
        summary[0] = tot[0];
        summary[1] = mx[0];
        summary[2] = part[1023];
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

using KernelFn = void (*)(const BucketDesc *, const TestArgs, uint32_t, uint32_t);

template <int MODE, bool HOT>
static KernelFn pick_lpc(uint32_t lpc) {
    switch (lpc) {
    case 1: return k_test<1, MODE, HOT>;
    case 2: return k_test<2, MODE, HOT>;
    case 4: return k_test<4, MODE, HOT>;
    case 8: return k_test<8, MODE, HOT>;
    case 16: return k_test<16, MODE, HOT>;
    case 32: return k_test<32, MODE, HOT>;
    default: return k_test<64, MODE, HOT>;
    }
}

static KernelFn pick_kernel(uint32_t lpc, int mode, bool hot) {
    if (mode == 0) return hot ? pick_lpc<0, true>(lpc) : pick_lpc<0, false>(lpc);
    return hot ? pick_lpc<1, true>(lpc) : pick_lpc<1, false>(lpc);
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
    for (int b = 0; b < kMaxBuckets; ++b) {
        const Bucket &B = c.buckets[b];
        if (B.n_slots == 0 || B.n_dead == B.n_slots) continue;
        BucketDesc d{};
        d.lits = B.lits;
        d.meta = B.meta;
        d.stride_log2 = B.stride_log2;
        d.tile_begin = tiles;
        h[nb++] = d;
        tiles += (uint32_t)((B.n_slots + c.T - 1) / c.T);
    }
    a.n_buckets = nb;
    a.n_tiles = tiles;
    a.planes = c.planes;
    a.active = c.active;
    a.W = c.W;
    const bool hot = c.hot_rows > 0 && !(flags & GSS_TEST_NO_HOT);
    a.hot_rows = hot ? c.hot_rows : 0;
    a.reports = c.reports;
    a.seg_counts = c.seg_counts;
    a.seg_cap = c.seg_cap;
    a.dense = c.dense;
    if (nb) GSS_HIP(hipMemcpyAsync(c.d_desc, h, nb * sizeof(BucketDesc), hipMemcpyHostToDevice, c.stream));
    L.descs = (const BucketDesc *)c.d_desc;
    L.fn = pick_kernel(c.LPC, (flags & GSS_TEST_TRIGGER) ? 1 : 0, hot);
    uint64_t per_cu = kTestBlocksPerCU;
    if (hot) {
        L.lds = (size_t)a.hot_rows * c.W * 8;
        per_cu = std::max<uint64_t>(1, std::min<uint64_t>(per_cu, (160u * 1024u) / L.lds));
    }
    const uint64_t one_tile_each = (tiles + kTestWavesPerBlock - 1) / kTestWavesPerBlock;
    L.grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(one_tile_each, per_cu * c.n_cu));
    return L;
}

static void run(Ctx &c, const Launch &L, uint32_t flags) {
    GSS_HIP(hipEventRecord(c.ev_start, c.stream));
    hipLaunchKernelGGL(L.fn, dim3(L.grid), dim3(kTestWavesPerBlock * 64), L.lds, c.stream, L.descs, L.args,
                       (flags & GSS_TEST_NO_EARLY_EXIT) ? 0u : 1u, (flags & GSS_TEST_DENSE) ? 1u : 0u);
    GSS_HIP(hipGetLastError());
    GSS_HIP(hipEventRecord(c.ev_stop, c.stream));
    const uint32_t n_waves = L.grid * kTestWavesPerBlock;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, c.stream, c.seg_counts, n_waves, c.seg_cap, c.seg_offsets,
                       c.d_summary);
    GSS_HIP(hipGetLastError());
    GSS_HIP(hipMemcpyAsync(c.h_summary, c.d_summary, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    float ms = 0.f;
    GSS_HIP(hipEventElapsedTime(&ms, c.ev_start, c.ev_stop));
    c.stats.last_kernel_ms = ms;
    c.stats.total_kernel_ms += ms;
    c.stats.timed_launches++;
    c.stats.kernel_launches++;
    c.last_waves = n_waves;
}

}  // namespace gss

using namespace gss;

extern "C" gss_status gss_test(gss_ctx *ctx, uint32_t flags, uint64_t *out_n_reports) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    const uint32_t known = GSS_TEST_TRIGGER | GSS_TEST_NO_EARLY_EXIT | GSS_TEST_SORTED | GSS_TEST_DENSE |
                           GSS_TEST_NO_REGROW | GSS_TEST_NO_HOT;
    GSS_REQUIRE((flags & ~known) == 0, GSS_ERR_INVALID_ARG, "unknown gss_test flag");
    GSS_REQUIRE(!(flags & GSS_TEST_SORTED), GSS_ERR_INVALID_ARG, "GSS_TEST_SORTED is not supported by this build");
    if (out_n_reports) *out_n_reports = 0;
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
    }
    uint64_t act = 0;
    for (uint64_t x : c.h_active) act += __builtin_popcountll(x);
    uint64_t lits = 0;
    for (const auto &B : c.buckets) lits += B.n_lits;
    c.stats.last_pairs = c.live * act;
    c.stats.last_literals = lits;

    Launch L = prepare(c, flags);
    uint64_t n = 0, kept = 0;
    c.tested = false;
    if (L.args.n_tiles > 0) {
        run(c, L, flags);
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
                grown = true;
            } catch (const Error &e) {
                if (e.code != GSS_ERR_CAPACITY) throw;
            }
            if (grown) {
                c.stats.regrows++;
                L = prepare(c, flags);
                run(c, L, flags);
                n = c.h_summary[0];
                kept = c.h_summary[2];
            }
        }
    } else {
        c.last_waves = 0;
    }
    c.stats.tests_run++;
    c.tested = true;
    c.last_flags = flags;
    if (flags & GSS_TEST_DENSE) n = kept = 0;
    c.n_reports = n;
    c.n_kept = kept;
    c.stats.last_reports = n;
    if (out_n_reports) *out_n_reports = n;
    GSS_REQUIRE(kept == n, GSS_ERR_REPORT_OVERFLOW,
                "report segments of " + std::to_string(c.seg_cap) + " records kept " + std::to_string(kept) + " of " +
                    std::to_string(n) + " records");
    GSS_API_END
}

extern "C" gss_status gss_fetch_reports(gss_ctx *ctx, gss_report *out, uint64_t cap, uint64_t *out_n) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(c.tested, GSS_ERR_STATE, "no test has run yet");
    GSS_REQUIRE(out_n != nullptr, GSS_ERR_INVALID_ARG, "null argument");
    const uint64_t n = std::min(c.n_kept, cap);
    *out_n = 0;
    if (n) {
        GSS_REQUIRE(out != nullptr, GSS_ERR_INVALID_ARG, "null argument");
        const bool dev = is_device_pointer(out);
        gss_report *dst = dev ? out : (gss_report *)c.device_stage(n * sizeof(gss_report));
        const unsigned grid = std::max<uint32_t>(1, std::min<uint32_t>(c.last_waves, 65535));
        hipLaunchKernelGGL(k_stitch, dim3(grid), dim3(256), 0, c.stream, c.reports, c.seg_counts, c.seg_offsets,
                           c.seg_cap, c.last_waves, n, dst);
        GSS_HIP(hipGetLastError());
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
