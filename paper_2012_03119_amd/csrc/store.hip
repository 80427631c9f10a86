// The clause store: length-bucketed SoA tiles of literal codes, with insertion,
// deletion and compaction.
//
// Layout (per length class b, stride S = 2^b codes, S >= 4): slot s holds its
// clause at lits[s * S .. s * S + S), padded with code 0, so the test kernel reads
// four codes per 16-byte load; a tile is T consecutive slots (T = 64 /
// lanes-per-clause), one wavefront's share.  A clause's smallest code (its lead)
// comes first and the clauses of a batch are laid out by lead, so neighbouring
// clauses start on the same plane row; the order of the other codes does not
// change the result (a full sort measured no faster and costs O(L log L)).
#include "gss_internal.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <thread>

namespace gss {

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------

// Appends one segment of new clauses to a bucket: thread per literal.  Clause i
// of the segment goes to slot slot0 + i; its codes are codes[coff[i] .. coff[i+1]).
__global__ void k_append_lits(uint32_t *lits, uint32_t stride_log2, uint32_t tile_log2, uint64_t slot0,
                              const uint32_t *codes, const uint64_t *coff, uint32_t n_clauses, uint64_t n_lits) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n_lits; x += (uint64_t)gridDim.x * blockDim.x) {
        // clause owning literal x: last i with coff[i] <= x
        uint32_t lo = 0, hi = n_clauses;  // coff[lo] <= x < coff[hi]
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (coff[mid] <= x) lo = mid; else hi = mid;
        }
        const uint64_t k = x - coff[lo];
        lits[code_index(slot0 + lo, (uint32_t)k, stride_log2, tile_log2)] = codes[x];
    }
}

__global__ void k_append_meta(uint2 *meta, uint64_t slot0, const uint64_t *coff, const uint32_t *new_ids,
                              uint32_t n_clauses) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_clauses; i += gridDim.x * blockDim.x)
        meta[slot0 + i] = make_uint2((uint32_t)(coff[i + 1] - coff[i]), new_ids[i]);
}

// Marks slots removed: length 0 (the test skips the slot without reading a literal).
__global__ void k_tombstone(uint2 *meta, const uint64_t *slots, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        meta[slots[i]] = make_uint2(0u, kDeadId);
}

// Compaction: new slot s takes the clause of old slot old_slot[s]; thread per
// (new slot, literal row).
__global__ void k_compact_lits(uint32_t *dst, const uint32_t *src, uint32_t stride_log2, uint32_t tile_log2,
                               const uint64_t *old_slot, uint64_t n_new) {
    const uint64_t S = 1ull << stride_log2;
    const uint64_t total = n_new * S;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = x >> stride_log2;
        const uint32_t k = (uint32_t)(x & (S - 1));
        dst[code_index(s, k, stride_log2, tile_log2)] = src[code_index(old_slot[s], k, stride_log2, tile_log2)];
    }
}

__global__ void k_compact_meta(uint2 *dmeta, const uint2 *smeta, const uint64_t *old_slot, uint64_t n_new) {
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < n_new; s += (uint64_t)gridDim.x * blockDim.x)
        dmeta[s] = smeta[old_slot[s]];
}

// Compaction map, K7 (a prefix sum over the live flags, length != 0): slot s of a
// class is live when its length is nonzero; block b covers slots [1024 b, 1024 b
// + 1024), four per thread.  First the live count of each block; then, after an
// exclusive scan of the counts, every live slot's new place: the number of live
// slots before it.  The map is in slot order, so the host mirror follows it
// without reading it back.
__global__ __launch_bounds__(256) void k_live_counts(const uint2 *meta, uint64_t n_slots, uint32_t *block_counts) {
    __shared__ uint32_t part[4];
    const uint64_t s0 = (uint64_t)blockIdx.x * 1024 + 4ull * threadIdx.x;
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) mine += (s0 + k < n_slots && meta[s0 + k].x != 0) ? 1u : 0u;
    for (uint32_t off = 32; off; off >>= 1) mine += __shfl_xor(mine, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x / 64] = mine;
    __syncthreads();
    if (threadIdx.x == 0) block_counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// old_slot holds n_new entries (the host's live count; writes past it are dropped).
__global__ __launch_bounds__(256) void k_live_place(const uint2 *meta, uint64_t n_slots, const uint32_t *block_base,
                                                    uint64_t *old_slot, uint64_t n_new) {
    __shared__ uint32_t pre[256];
    const uint32_t t = threadIdx.x;
    const uint64_t s0 = (uint64_t)blockIdx.x * 1024 + 4ull * t;
    uint32_t flags = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) flags |= (s0 + k < n_slots && meta[s0 + k].x != 0 ? 1u : 0u) << k;
    const uint32_t mine = __builtin_popcount(flags);
    pre[t] = mine;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {  // inclusive scan
        const uint32_t v = t >= off ? pre[t - off] : 0u;
        __syncthreads();
        pre[t] += v;
        __syncthreads();
    }
    uint64_t pos = (uint64_t)block_base[blockIdx.x] + pre[t] - mine;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
        if ((flags >> k) & 1u) {
            if (pos < n_new) old_slot[pos] = s0 + k;
            ++pos;
        }
}

static unsigned grid_for(uint64_t n, unsigned block = 256) {
    uint64_t g = (n + block - 1) / block;
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, 16384));
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

static uint64_t bucket_bytes(uint64_t cap_slots, uint32_t stride_log2) {
    return cap_slots * ((4ull << stride_log2) + 8ull) + 2 * 256;
}

static uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

// Runs fn(begin, end) over [0, n) split across host threads when the work
// (weight: literals) is large enough to pay for them.
template <typename F>
static void host_parallel(uint64_t n, uint64_t weight, F fn) {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const unsigned k = (unsigned)std::min<uint64_t>({hw, n, weight / (1u << 20) + 1});
    if (k <= 1) {
        fn((uint64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(k);
    for (unsigned t = 0; t < k; ++t) th.emplace_back(fn, n * t / k, n * (t + 1) / k);
    for (auto &x : th) x.join();
}

static uint32_t tile_log2(const Ctx &c) {
    uint32_t l = 0;
    while ((1u << l) < c.T) ++l;
    return l;
}

// Fills a meta array with empty slots (length 0, dead id).
static void fill_meta(Ctx &c, uint2 *meta, uint64_t n) {
    launch_fill_u64(c, reinterpret_cast<uint64_t *>(meta), n, (uint64_t)kDeadId << 32);
}

// Allocates the arrays of a bucket with capacity cap (tail empty: length 0, codes
// 0) and copies the used prefix of the old arrays.
static void grow_bucket(Ctx &c, Bucket &b, uint64_t cap) {
    const uint64_t S = 1ull << b.stride_log2;
    uint32_t *lits = (uint32_t *)c.dalloc(cap * S * 4);
    uint2 *meta = (uint2 *)c.dalloc(cap * 8);
    launch_fill_u32(c, lits, cap * S, 0);
    fill_meta(c, meta, cap);
    if (b.n_slots) {  // whole tiles: a tile's codes are interleaved (code_index)
        const uint64_t used = (b.n_slots + c.T - 1) / c.T * c.T;
        GSS_HIP(hipMemcpyAsync(lits, b.lits, used * S * 4, hipMemcpyDeviceToDevice, c.stream));
        GSS_HIP(hipMemcpyAsync(meta, b.meta, b.n_slots * 8, hipMemcpyDeviceToDevice, c.stream));
    }
    // the old arrays may still be read by a test in flight and by the copies just
    // queued: freed once the next test completes, without waiting here
    c.defer_free(b.lits);
    c.defer_free(b.meta);
    b.lits = lits;
    b.meta = meta;
    b.cap_slots = cap;
}

// Rewrites bucket b keeping only its live clauses, in slot order.  Returns false
// (and changes nothing) when the HBM budget has no room for the new arrays.
static bool compact_bucket(Ctx &c, int bi) {
    Bucket &b = c.buckets[bi];
    const uint64_t n_new = b.n_slots - b.n_dead;
    const uint64_t S = 1ull << b.stride_log2;
    const uint64_t cap = round_up(std::max<uint64_t>(n_new + n_new / 4, 256), c.T);
    const uint64_t n_blocks = (b.n_slots + 1023) / 1024;
    const uint64_t need = cap * S * 4 + cap * 8 + n_new * 8 + n_blocks * 4 + 4096;
    if (!c.fits(need)) return false;

    uint32_t *lits = (uint32_t *)c.dalloc(cap * S * 4);
    uint2 *meta = (uint2 *)c.dalloc(cap * 8);
    // the map (old slot of each new slot), then the per-block live counts
    char *mbuf = (char *)c.dalloc(round_up(std::max<uint64_t>(n_new, 1) * 8, 256) + n_blocks * 4);
    uint64_t *dmap = (uint64_t *)mbuf;
    uint32_t *block_counts = (uint32_t *)(mbuf + round_up(std::max<uint64_t>(n_new, 1) * 8, 256));
    launch_fill_u32(c, lits, cap * S, 0);
    fill_meta(c, meta, cap);
    if (n_new) {
        // the map is built on the device from the lengths (the removals are queued
        // before it on the same stream)
        hipLaunchKernelGGL(k_live_counts, dim3((unsigned)n_blocks), dim3(256), 0, c.stream, b.meta, b.n_slots,
                           block_counts);
        GSS_HIP(hipGetLastError());
        launch_scan_u32(c, block_counts, n_blocks);
        hipLaunchKernelGGL(k_live_place, dim3((unsigned)n_blocks), dim3(256), 0, c.stream, b.meta, b.n_slots,
                           block_counts, dmap, n_new);
        GSS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_compact_lits, dim3(grid_for(n_new * S)), dim3(256), 0, c.stream, lits, b.lits,
                           b.stride_log2, tile_log2(c), dmap, n_new);
        GSS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_compact_meta, dim3(grid_for(n_new)), dim3(256), 0, c.stream, meta, b.meta, dmap, n_new);
        GSS_HIP(hipGetLastError());
    }
    c.defer_free(mbuf);  // read by the compaction kernels just queued
    c.defer_free(b.lits);
    c.defer_free(b.meta);
    b.lits = lits;
    b.meta = meta;
    b.cap_slots = cap;

    // the host mirror, in the same order: live slots keep their relative order
    std::vector<uint32_t> h_ids(n_new), h_len(n_new);
    uint64_t s = 0;
    for (uint64_t o = 0; o < b.n_slots; ++o) {
        const uint32_t id = b.h_ids[o];
        if (id == kDeadId) continue;
        GSS_REQUIRE(s < n_new, GSS_ERR_DEVICE, "store mirror holds more live slots than counted");
        h_ids[s] = id;
        h_len[s] = b.h_len[o];
        c.id_loc[id] = ((uint64_t)bi << 40) | s;
        ++s;
    }
    GSS_REQUIRE(s == n_new, GSS_ERR_DEVICE, "store mirror holds fewer live slots than counted");
    b.h_ids.swap(h_ids);
    b.h_len.swap(h_len);
    b.n_slots = n_new;
    b.n_dead = 0;
    c.stats.compactions++;
    return true;
}

// ---- ingest, part 1: validation and encoding (no context state; any thread)
void prepare_clauses(int64_t num_vars, const int32_t *lits, const uint64_t *offsets, uint32_t n, Prepared &p,
                     const uint32_t *perm) {
    p.clear();
    if (n == 0) return;
    GSS_REQUIRE(lits && offsets, GSS_ERR_INVALID_ARG, "null argument");
    p.cls.resize(n);
    p.lead.resize(n);
    p.offs.resize((size_t)n + 1);
    p.offs[0] = 0;
    for (uint32_t i = 0; i < n; ++i) {
        GSS_REQUIRE(offsets[i + 1] >= offsets[i], GSS_ERR_INVALID_ARG, "offsets must be non-decreasing");
        const uint64_t L = offsets[i + 1] - offsets[i];
        GSS_REQUIRE(L >= 1, GSS_ERR_INVALID_ARG, "empty clause at index " + std::to_string(i));
        GSS_REQUIRE(L <= kMaxClauseLen, GSS_ERR_INVALID_ARG,
                    "clause longer than 65536 literals at index " + std::to_string(i));
        p.cls[i] = (uint8_t)length_class((uint32_t)L);
        p.offs[i + 1] = p.offs[i] + L;
    }
    p.codes.resize(p.offs[n]);
    // literals in range; codes with the lead (smallest) first; the first bad clause wins
    uint64_t first_bad = ~0ull;
    std::mutex mu;
    host_parallel(n, p.offs[n], [&](uint64_t b, uint64_t e) {
        for (uint64_t i = b; i < e; ++i) {
            const uint64_t L = offsets[i + 1] - offsets[i];
            uint32_t *dst = p.codes.data() + p.offs[i];
            bool ok = true;
            for (uint64_t k = 0; k < L; ++k) {
                const int64_t l = lits[offsets[i] + k];
                const int64_t v = l < 0 ? -l : l;
                ok &= v >= 1 && v <= num_vars;
                dst[k] = (perm && ok) ? 2u * perm[v] + (l < 0 ? 1u : 0u) : lit_code((int32_t)l);
            }
            if (!ok) {
                std::lock_guard<std::mutex> g(mu);
                first_bad = std::min<uint64_t>(first_bad, i);
                return;
            }
            std::nth_element(dst, dst, dst + L);
            p.lead[i] = dst[0];
        }
    });
    if (first_bad != ~0ull) {
        const uint64_t i = first_bad;
        for (uint64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            const int64_t l = lits[k];
            const int64_t v = l < 0 ? -l : l;
            GSS_REQUIRE(v >= 1 && v <= num_vars, GSS_ERR_BAD_LITERAL,
                        "literal " + std::to_string(l) + " of clause " + std::to_string(i) + " is 0 or beyond num_vars");
        }
    }
}

void Prepared::append(const Prepared &o) {
    const uint64_t base = codes.size();
    codes.insert(codes.end(), o.codes.begin(), o.codes.end());
    for (size_t i = 1; i < o.offs.size(); ++i) offs.push_back(base + o.offs[i]);
    lead.insert(lead.end(), o.lead.begin(), o.lead.end());
    cls.insert(cls.end(), o.cls.begin(), o.cls.end());
}

// ---- ingest, part 2: ids, order, growth and upload
// Appends one chunk staged on the device at d: codes | coff[m+1] | ids[m].
static void launch_append(Ctx &c, Bucket &B, uint64_t slot0, const char *d, size_t codes_bytes, size_t coff_bytes,
                          uint32_t m, uint64_t nl) {
    const uint32_t *dcodes = (const uint32_t *)d;
    const uint64_t *dcoff = (const uint64_t *)(d + codes_bytes);
    const uint32_t *dids = (const uint32_t *)(d + codes_bytes + coff_bytes);
    hipLaunchKernelGGL(k_append_lits, dim3(grid_for(nl)), dim3(256), 0, c.stream, B.lits, B.stride_log2, tile_log2(c), slot0, dcodes,
                       dcoff, m, nl);
    GSS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_append_meta, dim3(grid_for(m)), dim3(256), 0, c.stream, B.meta, slot0, dcoff, dids, m);
    GSS_HIP(hipGetLastError());
}

void commit_clauses(Ctx &c, const Prepared &p, uint32_t *out_ids) {
    const uint32_t n = p.size();
    if (n == 0) return;
    c.mutations++;  // a test in flight no longer sees the current state
    const uint64_t next = c.id_loc.size();
    GSS_REQUIRE(next + n < (uint64_t)kDeadId, GSS_ERR_CAPACITY, "clause id space exhausted");
    const std::vector<uint8_t> &cls = p.cls;
    const std::vector<uint32_t> &lead = p.lead;
    const std::vector<uint64_t> &offsets = p.offs;
    uint64_t add[kMaxBuckets] = {0};
    for (uint32_t i = 0; i < n; ++i) add[cls[i]]++;
    // ---- order the batch by bucket, and inside a bucket by lead code: clauses a
    //      wavefront (and an XCD) tests at the same time then share the plane row
    //      of their first literal, the one every clause reads in full.  The lead
    //      is the smallest of about S codes out of 2 V, so two clauses of a class
    //      share it with probability about S / 4V: a class that adds fewer than
    //      V / 4S clauses (the small batches of a served store) would share almost
    //      none, and keeps the arrival order.  Then cut the batch into upload
    //      chunks, each a run of clauses of one bucket; stage buffers are sized
    //      for the largest chunk.
    std::vector<uint32_t> order(n);
    {
        uint64_t pos[kMaxBuckets + 1] = {0};
        for (int b = 0; b < kMaxBuckets; ++b) pos[b + 1] = pos[b] + add[b];
        uint64_t start[kMaxBuckets + 1];
        std::copy(pos, pos + kMaxBuckets + 1, start);
        for (uint32_t i = 0; i < n; ++i) order[pos[cls[i]]++] = i;
        for (int b = 0; b < kMaxBuckets; ++b)
            if ((add[b] << c.buckets[b].stride_log2 << 2) >= (uint64_t)c.cfg.num_vars)
                std::stable_sort(order.begin() + start[b], order.begin() + start[b + 1],
                                 [&](uint32_t x, uint32_t y) { return lead[x] < lead[y]; });
    }
    const uint64_t kChunkLits = 1ull << 24, kChunkClauses = 1ull << 21;
    std::vector<uint32_t> cuts{0};
    std::vector<uint64_t> chunk_lits;
    size_t stage_bytes = 0;
    {
        uint32_t a = 0;
        while (a < n) {
            const int b = cls[order[a]];
            uint32_t q = a;
            uint64_t nl = 0;
            while (q < n && cls[order[q]] == b && (q - a) < kChunkClauses) {
                const uint32_t i = order[q];
                const uint64_t L = offsets[i + 1] - offsets[i];
                if (q > a && nl + L > kChunkLits) break;
                nl += L;
                ++q;
            }
            cuts.push_back(q);
            chunk_lits.push_back(nl);
            stage_bytes = std::max<size_t>(stage_bytes, round_up(nl * 4, 256) + round_up((uint64_t)(q - a + 1) * 8, 256) +
                                                            round_up((uint64_t)(q - a) * 4, 256));
            a = q;
        }
    }
    // a batch of up to 64 MiB goes through one slot of the upload ring, every chunk
    // after the previous one (no waiting for queued tests); a larger one uses the
    // bulk staging, one chunk at a time
    size_t ring_bytes = 0;
    for (size_t ch = 0; ch + 1 < cuts.size(); ++ch) {
        const uint64_t m = cuts[ch + 1] - cuts[ch];
        ring_bytes += round_up(chunk_lits[ch] * 4, 256) + round_up((m + 1) * 8, 256) + round_up(m * 4, 256);
    }
    const bool ring = ring_bytes <= (64u << 20);
    Ctx::Staged rs{nullptr, nullptr, -1, nullptr};
    size_t ring_off = 0;
    struct ChunkLaunch {
        int b;
        uint64_t slot0, nl;
        uint32_t m;
        size_t off, codes_bytes, coff_bytes;
    };
    std::vector<ChunkLaunch> launches;
    if (ring) {
        rs = c.stage_upload(ring_bytes);  // may raise CAPACITY; nothing has changed yet
    } else {
        c.device_stage(stage_bytes);
        c.host_stage(stage_bytes);
    }

    // the priority state of the new ids first: its growth may fail on the budget
    priority_reserve(c, next + n);

    // ---- capacity: every bucket that must grow, checked against the budget up front
    uint64_t new_cap[kMaxBuckets] = {0};
    uint64_t grow_bytes = 0;
    for (int b = 0; b < kMaxBuckets; ++b) {
        Bucket &B = c.buckets[b];
        if (!add[b] || B.n_slots + add[b] <= B.cap_slots) continue;
        const uint64_t S = 1ull << B.stride_log2;
        const uint64_t min_slots = std::max<uint64_t>(c.T, std::min<uint64_t>(256, (1ull << 20) / S));
        uint64_t want = std::max<uint64_t>({B.n_slots + add[b], B.cap_slots + B.cap_slots / 2, min_slots});
        new_cap[b] = round_up(want, c.T);
        // the test kernel addresses a class's codes with 32-bit byte offsets
        if ((new_cap[b] << B.stride_log2 << 2) >= (1ull << 32))
            new_cap[b] = std::max<uint64_t>(B.n_slots + add[b], ((1ull << 30) >> B.stride_log2) / c.T * c.T - c.T);
        GSS_REQUIRE((new_cap[b] << B.stride_log2 << 2) < (1ull << 32) && new_cap[b] >= B.n_slots + add[b],
                    GSS_ERR_CAPACITY, "length class " + std::to_string(1u << B.stride_log2) + " would exceed 4 GiB of codes");
        grow_bytes += bucket_bytes(new_cap[b], B.stride_log2);
    }
    GSS_REQUIRE(c.fits(grow_bytes), GSS_ERR_CAPACITY, "HBM budget exhausted by the clause store");
    for (int b = 0; b < kMaxBuckets; ++b)
        if (new_cap[b]) grow_bucket(c, c.buckets[b], new_cap[b]);

    for (uint32_t i = 0; i < n; ++i) out_ids[i] = (uint32_t)(next + i);

    // ---- upload chunk by chunk
    uint64_t slot_cursor[kMaxBuckets];
    for (int b = 0; b < kMaxBuckets; ++b) {
        slot_cursor[b] = c.buckets[b].n_slots;
        c.buckets[b].h_ids.resize(c.buckets[b].n_slots + add[b], kDeadId);
        c.buckets[b].h_len.resize(c.buckets[b].n_slots + add[b], 0);
    }
    c.id_loc.resize(next + n, kNoLoc);

    for (size_t ch = 0; ch + 1 < cuts.size(); ++ch) {
        const uint32_t q0 = cuts[ch], q = cuts[ch + 1];
        const uint64_t nl = chunk_lits[ch];
        const int b = cls[order[q0]];
        Bucket &B = c.buckets[b];
        const uint32_t m = q - q0;
        // host staging: codes | coff[m+1] | ids[m]
        const size_t codes_bytes = round_up(nl * 4, 256);
        const size_t coff_bytes = round_up((uint64_t)(m + 1) * 8, 256);
        const size_t ids_bytes = round_up((uint64_t)m * 4, 256);
        const size_t bytes = codes_bytes + coff_bytes + ids_bytes;
        char *h = ring ? rs.h + ring_off : (char *)c.host_stage(bytes);
        char *d = ring ? rs.d + ring_off : (char *)c.device_stage(bytes);
        uint32_t *hcodes = (uint32_t *)h;
        uint64_t *hcoff = (uint64_t *)(h + codes_bytes);
        uint32_t *hids = (uint32_t *)(h + codes_bytes + coff_bytes);
        uint64_t off = 0;
        const uint64_t slot0 = slot_cursor[b];
        for (uint32_t r = 0; r < m; ++r) {
            const uint32_t i = order[q0 + r];
            const uint64_t L = offsets[i + 1] - offsets[i];
            hcoff[r] = off;
            off += L;
            const uint32_t id = (uint32_t)(next + i);
            hids[r] = id;
            const uint64_t slot = slot0 + r;
            c.id_loc[id] = ((uint64_t)b << 40) | slot;
            B.h_ids[slot] = id;
            B.h_len[slot] = (uint32_t)L;
        }
        hcoff[m] = off;
        for (uint32_t r = 0; r < m; ++r) {  // the prepared codes, in slot order
            const uint32_t i = order[q0 + r];
            std::memcpy(hcodes + hcoff[r], p.codes.data() + offsets[i], (offsets[i + 1] - offsets[i]) * 4);
        }
        if (ring) {  // launched once the whole slot is on the device
            launches.push_back({b, slot0, nl, m, ring_off, codes_bytes, coff_bytes});
            ring_off += bytes;
        } else {
            GSS_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c.stream));
            launch_append(c, B, slot0, d, codes_bytes, coff_bytes, m, nl);
            c.stage_release();  // the next chunk's host_stage waits for this one
        }
        slot_cursor[b] += m;
        B.n_slots = slot_cursor[b];
        B.n_lits += nl;
    }
    if (ring) {
        copy_in(c, rs.d, rs.hd, ring_off);
        for (const ChunkLaunch &L : launches)
            launch_append(c, c.buckets[L.b], L.slot0, rs.d + L.off, L.codes_bytes, L.coff_bytes, L.m, L.nl);
        c.stage_done(rs);
    }
    c.live += n;
    c.version++;
    priority_added(c, next, n, offsets.data());
}

}  // namespace gss

using namespace gss;

extern "C" gss_status gss_add_clauses(gss_ctx *ctx, const int32_t *lits, const uint64_t *offsets, uint32_t n,
                                      uint32_t *out_ids) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;
    Ctx &c = *c_;
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(lits && offsets && out_ids, GSS_ERR_INVALID_ARG, "null argument");
    Prepared p;
    prepare_clauses(c.cfg.num_vars, lits, offsets, n, p, c.perm());
    commit_clauses(c, p, out_ids);
    GSS_API_END
}

extern "C" gss_status gss_remove_clauses(gss_ctx *ctx, const uint32_t *ids, uint32_t n) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;  // a test in flight no longer sees the current state
    Ctx &c = *c_;
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(ids != nullptr, GSS_ERR_INVALID_ARG, "null argument");
    // ---- validate: issued, live, and each id once
    std::vector<uint32_t> sorted(ids, ids + n);
    std::sort(sorted.begin(), sorted.end());
    for (uint32_t i = 0; i < n; ++i) {
        GSS_REQUIRE(sorted[i] < c.id_loc.size() && c.id_loc[sorted[i]] != kNoLoc, GSS_ERR_UNKNOWN_ID,
                    "clause id " + std::to_string(sorted[i]) + " is not live");
        GSS_REQUIRE(i == 0 || sorted[i] != sorted[i - 1], GSS_ERR_UNKNOWN_ID,
                    "clause id " + std::to_string(sorted[i]) + " repeated");
    }
    // ---- apply (the kernels read the slot lists from pinned host memory: taking
    //      the upload slot needs no device memory, so a removal works with the
    //      HBM budget exhausted)
    const Ctx::Staged st = c.stage_upload((size_t)n * 8, true);
    std::vector<uint64_t> per[kMaxBuckets];
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t loc = c.id_loc[ids[i]];
        int b = (int)(loc >> 40);
        uint64_t slot = loc & ((1ull << 40) - 1);
        per[b].push_back(slot);
        Bucket &B = c.buckets[b];
        B.n_lits -= B.h_len[slot];
        B.h_ids[slot] = kDeadId;
        B.h_len[slot] = 0;
        B.n_dead++;
        c.id_loc[ids[i]] = kNoLoc;
    }
    c.live -= n;
    {
        // one upload of every class's slot list, one kernel per class
        size_t total = 0;
        for (int b = 0; b < kMaxBuckets; ++b) total += per[b].size();
        size_t off = 0;
        for (int b = 0; b < kMaxBuckets; ++b) {
            if (per[b].empty()) continue;  // (an empty vector may hold no storage at all)
            std::memcpy(st.h + off * 8, per[b].data(), per[b].size() * 8);
            off += per[b].size();
        }
        off = 0;
        for (int b = 0; b < kMaxBuckets; ++b) {  // the kernels read the lists from pinned memory
            if (per[b].empty()) continue;
            Bucket &B = c.buckets[b];
            hipLaunchKernelGGL(k_tombstone, dim3(grid_for(per[b].size())), dim3(256), 0, c.stream, B.meta,
                               (const uint64_t *)st.hd + off, (uint32_t)per[b].size());
            GSS_HIP(hipGetLastError());
            off += per[b].size();
        }
        c.stage_done(st);
    }
    c.version++;
    priority_removed(c, ids, n);
    // ---- reclaim: compact a class once more than a quarter of its slots are dead
    for (int b = 0; b < kMaxBuckets; ++b) {
        Bucket &B = c.buckets[b];
        if (B.n_dead && B.n_dead * 4 > B.n_slots) compact_bucket(c, b);
    }
    GSS_API_END
}

extern "C" gss_status gss_store_info(const gss_ctx *ctx, uint64_t *live_clauses, uint64_t *next_id,
                                     uint64_t *device_bytes) {
    const Ctx *c = reinterpret_cast<const Ctx *>(ctx);
    if (!c) return GSS_ERR_INVALID_ARG;
    if (live_clauses) *live_clauses = c->live;
    if (next_id) *next_id = c->id_loc.size();
    if (device_bytes) *device_bytes = c->device_bytes;
    return GSS_OK;
}
