// Learned clause priority: per-clause statistics, training samples, scoring by
// the network of mlp.h, and the schedule the test kernel follows.
//
// Section 3.2 of the paper finds that a clause used recently is likely to be used
// again soon, and Section 3.7 keeps the GPU's store small with activity-based
// deletion.  Here that history feeds a network instead: after each run, every
// clause the run tested shifts its last-8 hit counts; a seeded fraction of the
// tested clauses become training samples (features before the run, label = hit
// in the run).  Scoring marks clauses below a threshold as low priority, and a
// scheduled test runs a low clause only when (run + id) % 4 == 0.
//
// State is kept per clause id (structure of arrays, grown with the id space):
// length, LBD, birth run, source thread, alive flag, 8 hit counts (16 bits each,
// one 16-byte word), this run's hit count, score and low flag, and two flag
// bytes (the history is nonzero; the test being observed reported the clause), so
// that the observation after a run reads the history and the hit count only where
// they can be nonzero.  The schedule bits the test kernel reads are
// per slot of each length class, rebuilt from the low flags when the store or
// the scores changed.
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <type_traits>

namespace gss {

struct Priority {
    gss_priority_config cfg{};
    uint64_t cap = 0;    // ids with state
    uint64_t n_ids = 0;  // ids issued so far (state valid below)
    uint32_t *len = nullptr, *birth = nullptr, *src = nullptr, *hits = nullptr;
    uint4 *hist = nullptr;  // [cap]: 8 hit counts of 16 bits, most recent in the low bits of .x
    float *lbd = nullptr, *score = nullptr;
    float *act = nullptr;  // activity (Section 3.7)
    uint8_t *alive = nullptr, *low = nullptr;
    uint8_t *dirty = nullptr;  // features changed (beyond age) since the clause was last scored
    uint8_t *hnz = nullptr;    // the history holds a nonzero count
    uint8_t *rec = nullptr;    // the test being observed reported the clause (its hit count is nonzero)
    float *sx = nullptr, *sy = nullptr;  // samples [sample_cap][kFeat], [sample_cap]
    uint32_t *counters = nullptr;        // [0] samples taken, [1] low clauses of the last scoring
    uint32_t *h_counters = nullptr;      // pinned copy
    float *params = nullptr;             // [kParams]
    uint32_t run = 0;
    uint64_t observed_serial = ~0ull;
    uint64_t score_epoch = 0;
    uint64_t built_version = ~0ull, built_epoch = ~0ull;
    float threshold = 0.f;
    double decay = 0.999;  // activity bump growth 1/decay per run
    double bump = 1.0;     // current bump
    uint32_t *list = nullptr;  // ids of the clauses an update rescores
    uint64_t list_cap = 0;
    bool scored = false;  // a full scoring (or marking) has set every low flag
};

namespace {

__device__ inline uint32_t lanes_below_(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct ProbeArgs {  // per-id arrays as the kernels see them
    uint32_t *len, *birth, *src, *hits;
    uint4 *hist;
    float *lbd, *score, *act;
    uint8_t *alive, *low, *dirty, *hnz, *rec;
    uint64_t cap;
};

ProbeArgs args_of(const Priority &p) {
    return ProbeArgs{p.len, p.birth, p.src,   p.hits,  p.hist, p.lbd, p.score,
                     p.act, p.alive, p.low,   p.dirty, p.hnz,  p.rec, p.cap};
}

__device__ inline void load_features(const ProbeArgs &a, uint64_t id, uint32_t run, float src_scale,
                                     float (&x)[kFeat]) {
    const uint4 v = a.hist[id];
    const uint32_t c[4] = {v.x, v.y, v.z, v.w};
    uint32_t h[kHist];
#pragma unroll
    for (int k = 0; k < kHist; ++k) h[k] = (c[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
    clause_features(x, a.len[id], a.lbd[id], run - a.birth[id], a.src[id], src_scale, h);
}

__global__ void k_prio_init(ProbeArgs a, uint64_t first, uint32_t n, const uint32_t *lens, uint32_t run) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t id = first + i;
    a.len[id] = lens[i];
    a.lbd[id] = (float)lens[i];
    a.birth[id] = run;
    a.src[id] = 0;
    a.hits[id] = 0;
    a.hist[id] = make_uint4(0, 0, 0, 0);
    a.alive[id] = 1;
    a.low[id] = 0;
    a.dirty[id] = 1;
    a.hnz[id] = 0;
    a.rec[id] = 0;
    a.score[id] = 1.f;
    a.act[id] = 0.f;
}

__global__ void k_prio_kill(ProbeArgs a, const uint32_t *ids, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    a.alive[ids[i]] = 0;
    a.low[ids[i]] = 0;
}

__global__ void k_prio_info(ProbeArgs a, const uint32_t *ids, uint32_t n, const float *lbd, const uint32_t *src) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    a.lbd[ids[i]] = lbd[i];
    a.src[ids[i]] = src[i];
    a.dirty[ids[i]] = 1;
}

// ---- counting with one atomic per workgroup.  Wavefronts of one address's
//      atomics serialize at the cache (one per wavefront over millions of ids
//      cost milliseconds), so a workgroup of 256 lanes sums first, or claims one
//      range of output rows for all its lanes.

constexpr uint32_t kPerThread = 16;  // ids per lane in the counting kernels (grid-stride free)

// Inclusive sum of v over the workgroup's lanes below and including this one;
// *total gets the workgroup's sum.  All 256 lanes must call it.
__device__ inline uint32_t block_inclusive_sum(uint32_t v, uint32_t &total) {
    __shared__ uint32_t wave_sum[4];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= (uint32_t)d) x += y;
    }
    if (lane == 63) wave_sum[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (uint32_t w = 0; w < 4; ++w) {
        before += w < wave ? wave_sum[w] : 0u;
        total += wave_sum[w];
    }
    __syncthreads();
    return before + x;
}

// Adds the workgroup's sum of v to *counter with one atomic (signed).
__device__ inline void block_add(int32_t v, uint32_t *counter) {
    uint32_t total = 0;
    block_inclusive_sum((uint32_t)v, total);
    if (threadIdx.x == 0 && total) atomicAdd(counter, total);  // wraps for negative sums
}

// Hit counts of the last run: one workgroup per report segment.  A clause's
// records may sit in several segments; the threads that flag it all store 1.
__global__ void k_prio_hits(ProbeArgs a, const gss_report *reports, const uint32_t *counts, uint32_t seg_cap,
                            uint32_t n_segments) {
    for (uint32_t s = blockIdx.x; s < n_segments; s += gridDim.x) {
        const uint32_t n = min(counts[s], seg_cap);
        const gss_report *seg = reports + (uint64_t)s * seg_cap;
        for (uint32_t r = threadIdx.x; r < n; r += blockDim.x) {
            const uint32_t id = seg[r].clause_id;
            atomicAdd(&a.hits[id], (uint32_t)__popcll(seg[r].mask));
            a.rec[id] = 1;
        }
    }
}

// After a run: samples, history shift, hit counter reset.  Each lane takes
// kObserve ids (strided by the workgroup size) and moves them through three
// phases: their flag bytes (alive, low, history nonzero, reported); then the hit counts, the
// histories and the activities the flags call for; then the stores.  Within a
// phase every load is issued before any is used, and no load sits under a branch
// (a lane that needs no value reads the workgroup's first element instead, a line
// all such lanes share), so that a lane waits for memory once per phase rather than
// once per id.  Most clauses neither hit nor carry a nonzero history, so their
// lanes read four bytes per id.  The arrays are addressed from the workgroup's
// first id (a uniform base) with 32-bit lane offsets.  The workgroup claims its
// sample rows with one atomic.  SAMPLE is false when no samples are taken (period 0).
constexpr uint32_t kObserve = 8;

template <bool SAMPLE>
__global__ __launch_bounds__(256) void k_prio_observe(ProbeArgs a, uint64_t n_ids, uint32_t run, uint32_t scheduled,
                                                      float src_scale, uint32_t period, uint64_t seed, float *sx,
                                                      float *sy, uint64_t sample_cap, uint32_t *counters, float bump) {
    __shared__ uint32_t base_s;
    const uint64_t base = (uint64_t)blockIdx.x * 256 * kObserve;  // below n_ids: the grid covers n_ids
    const uint8_t *alive = a.alive + base, *lowf = a.low + base;
    uint8_t *hnzf = a.hnz + base, *recf = a.rec + base, *dirty = a.dirty + base;
    uint32_t *hits = a.hits + base;
    uint4 *hist = a.hist + base;
    float *act = a.act + base;
    // lane offset of the k-th id (below 256 kObserve, so 32 bits hold every byte offset)
    auto off = [](uint32_t k) { return threadIdx.x + k * 256u; };
    auto at = [&](uint32_t k, uint32_t need) { return ((need >> k) & 1u) ? off(k) : 0u; };
    uint32_t in = 0;
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) in |= (base + off(k) < n_ids ? 1u : 0u) << k;
    uint32_t al[kObserve], lo[kObserve], hz[kObserve], rc[kObserve];
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) {
        al[k] = alive[at(k, in)];
        lo[k] = lowf[at(k, in)];
        hz[k] = hnzf[at(k, in)];
        rc[k] = recf[at(k, in)];
    }
    uint32_t live = 0, low = 0, nz = 0, hit = 0, tested = 0, sample = 0;  // bit k: id base + off(k)
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) {
        const bool i = (in >> k) & 1u;
        live |= (i && al[k] ? 1u : 0u) << k;
        low |= (i && lo[k] ? 1u : 0u) << k;
        nz |= (i && hz[k] ? 1u : 0u) << k;
        hit |= (i && rc[k] ? 1u : 0u) << k;
    }
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) {
        const uint64_t id = base + off(k);
        const bool skipped = scheduled && ((low >> k) & 1u) && ((run + (uint32_t)id) & 3u) != 0;
        const bool t = ((live >> k) & 1u) && !skipped;
        tested |= (t ? 1u : 0u) << k;
        if (SAMPLE) sample |= (t && mix64(seed ^ (id << 32) ^ run) % period == 0 ? 1u : 0u) << k;
    }
    // a clause without records has a zero count, one with a zero history a zero word
    const uint32_t need_hist = tested & nz, bumped = live & hit;
    uint32_t h[kObserve];
    float ac[kObserve];
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) {
        h[k] = hits[at(k, hit)];
        ac[k] = act[at(k, bumped)];
    }
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) h[k] = ((hit >> k) & 1u) ? h[k] : 0u;
    uint32_t pos = 0;
    if (SAMPLE) {  // sample rows are claimed only while samples are taken
        const uint32_t mine = __popc(sample);
        uint32_t total = 0;
        pos = block_inclusive_sum(mine, total) - mine;
        if (threadIdx.x == 0) base_s = total ? atomicAdd(&counters[0], total) : 0u;
        __syncthreads();
        pos += base_s;
    }
    // samples take the features as they were before this run, labelled by its hits
    for (uint32_t k = 0; SAMPLE && k < kObserve && sample; ++k) {
        if (!((sample >> k) & 1u)) continue;
        if (pos < sample_cap) {
            float x[kFeat];
            load_features(a, base + off(k), run, src_scale, x);
#pragma unroll
            for (int q = 0; q < kFeat; ++q) sx[(uint64_t)pos * kFeat + q] = x[q];
            sy[pos] = h[k] ? 1.f : 0.f;
        }
        ++pos;
    }
    uint4 v[kObserve];
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) v[k] = hist[at(k, need_hist)];
#pragma unroll
    for (uint32_t k = 0; k < kObserve; ++k) {
        const uint32_t nzk = (nz >> k) & 1u;
        // a tested clause shifts in this run's count (a history of zeros stays as it is)
        if (((tested >> k) & 1u) && (h[k] || nzk)) {
            const uint4 o = nzk ? v[k] : make_uint4(0, 0, 0, 0);
            const uint32_t hc = min(h[k], 0xFFFFu);  // at most 64 x 64 slots: never clipped
            const uint4 w = make_uint4((o.x << 16) | hc, (o.y << 16) | (o.x >> 16), (o.z << 16) | (o.y >> 16),
                                       (o.w << 16) | (o.z >> 16));
            hist[off(k)] = w;
            const uint32_t now = (w.x | w.y | w.z | w.w) ? 1u : 0u;
            if (now != nzk) hnzf[off(k)] = (uint8_t)now;
            // rescored by the next update only where its side of the threshold may
            // change: a low clause that hit, a high one that did not (the next full
            // scoring catches everything else)
            if (((low >> k) & 1u) ? h[k] != 0 : h[k] == 0) dirty[off(k)] = 1;
        }
        if (((live >> k) & 1u) && h[k]) {  // the count and its flag are cleared together (a dead clause keeps both)
            act[off(k)] = ac[k] + bump;  // Section 3.7: bumped whenever the clause triggers
            hits[off(k)] = 0;
            recf[off(k)] = 0;
        }
    }
}

// The light form of an observation (activity only): every clause with a record
// in the last test gets the current bump once, and its hit count is cleared.
// Runs after k_prio_hits over the same segments.
__global__ void k_prio_bump(ProbeArgs a, const gss_report *reports, const uint32_t *counts, uint32_t seg_cap,
                            uint32_t n_segments, float bump) {
    for (uint32_t s = blockIdx.x; s < n_segments; s += gridDim.x) {
        const uint32_t n = min(counts[s], seg_cap);
        const gss_report *seg = reports + (uint64_t)s * seg_cap;
        for (uint32_t r = threadIdx.x; r < n; r += blockDim.x) {
            const uint32_t id = seg[r].clause_id;
            if (atomicExch(&a.hits[id], 0u) != 0u) a.act[id] += bump;  // the first record of the clause
            a.rec[id] = 0;
        }
    }
}

__global__ void k_prio_scale(float *act, uint64_t n, float f) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        act[i] *= f;
}

__global__ void k_prio_gather_act(ProbeArgs a, const uint32_t *ids, uint32_t n, float *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a.act[ids[i]];
}


// Scoring on the matrix cores.  A wavefront scores 32 clauses per step with
// fp32 MFMAs (32x32 outputs, K = 2 per instruction) on the transposed
// activations: H1^T = W1^T X^T (K = the 12 features), then H2^T = W2^T H1^T
// (K = the 64 hidden units).  In the 32x32 result a lane holds one clause (its
// column, lane % 32) and 16 rows; those are exactly the values that lane must
// supply as the B operand (one K row for one clause) of the next product, so
// the activations never move between lanes: step s of the second product takes
// its two K rows from register s % 16 of tile s / 16 of the two lane halves,
// and the weights (the A operand) are loaded in that same row order.  The
// output layer sums each lane's 32 rows and its partner lane's (lane ^ 32).
// The weights stay in registers for all of a wavefront's steps.
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Workgroups of 4 wavefronts for scoring n ids, 32 per wavefront step; at most
// 4 workgroups per compute unit (the kernel holds its weights in registers).
unsigned score_grid(const Ctx &c, uint64_t n) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 127) / 128, (uint64_t)c.n_cu * 4));
}

// row of the 32x32 result held in register v by a lane of half `half`
__device__ constexpr uint32_t mfma_row(uint32_t v, uint32_t half) { return 8 * (v / 4) + 4 * half + (v % 4); }

// The raw per-clause statistics the features are made of, loaded ahead of use.
struct RawFeat {
    uint32_t len, birth, src;
    float lbd;
    uint4 hist;
};

__device__ inline void raw_load(const ProbeArgs &a, uint32_t id, RawFeat &r) {
    r.len = a.len[id];
    r.birth = a.birth[id];
    r.src = a.src[id];
    r.lbd = a.lbd[id];
    r.hist = a.hist[id];
}

// LIST: score the n ids of list[] (n = *list_n); else ids 0..n_ids-1 (removed
// ones get score 0 and are not low).  The first weight matrix and the second
// live in registers as MFMA operands; the biases and output weights in LDS; the
// next step's clause statistics are loaded while the current step multiplies.
template <bool LIST>
__global__ __launch_bounds__(256) void k_prio_score_mfma(ProbeArgs a, const float *__restrict__ params,
                                                         const uint32_t *list, const uint32_t *list_n, uint64_t n_ids,
                                                         uint32_t run, float src_scale, float threshold,
                                                         uint32_t *counters) {
    __shared__ float b1s[kHid], b2s[kHid], w3s[kHid];
    for (uint32_t t = threadIdx.x; t < kHid; t += blockDim.x) {
        b1s[t] = params[kOffB1 + t];
        b2s[t] = params[kOffB2 + t];
        w3s[t] = params[kOffW3 + t];
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
    float w1a[2][kFeat / 2], w2a[2][kHid / 2];
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
#pragma unroll
        for (uint32_t st = 0; st < kFeat / 2; ++st) w1a[u][st] = params[kOffW1 + (2 * st + half) * kHid + 32 * u + col];
#pragma unroll
        for (uint32_t st = 0; st < kHid / 2; ++st) {
            const uint32_t hid = 32 * (st / 16) + mfma_row(st % 16, half);
            w2a[u][st] = params[kOffW2 + hid * kHid + 32 * u + col];
        }
    }
    const float b3 = params[kOffB3];
    const uint64_t n = LIST ? (uint64_t)*list_n : n_ids;
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / 64;
    const uint64_t n_waves = (uint64_t)gridDim.x * blockDim.x / 64;
    int32_t count = 0;  // LIST: change in the number of low clauses; else low clauses
    // this lane's clause of a step starting at `base`
    auto clause_of = [&](uint64_t base, uint32_t &id, bool &valid, bool &live, RawFeat &r) {
        const uint64_t i = base + col;
        valid = i < n;
        id = valid ? (LIST ? list[i] : (uint32_t)i) : 0u;
        live = valid && (LIST || a.alive[id]);
        if (live) raw_load(a, id, r);
    };
    uint64_t base = wave * 32;
    uint32_t id = 0;
    bool valid = false, live = false;
    RawFeat r{};
    if (base < n) clause_of(base, id, valid, live, r);
    for (; base < n; base += n_waves * 32) {  // uniform per wavefront
        float x[kFeat];
        if (live) {
            uint32_t h[kHist];
            const uint32_t c4[4] = {r.hist.x, r.hist.y, r.hist.z, r.hist.w};
#pragma unroll
            for (int k = 0; k < kHist; ++k) h[k] = (c4[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
            clause_features(x, r.len, r.lbd, run - r.birth, r.src, src_scale, h);
        } else {
#pragma unroll
            for (int f = 0; f < kFeat; ++f) x[f] = 0.f;
        }
        const uint32_t cur_id = id;
        const bool cur_valid = valid, cur_live = live;
        const uint64_t next = base + n_waves * 32;
        if (next < n) clause_of(next, id, valid, live, r);  // in flight during the products
        // an index the compiler cannot see through: the LDS reads stay in the
        // loop instead of being hoisted into 96 more registers per lane
        uint32_t lds_row = 4 * half;
        asm volatile("" : "+v"(lds_row));
        f32x16 acc1[2], acc2[2];
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t v = 0; v < 16; ++v) {
                const uint32_t row = 32 * u + 8 * (v / 4) + (v % 4) + lds_row;  // mfma_row(v, half)
                acc1[u][v] = b1s[row];
                acc2[u][v] = b2s[row];
            }
#pragma unroll
        for (uint32_t st = 0; st < kFeat / 2; ++st) {
            const float bx = half ? x[2 * st + 1] : x[2 * st];
#pragma unroll
            for (uint32_t u = 0; u < 2; ++u)
                acc1[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(w1a[u][st], bx, acc1[u], 0, 0, 0);
        }
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t v = 0; v < 16; ++v) acc1[u][v] = fmaxf(acc1[u][v], 0.f);
#pragma unroll
        for (uint32_t st = 0; st < kHid / 2; ++st) {
            const float bh = acc1[st / 16][st % 16];
#pragma unroll
            for (uint32_t u = 0; u < 2; ++u)
                acc2[u] = __builtin_amdgcn_mfma_f32_32x32x2f32(w2a[u][st], bh, acc2[u], 0, 0, 0);
        }
        float part = 0.f;
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t v = 0; v < 16; ++v)
                part = fmaf(fmaxf(acc2[u][v], 0.f), w3s[32 * u + 8 * (v / 4) + (v % 4) + lds_row], part);
        const float z = part + __shfl_xor(part, 32) + b3;
        if (half == 0 && cur_valid) {
            if (!cur_live) {  // a removed clause: no score
                a.score[cur_id] = 0.f;
                a.low[cur_id] = 0;
            } else {
                const float prob = sigmoidf_(z);
                const bool now = prob < threshold;
                a.score[cur_id] = prob;
                if (LIST)
                    count += (int32_t)now - (int32_t)a.low[cur_id];
                else
                    count += now ? 1 : 0;
                a.low[cur_id] = now;
                a.dirty[cur_id] = 0;
            }
        }
    }
    block_add(count, &counters[1]);
}

// The dirty live clauses, compacted into a list (counters[2] = its length), so
// that the network runs on dense wavefronts rather than on scattered lanes.  The
// flag bytes are loaded once, all in flight together (an id past the end reads
// the workgroup's first byte instead, and is not counted).
__global__ __launch_bounds__(256) void k_prio_collect(ProbeArgs a, uint64_t n_ids, uint32_t *list, uint32_t *counters) {
    __shared__ uint32_t base_s;
    const uint64_t base = (uint64_t)blockIdx.x * 256 * kPerThread;  // below n_ids: the grid covers n_ids
    const uint8_t *alive = a.alive + base, *dirty = a.dirty + base;
    uint32_t al[kPerThread], di[kPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kPerThread; ++k) {
        const uint32_t o = base + threadIdx.x + k * 256u < n_ids ? threadIdx.x + k * 256u : 0u;
        al[k] = alive[o];
        di[k] = dirty[o];
    }
    uint32_t flags = 0;  // bit k: id base + threadIdx.x + 256 k is live and dirty
#pragma unroll
    for (uint32_t k = 0; k < kPerThread; ++k)
        flags |= (base + threadIdx.x + k * 256u < n_ids && al[k] && di[k] ? 1u : 0u) << k;
    const uint32_t mine = __popc(flags);
    uint32_t total = 0;
    uint32_t pos = block_inclusive_sum(mine, total) - mine;
    if (threadIdx.x == 0) base_s = total ? atomicAdd(&counters[2], total) : 0u;
    __syncthreads();
    pos += base_s;
    for (uint32_t f = flags; f; f &= f - 1)
        list[pos++] = (uint32_t)(base + threadIdx.x + 256u * (uint32_t)__builtin_ctz(f));
}


// Schedule bits of every length class in one launch: bit s of word s / 32 of a
// class is set when slot s holds a live low-priority clause.  Workgroup g takes
// 256 slots of the class whose block range holds g.
struct SchedBitsClass {
    const uint2 *meta;
    uint32_t *bits;
    uint64_t n_slots, n_words;
    uint32_t block_begin;
};

struct SchedBitsTable {
    SchedBitsClass cls[kMaxBuckets];
    uint32_t n;
};

__global__ __launch_bounds__(256) void k_sched_bits(const SchedBitsTable tab, const uint8_t *low) {
    uint32_t c = 0;
    while (c + 1 < tab.n && blockIdx.x >= tab.cls[c + 1].block_begin) ++c;
    const SchedBitsClass &C = tab.cls[c];
    const uint64_t s = (uint64_t)(blockIdx.x - C.block_begin) * 256 + threadIdx.x;
    bool b = false;
    if (s < C.n_slots) {
        const uint2 m = C.meta[s];
        b = m.x != 0 && low[m.y];
    }
    const uint64_t bal = __ballot(b);
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t w = (s - lane) / 32;
    if (lane == 0 && w < C.n_words) C.bits[w] = (uint32_t)bal;
    if (lane == 32 && w + 1 < C.n_words) C.bits[w + 1] = (uint32_t)(bal >> 32);
}

__global__ __launch_bounds__(256) void k_prio_mark(ProbeArgs a, const uint8_t *low, uint64_t n, uint32_t *counters) {
    uint32_t lows = 0;
    for (uint64_t id = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; id < n; id += (uint64_t)gridDim.x * blockDim.x) {
        const bool lo = a.alive[id] && low[id];
        a.low[id] = lo;
        lows += lo ? 1u : 0u;
    }
    block_add((int32_t)lows, &counters[1]);
}

__global__ void k_prio_fetch(ProbeArgs a, const uint32_t *ids, uint32_t n, uint32_t run, float src_scale, float *x,
                             float *score, uint8_t *low) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[kFeat];
    load_features(a, ids[i], run, src_scale, f);
#pragma unroll
    for (int k = 0; k < kFeat; ++k) x[(uint64_t)i * kFeat + k] = f[k];
    score[i] = a.score[ids[i]];
    low[i] = a.low[ids[i]];
}

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

unsigned grid_of(uint64_t n, unsigned block = 256) { return (unsigned)std::max<uint64_t>(1, (n + block - 1) / block); }

float src_scale(const Priority &p) { return 1.f / (float)std::max<uint32_t>(1, p.cfg.n_sources - 1); }

// Grows the per-id arrays to hold `need` ids (contents kept).
void grow(Ctx &c, Priority &p, uint64_t need) {
    if (need <= p.cap) return;
    const uint64_t cap = std::max<uint64_t>({need, p.cap + p.cap / 2, 1u << 16});
    c.sync();
    auto move = [&](auto *&arr, size_t elem, uint64_t rows) {
        using T = std::remove_reference_t<decltype(*arr)>;
        T *q = (T *)c.dalloc(cap * elem * rows);
        for (uint64_t r = 0; r < rows && arr; ++r)
            GSS_HIP(hipMemcpyAsync((char *)q + r * cap * elem, (char *)arr + r * p.cap * elem, p.n_ids * elem,
                                   hipMemcpyDeviceToDevice, c.stream));
        c.sync();
        c.dfree(arr);
        arr = q;
    };
    move(p.len, 4, 1);
    move(p.birth, 4, 1);
    move(p.src, 4, 1);
    move(p.hits, 4, 1);
    move(p.hist, 16, 1);
    move(p.lbd, 4, 1);
    move(p.score, 4, 1);
    move(p.act, 4, 1);
    move(p.alive, 1, 1);
    move(p.low, 1, 1);
    move(p.dirty, 1, 1);
    move(p.hnz, 1, 1);
    move(p.rec, 1, 1);
    p.cap = cap;
}

Priority &need_prio(Ctx &c) {
    GSS_REQUIRE(c.prio, GSS_ERR_STATE, "the learned priority is not enabled (gss_priority_enable)");
    return *c.prio;
}

}  // namespace

void priority_added(Ctx &c, uint64_t first, uint32_t n, const uint64_t *offsets) {
    if (!c.prio || n == 0) return;
    Priority &p = *c.prio;
    grow(c, p, first + n);
    const Ctx::Staged st = c.stage_upload((size_t)n * 4);
    uint32_t *h = (uint32_t *)st.h;
    for (uint32_t i = 0; i < n; ++i) h[i] = (uint32_t)(offsets[i + 1] - offsets[i]);
    GSS_HIP(hipMemcpyAsync(st.d, st.h, (size_t)n * 4, hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(k_prio_init, dim3(grid_of(n)), dim3(256), 0, c.stream, args_of(p), first, n,
                       (const uint32_t *)st.d, p.run);
    GSS_HIP(hipGetLastError());
    c.stage_done(st);
    p.n_ids = std::max<uint64_t>(p.n_ids, first + n);
}

void priority_removed(Ctx &c, const uint32_t *ids, uint32_t n) {
    if (!c.prio || n == 0) return;
    Priority &p = *c.prio;
    // read over the bus from pinned memory: a removal takes no device memory
    const Ctx::Staged st = c.stage_upload((size_t)n * 4, true);
    std::memcpy(st.h, ids, (size_t)n * 4);
    hipLaunchKernelGGL(k_prio_kill, dim3(grid_of(n)), dim3(256), 0, c.stream, args_of(p), (const uint32_t *)st.hd, n);
    GSS_HIP(hipGetLastError());
    c.stage_done(st);
}

void priority_reserve(Ctx &c, uint64_t n_ids) {
    if (c.prio) grow(c, *c.prio, n_ids);
}

// Grows the bump by 1/decay after an observed run; activities and bump are
// scaled by 1e-20 together once the bump passes 1e20 (float range).
static void next_bump(Ctx &c, Priority &p) {
    p.run++;
    p.bump /= p.decay;
    if (p.bump > 1e20) {
        if (p.n_ids)
            hipLaunchKernelGGL(k_prio_scale, dim3((unsigned)std::min<uint64_t>(grid_of(p.n_ids), 65536)), dim3(256), 0,
                               c.stream, p.act, p.n_ids, 1e-20f);
        GSS_HIP(hipGetLastError());
        p.bump *= 1e-20;
    }
}

void priority_bump_hits(Ctx &c) {
    Priority &p = need_prio(c);
    if (c.last_waves && c.n_reports) {
        const dim3 grid(std::min<uint32_t>(c.last_waves, 65535));
        hipLaunchKernelGGL(k_prio_hits, grid, dim3(256), 0, c.stream, args_of(p), c.reports, c.seg_counts, c.seg_cap,
                           c.last_waves);
        GSS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_prio_bump, grid, dim3(256), 0, c.stream, args_of(p), c.reports, c.seg_counts, c.seg_cap,
                           c.last_waves, (float)p.bump);
        GSS_HIP(hipGetLastError());
    }
    p.observed_serial = c.test_serial;
    next_bump(c, p);
}

std::vector<uint32_t> priority_evict(Ctx &c, uint64_t keep) {
    Priority &p = need_prio(c);
    if (c.live <= keep) return {};
    // activities of every issued id to the host; the live ones sorted, least active first
    std::vector<float> act(p.n_ids);
    if (p.n_ids) GSS_HIP(hipMemcpyAsync(act.data(), p.act, p.n_ids * 4, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    std::vector<uint32_t> live;
    live.reserve(c.live);
    for (uint64_t id = 0; id < c.id_loc.size(); ++id)
        if (c.id_loc[id] != kNoLoc) live.push_back((uint32_t)id);
    const uint64_t n_rm = live.size() - keep;
    auto before = [&](uint32_t x, uint32_t y) { return act[x] != act[y] ? act[x] < act[y] : x < y; };
    std::nth_element(live.begin(), live.begin() + (ptrdiff_t)(n_rm - 1), live.end(), before);
    std::vector<uint32_t> rm(live.begin(), live.begin() + (ptrdiff_t)n_rm);
    gss_ctx *ctx = reinterpret_cast<gss_ctx *>(&c);
    for (uint64_t k = 0; k < n_rm; k += 1u << 24) {
        const uint32_t m = (uint32_t)std::min<uint64_t>(n_rm - k, 1u << 24);
        const gss_status rc = gss_remove_clauses(ctx, rm.data() + k, m);
        if (rc != GSS_OK) throw Error(rc, c.last_error);
    }
    return rm;
}

uint32_t priority_schedule(Ctx &c) {
    Priority &p = need_prio(c);
    GSS_REQUIRE(p.score_epoch > 0, GSS_ERR_STATE, "a scheduled test needs a scoring first (gss_priority_score)");
    bool fresh = p.built_version == c.version && p.built_epoch == p.score_epoch;
    for (int b = 0; b < kMaxBuckets && fresh; ++b)
        fresh = c.buckets[b].low_words >= (c.buckets[b].cap_slots + 31) / 32;
    if (!fresh) {
        SchedBitsTable tab{};
        uint32_t blocks = 0;
        for (int b = 0; b < kMaxBuckets; ++b) {
            Bucket &B = c.buckets[b];
            if (B.cap_slots == 0) continue;
            const uint64_t words = (B.cap_slots + 31) / 32;
            if (B.low_words < words) {
                c.sync();
                c.dfree(B.low);
                B.low = nullptr;
                B.low_words = 0;
                B.low = (uint32_t *)c.dalloc(words * 4);
                B.low_words = words;
            }
            tab.cls[tab.n++] = SchedBitsClass{B.meta, B.low, B.n_slots, B.low_words, blocks};
            blocks += (uint32_t)((B.low_words * 32 + 255) / 256);
        }
        if (blocks) {  // every class in one launch
            hipLaunchKernelGGL(k_sched_bits, dim3(blocks), dim3(256), 0, c.stream, tab, (const uint8_t *)p.low);
            GSS_HIP(hipGetLastError());
        }
        p.built_version = c.version;
        p.built_epoch = p.score_epoch;
    }
    return p.run;
}

void priority_release(Ctx &c) {
    Priority *p = c.prio;
    if (!p) return;
    for (void *q : {(void *)p->len, (void *)p->birth, (void *)p->src, (void *)p->hits, (void *)p->hist, (void *)p->lbd,
                    (void *)p->score, (void *)p->act, (void *)p->alive, (void *)p->low, (void *)p->dirty, (void *)p->hnz, (void *)p->rec, (void *)p->sx, (void *)p->sy,
                    (void *)p->counters, (void *)p->params, (void *)p->list})
        c.dfree(q);
    if (p->h_counters) (void)hipHostFree(p->h_counters);
    delete p;
    c.prio = nullptr;
}

}  // namespace gss

using namespace gss;

extern "C" gss_status gss_priority_enable(gss_ctx *ctx, const gss_priority_config *cfg) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(cfg, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(!c.prio, GSS_ERR_STATE, "the learned priority is already enabled");
    GSS_REQUIRE(cfg->n_sources >= 1, GSS_ERR_INVALID_ARG, "n_sources must be at least 1");
    GSS_REQUIRE(cfg->sample_period == 0 || cfg->sample_capacity >= 1, GSS_ERR_INVALID_ARG,
                "sampling needs a sample capacity");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    GSS_REQUIRE(cfg->activity_decay == 0 || (cfg->activity_decay > 0 && cfg->activity_decay <= 1), GSS_ERR_INVALID_ARG,
                "activity_decay must be in (0, 1]");
    auto p = std::make_unique<Priority>();
    p->cfg = *cfg;
    p->decay = cfg->activity_decay ? cfg->activity_decay : 0.999;
    c.prio = p.get();
    try {
        Priority &q = *p;
        q.counters = (uint32_t *)c.dalloc(256);
        GSS_HIP(hipHostMalloc((void **)&q.h_counters, 256, hipHostMallocDefault));
        launch_fill_u32(c, q.counters, 64, 0);
        q.params = (float *)c.dalloc(kParams * 4);
        if (cfg->sample_capacity) {
            q.sx = (float *)c.dalloc(cfg->sample_capacity * kFeat * 4);
            q.sy = (float *)c.dalloc(cfg->sample_capacity * 4);
        }
        // He-uniform weights (bound sqrt(6 / fan_in)), zero biases, from the seed
        std::vector<float> w(kParams, 0.f);
        uint64_t s = cfg->seed * 0x9E3779B97F4A7C15ull + 1;
        auto uni = [&](float bound) { return (float)((splitmix(s) >> 11) * (1.0 / 9007199254740992.0) * 2 - 1) * bound; };
        for (int i = 0; i < kFeat * kHid; ++i) w[kOffW1 + i] = uni(std::sqrt(6.f / kFeat));
        for (int i = 0; i < kHid * kHid; ++i) w[kOffW2 + i] = uni(std::sqrt(6.f / kHid));
        for (int i = 0; i < kHid; ++i) w[kOffW3 + i] = uni(std::sqrt(6.f / kHid));
        GSS_HIP(hipMemcpy(q.params, w.data(), kParams * 4, hipMemcpyHostToDevice));
        // clauses already in the store get their lengths now; LBD defaults to the length
        std::vector<uint64_t> offs(c.id_loc.size() + 1, 0);
        for (uint64_t id = 0; id < c.id_loc.size(); ++id) {
            uint32_t L = 0;
            if (c.id_loc[id] != kNoLoc) {
                const uint64_t loc = c.id_loc[id];
                L = c.buckets[loc >> 40].h_len[loc & ((1ull << 40) - 1)];
            }
            offs[id + 1] = offs[id] + L;
        }
        const uint64_t n = c.id_loc.size();
        for (uint64_t first = 0; first < n; first += 1u << 22) {
            const uint32_t m = (uint32_t)std::min<uint64_t>(n - first, 1u << 22);
            std::vector<uint64_t> o(offs.begin() + first, offs.begin() + first + m + 1);
            priority_added(c, first, m, o.data());
        }
        std::vector<uint32_t> dead;
        for (uint64_t id = 0; id < n; ++id)
            if (c.id_loc[id] == kNoLoc) dead.push_back((uint32_t)id);
        for (size_t k = 0; k < dead.size(); k += 1u << 20)
            priority_removed(c, dead.data() + k, (uint32_t)std::min<size_t>(dead.size() - k, 1u << 20));
        c.sync();
    } catch (...) {
        priority_release(c);
        p.release();
        throw;
    }
    p.release();
    GSS_API_END
}

extern "C" gss_status gss_priority_set_clause_info(gss_ctx *ctx, const uint32_t *ids, uint32_t n, const float *lbd,
                                                   const uint32_t *source) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(ids && lbd && source, GSS_ERR_INVALID_ARG, "null argument");
    for (uint32_t i = 0; i < n; ++i) {
        GSS_REQUIRE(ids[i] < c.id_loc.size() && c.id_loc[ids[i]] != kNoLoc, GSS_ERR_UNKNOWN_ID, "clause id not live");
        GSS_REQUIRE(source[i] < p.cfg.n_sources, GSS_ERR_INVALID_ARG, "source beyond n_sources");
        GSS_REQUIRE(lbd[i] >= 0 && std::isfinite(lbd[i]), GSS_ERR_INVALID_ARG, "LBD must be finite and >= 0");
    }
    const Ctx::Staged st = c.stage_upload((size_t)n * 12);
    std::memcpy(st.h, ids, (size_t)n * 4);
    std::memcpy(st.h + (size_t)n * 4, lbd, (size_t)n * 4);
    std::memcpy(st.h + (size_t)n * 8, source, (size_t)n * 4);
    GSS_HIP(hipMemcpyAsync(st.d, st.h, (size_t)n * 12, hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(k_prio_info, dim3(grid_of(n)), dim3(256), 0, c.stream, args_of(p), (const uint32_t *)st.d, n,
                       (const float *)(st.d + (size_t)n * 4), (const uint32_t *)(st.d + (size_t)n * 8));
    GSS_HIP(hipGetLastError());
    c.stage_done(st);
    GSS_API_END
}

extern "C" gss_status gss_priority_observe(gss_ctx *ctx) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    GSS_REQUIRE(c.tested, GSS_ERR_STATE, "no test to observe");
    GSS_REQUIRE(p.observed_serial != c.test_serial, GSS_ERR_STATE, "this test was already observed");
    GSS_REQUIRE(!(c.last_flags & GSS_TEST_DENSE), GSS_ERR_STATE, "a dense test has no records to observe");
    GSS_REQUIRE(c.n_kept == c.n_reports, GSS_ERR_REPORT_OVERFLOW, "the test lost records: its hits are incomplete");
    if (c.last_waves)
        hipLaunchKernelGGL(k_prio_hits, dim3(std::min<uint32_t>(c.last_waves, 65535)), dim3(256), 0, c.stream,
                           args_of(p), c.reports, c.seg_counts, c.seg_cap, c.last_waves);
    GSS_HIP(hipGetLastError());
    if (p.n_ids)
        hipLaunchKernelGGL(p.cfg.sample_period ? k_prio_observe<true> : k_prio_observe<false>,
                           dim3(grid_of(p.n_ids, 256 * kObserve)), dim3(256), 0, c.stream, args_of(p), p.n_ids, p.run,
                           (c.last_flags & GSS_TEST_SCHEDULED) ? 1u : 0u, src_scale(p), p.cfg.sample_period,
                           p.cfg.seed, p.sx, p.sy, p.cfg.sample_capacity, p.counters, (float)p.bump);
    GSS_HIP(hipGetLastError());
    p.observed_serial = c.test_serial;
    next_bump(c, p);
    GSS_API_END
}

extern "C" gss_status gss_priority_train(gss_ctx *ctx, uint32_t epochs, const gss_adam_config *cfg, uint64_t seed,
                                         float *out_loss) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(cfg && epochs >= 1 && cfg->batch >= 1 && cfg->lr > 0, GSS_ERR_INVALID_ARG, "bad training settings");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    GSS_HIP(hipMemcpyAsync(p.h_counters, p.counters, 8, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    const uint64_t n = std::min<uint64_t>(p.h_counters[0], p.cfg.sample_capacity);
    GSS_REQUIRE(n >= 1, GSS_ERR_STATE, "no training samples yet");
    // epochs of seeded Fisher-Yates permutations
    const uint64_t n_order = n * epochs;
    std::vector<uint32_t> order(n_order);
    uint64_t s = seed * 0xD1B54A32D192ED03ull + 7;
    for (uint32_t e = 0; e < epochs; ++e) {
        uint32_t *o = order.data() + (uint64_t)e * n;
        for (uint64_t i = 0; i < n; ++i) o[i] = (uint32_t)i;
        for (uint64_t i = n - 1; i > 0; --i) std::swap(o[i], o[splitmix(s) % (i + 1)]);
    }
    MlpWork &w = mlp_work(c);
    c.sync();
    char *st = mlp_stage(c, w, n_order * 4);
    GSS_HIP(hipMemcpyAsync(st, order.data(), n_order * 4, hipMemcpyHostToDevice, c.stream));
    GSS_HIP(hipMemcpyAsync(w.params, p.params, kParams * 4, hipMemcpyDeviceToDevice, c.stream));
    launch_fill_u32(c, (uint32_t *)w.m, kParams, 0);
    launch_fill_u32(c, (uint32_t *)w.v, kParams, 0);
    w.step = 0;
    for (uint64_t first = 0; first < n_order; first += cfg->batch) {
        const uint32_t nb = (uint32_t)std::min<uint64_t>(cfg->batch, n_order - first);
        mlp_queue_grad(c, w, p.sx, p.sy, (const uint32_t *)st, first, nb);
        mlp_queue_adam(c, w, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps);
    }
    GSS_HIP(hipMemcpyAsync(p.params, w.params, kParams * 4, hipMemcpyDeviceToDevice, c.stream));
    GSS_HIP(hipMemcpyAsync(w.h_loss, w.loss, 4, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    if (out_loss) *out_loss = *w.h_loss;
    GSS_API_END
}

extern "C" gss_status gss_priority_set_sampling(gss_ctx *ctx, uint32_t period) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(period == 0 || p.cfg.sample_capacity >= 1, GSS_ERR_INVALID_ARG, "sampling needs a sample capacity");
    p.cfg.sample_period = period;
    GSS_API_END
}

extern "C" gss_status gss_priority_clear_samples(gss_ctx *ctx) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    launch_fill_u32(c, p.counters, 1, 0);
    GSS_API_END
}

extern "C" gss_status gss_priority_score(gss_ctx *ctx, float threshold, uint64_t *out_n_low) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(std::isfinite(threshold), GSS_ERR_INVALID_ARG, "threshold must be finite");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    launch_fill_u32(c, p.counters + 1, 1, 0);
    if (p.n_ids)
        hipLaunchKernelGGL(k_prio_score_mfma<false>, dim3(score_grid(c, p.n_ids)), dim3(256), 0, c.stream, args_of(p),
                           p.params, nullptr, nullptr, p.n_ids, p.run, src_scale(p), threshold, p.counters);
    GSS_HIP(hipGetLastError());
    p.threshold = threshold;
    p.scored = true;
    p.score_epoch++;
    if (out_n_low) {
        GSS_HIP(hipMemcpyAsync(p.h_counters, p.counters, 8, hipMemcpyDeviceToHost, c.stream));
        c.sync();
        *out_n_low = p.h_counters[1];
    }
    GSS_API_END
}

extern "C" gss_status gss_priority_update(gss_ctx *ctx, uint64_t *out_n_low) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(p.scored, GSS_ERR_STATE, "gss_priority_update needs a full scoring first (gss_priority_score)");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    if (p.n_ids) {
        if (p.list_cap < p.cap) {
            c.sync();
            c.dfree(p.list);
            p.list = nullptr;
            p.list_cap = 0;
            p.list = (uint32_t *)c.dalloc(p.cap * 4);
            p.list_cap = p.cap;
        }
        launch_fill_u32(c, p.counters + 2, 1, 0);
        hipLaunchKernelGGL(k_prio_collect, dim3(grid_of(p.n_ids, 256 * kPerThread)), dim3(256), 0, c.stream, args_of(p),
                           p.n_ids, p.list, p.counters);
        GSS_HIP(hipGetLastError());
        // the list's length is on the device: a grid for all ids, whose surplus wavefronts exit at once
        hipLaunchKernelGGL(k_prio_score_mfma<true>, dim3(score_grid(c, p.n_ids)), dim3(256), 0, c.stream, args_of(p),
                           p.params, p.list, p.counters + 2, 0ull, p.run, src_scale(p), p.threshold, p.counters);
        GSS_HIP(hipGetLastError());
    }
    p.score_epoch++;
    if (out_n_low) {
        GSS_HIP(hipMemcpyAsync(p.h_counters, p.counters, 8, hipMemcpyDeviceToHost, c.stream));
        c.sync();
        *out_n_low = p.h_counters[1];
    }
    GSS_API_END
}

extern "C" gss_status gss_priority_mark(gss_ctx *ctx, const uint8_t *low, uint64_t n) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(low, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(n == p.n_ids, GSS_ERR_INVALID_ARG, "low must hold one flag per issued id");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    launch_fill_u32(c, p.counters + 1, 1, 0);
    if (n) {
        MlpWork &w = mlp_work(c);
        c.sync();
        char *st = mlp_stage(c, w, n);
        GSS_HIP(hipMemcpyAsync(st, low, n, hipMemcpyHostToDevice, c.stream));
        hipLaunchKernelGGL(k_prio_mark, dim3(std::min<uint64_t>(grid_of(n), (uint64_t)c.n_cu * 16)), dim3(256), 0,
                           c.stream, args_of(p), (const uint8_t *)st, n, p.counters);
        GSS_HIP(hipGetLastError());
        c.sync();
    }
    p.score_epoch++;
    p.scored = false;  // low flags of another policy: an update would mix the two
    GSS_API_END
}

extern "C" gss_status gss_priority_params(gss_ctx *ctx, float *get, const float *set) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    if (set) GSS_HIP(hipMemcpyAsync(p.params, set, kParams * 4, hipMemcpyHostToDevice, c.stream));
    if (get) GSS_HIP(hipMemcpyAsync(get, p.params, kParams * 4, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    GSS_API_END
}

extern "C" gss_status gss_priority_fetch(gss_ctx *ctx, const uint32_t *ids, uint32_t n, float *out_features,
                                         float *out_scores, uint8_t *out_low) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(ids && out_features && out_scores && out_low, GSS_ERR_INVALID_ARG, "null argument");
    for (uint32_t i = 0; i < n; ++i)
        GSS_REQUIRE(ids[i] < p.n_ids, GSS_ERR_UNKNOWN_ID, "clause id never issued");
    MlpWork &w = mlp_work(c);
    const size_t ib = ((size_t)n * 4 + 255) / 256 * 256, xb = ((size_t)n * kFeat * 4 + 255) / 256 * 256,
                 sb = ((size_t)n * 4 + 255) / 256 * 256;
    c.sync();
    char *st = mlp_stage(c, w, ib + xb + sb + n);
    GSS_HIP(hipMemcpyAsync(st, ids, (size_t)n * 4, hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(k_prio_fetch, dim3(grid_of(n)), dim3(256), 0, c.stream, args_of(p), (const uint32_t *)st, n,
                       p.run, src_scale(p), (float *)(st + ib), (float *)(st + ib + xb), (uint8_t *)(st + ib + xb + sb));
    GSS_HIP(hipGetLastError());
    GSS_HIP(hipMemcpyAsync(out_features, st + ib, (size_t)n * kFeat * 4, hipMemcpyDeviceToHost, c.stream));
    GSS_HIP(hipMemcpyAsync(out_scores, st + ib + xb, (size_t)n * 4, hipMemcpyDeviceToHost, c.stream));
    GSS_HIP(hipMemcpyAsync(out_low, st + ib + xb + sb, n, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    GSS_API_END
}

extern "C" gss_status gss_priority_reduce(gss_ctx *ctx, uint64_t keep, uint64_t *out_removed) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    (void)p;
    if (out_removed) *out_removed = 0;
    const uint64_t n_rm = priority_evict(c, keep).size();
    if (out_removed) *out_removed = n_rm;
    GSS_API_END
}

extern "C" gss_status gss_priority_activity(gss_ctx *ctx, const uint32_t *ids, uint32_t n, float *out_activity) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(ids && out_activity, GSS_ERR_INVALID_ARG, "null argument");
    for (uint32_t i = 0; i < n; ++i) GSS_REQUIRE(ids[i] < p.n_ids, GSS_ERR_UNKNOWN_ID, "clause id never issued");
    MlpWork &w = mlp_work(c);
    const size_t ib = ((size_t)n * 4 + 255) / 256 * 256;
    c.sync();
    char *st = mlp_stage(c, w, 2 * ib);
    GSS_HIP(hipMemcpyAsync(st, ids, (size_t)n * 4, hipMemcpyHostToDevice, c.stream));
    hipLaunchKernelGGL(k_prio_gather_act, dim3(grid_of(n)), dim3(256), 0, c.stream, args_of(p), (const uint32_t *)st, n,
                       (float *)(st + ib));
    GSS_HIP(hipGetLastError());
    GSS_HIP(hipMemcpyAsync(out_activity, st + ib, (size_t)n * 4, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    GSS_API_END
}

extern "C" gss_status gss_priority_samples(gss_ctx *ctx, float *out_x, float *out_y, uint64_t cap, uint64_t *out_n) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    Priority &p = need_prio(c);
    GSS_REQUIRE(out_n, GSS_ERR_INVALID_ARG, "null argument");
    GSS_HIP(hipMemcpyAsync(p.h_counters, p.counters, 8, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    const uint64_t n = std::min<uint64_t>({(uint64_t)p.h_counters[0], p.cfg.sample_capacity, cap});
    if (n && out_x) GSS_HIP(hipMemcpyAsync(out_x, p.sx, n * kFeat * 4, hipMemcpyDeviceToHost, c.stream));
    if (n && out_y) GSS_HIP(hipMemcpyAsync(out_y, p.sy, n * 4, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    *out_n = n;
    GSS_API_END
}

extern "C" gss_status gss_priority_info(const gss_ctx *ctx, uint32_t *out_run, uint64_t *out_samples,
                                        uint64_t *out_n_low) {
    const Ctx *c = reinterpret_cast<const Ctx *>(ctx);
    if (!c) return GSS_ERR_INVALID_ARG;
    if (!c->prio) return GSS_ERR_STATE;
    const Priority &p = *c->prio;
    if (hipMemcpyAsync(p.h_counters, p.counters, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return GSS_ERR_DEVICE;
    if (out_run) *out_run = p.run;
    if (out_samples) *out_samples = std::min<uint64_t>(p.h_counters[0], p.cfg.sample_capacity);
    if (out_n_low) *out_n_low = p.h_counters[1];
    return GSS_OK;
}
