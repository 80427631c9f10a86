// Device side of the clause test (Sections 3.4-3.5), shared by the single-store
// kernel (test.hip) and the batched kernel (batch.hip).
//
// Two forms of parallelism, as in Section 3.5: wavefront lanes work on different
// clauses, and each lane tests up to 256 assignment slots at once with 64-bit
// bitwise operations.  A clause is spread over LPC lanes, each lane owning WPL
// consecutive 64-slot words of the plane row (one 32-byte sector: the unit in
// which scattered reads are filled), so a wavefront covers T = 64 / LPC clauses.
//
// Falsified mode: the clause mask is the AND over its literals of the gathered
// plane words (the allFalse half of the bitwise trigger test of Section 3.4).
// Trigger mode (Definition 1): the same loop also carries the oneUndef words,
// which need the row of the opposite literal as well (isSet = F-row | T-row).
//
// Early exit: a wavefront stops reading literals once no lane of its clauses has
// a live bit left; a lane whose words are all dead issues no more loads.  Hot
// rows (the first `hot_rows` plane rows, those of the lowest variables; a
// clause's smallest code comes first) can be staged in LDS.
//
// Reports need no atomics: every wavefront owns one segment of the report buffer
// and appends its records at its running count + (records of lower lanes, from
// mbcnt).  Counts beyond a segment's capacity are still counted, so the exact
// size needed is always known.
#pragma once

#include "gss_internal.h"

#include <type_traits>

namespace gss {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Literals gathered between a lane's liveness checks.  Plain tests take one: a
// lane whose words died stops at once; its gathers then wait on each other, but
// the lines saved count for more than the latency hidden (measured: 4 -> 1 took
// the paper-scale test from 0.545 to 0.481 ms).  With the aggregate pre-test a
// group of four is checked at once: its aggregate loads and gathers go out
// together instead of as one long dependent chain.
template <bool AGG>
constexpr uint32_t kGroupOf = AGG ? 4u : 1u;

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so that a
// contiguous range of logical workgroups (neighbouring tiles, sharing cache lines
// of the code and metadata streams and, with clauses ordered by lead literal,
// the plane rows of their first literals) runs on one XCD and its L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    constexpr uint32_t X = 8;
    const uint32_t x = b % X, i = b / X, q = nb / X, r = nb % X;
    return x * q + (x < r ? x : r) + i;
}

// Buffer resources for the per-tile loads: pointers read from the descriptor
// table would otherwise become flat loads (tracked by the LDS counter too); a
// buffer load is a plain vector-memory load with a 32-bit byte offset.
constexpr int kBufferDword3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
// Cache policy of the per-tile streams (codes, metadata, schedule bits): each is
// read once, so they are marked non-temporal and leave the caches to the plane
// rows (measured at paper scale: 0.490 -> 0.488 ms).
constexpr int kStream = 2;

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint64_t bytes) {
    const int n = bytes >= 0xFFFFFFFFull ? -1 : (int)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, n, kBufferDword3);
}

__device__ inline uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <uint32_t X>
constexpr uint32_t ilog2() {
    return X <= 1 ? 0 : 1 + ilog2<X / 2>();
}

// What a wavefront's test did (GSS_TEST_COUNT; wave-uniform): plane rows its
// lanes read (a lane reads its words of one row; trigger mode reads the
// opposite literal's row beside it, counted once), and (clause, word) pairs the
// aggregate pre-test settled.
struct Counts {
    bool on = false;
    uint32_t gathers = 0;
    uint32_t settled = 0;
};

// A tile as one lane sees it: wave-uniform code resource and stride, this lane's
// byte offset of its clause's codes, its metadata (length, id) and its codes 0..3.
struct TileRef {
    __amdgpu_buffer_rsrc_t lits;
    uint32_t s_log2;
    uint32_t code_off;
    uint2 meta;
    uint4 c0;
    uint32_t lowword;   // schedule bits of the slot's 32-slot group (0: no schedule)
    uint32_t lowshift;  // this slot's bit in it
};

// Locates tile t of a store whose tiles hold T clauses (bi: bucket cursor, only
// ever advanced) and issues the loads of the metadata and first four codes of
// the tile's clause j.
__device__ inline void open_tile(const BucketDesc *descs, uint32_t n_buckets, uint32_t &bi, uint32_t t, uint32_t j,
                                 uint32_t T, TileRef &tl) {
    while (bi + 1 < n_buckets && t >= descs[bi + 1].tile_begin) ++bi;
    const BucketDesc &d = descs[bi];
    const uint32_t slot = (t - d.tile_begin) * T + j;
    tl.s_log2 = d.stride_log2;
    tl.lits = make_rsrc(d.lits, d.lits_bytes);
    // the tile's codes start at tile * T * S; this clause's first group at j * 16 B
    tl.code_off = (((t - d.tile_begin) * T) << (d.stride_log2 + 2)) + j * 16u;
    const auto m = __builtin_amdgcn_raw_buffer_load_b64(make_rsrc(d.meta, d.meta_bytes), slot * 8u, 0, kStream);
    tl.meta = make_uint2(m[0], m[1]);
    const auto q = __builtin_amdgcn_raw_buffer_load_b128(tl.lits, tl.code_off, 0, kStream);
    tl.c0 = make_uint4(q[0], q[1], q[2], q[3]);
    tl.lowshift = slot & 31u;
    tl.lowword = d.low ? __builtin_amdgcn_raw_buffer_load_b32(make_rsrc(d.low, d.low_bytes), (slot >> 5) * 4u, 0, kStream)
                       : 0u;
}

// The same for a scheduled test, whose wavefronts take the slots of a list
// (only the clauses this run tests) T at a time: chunk c of the run's chunks,
// chunk_begin[b] the first chunk of length class b, count[b] its listed slots.
// Lane j takes list entry (c - chunk_begin[b]) * T + j; past the end it tests
// nothing (length 0).  A listed slot's codes keep their tile layout: its group g
// still lies T * 16 bytes after group g - 1.
__device__ inline void open_listed(const BucketDesc *descs, uint32_t n_buckets, uint32_t &bi, uint32_t c,
                                   const uint32_t *chunk_begin, const uint32_t *count, uint32_t j, uint32_t t_log2,
                                   TileRef &tl) {
    while (bi + 1 < n_buckets && c >= chunk_begin[bi + 1]) ++bi;
    const BucketDesc &d = descs[bi];
    const uint32_t e = ((c - chunk_begin[bi]) << t_log2) + j;
    tl.s_log2 = d.stride_log2;
    tl.lits = make_rsrc(d.lits, d.lits_bytes);
    tl.lowword = 0;
    tl.lowshift = 0;
    tl.meta = make_uint2(0, 0);
    tl.c0 = make_uint4(0, 0, 0, 0);
    tl.code_off = 0;
    if (e < count[bi]) {
        const uint32_t slot = d.list[e];
        const uint32_t tile = slot >> t_log2, jj = slot & ((1u << t_log2) - 1);
        tl.code_off = ((tile << t_log2) << (d.stride_log2 + 2)) + jj * 16u;
        const auto m = __builtin_amdgcn_raw_buffer_load_b64(make_rsrc(d.meta, d.meta_bytes), slot * 8u, 0, kStream);
        tl.meta = make_uint2(m[0], m[1]);
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(tl.lits, tl.code_off, 0, kStream);
        tl.c0 = make_uint4(q[0], q[1], q[2], q[3]);
    }
}

// Plane words of one lane: WPL consecutive 64-slot words.
template <int WPL>
struct Words {
    uint64_t v[WPL];
};

template <int WPL>
__device__ inline Words<WPL> load_words(const char *p) {
    Words<WPL> r;
    if constexpr (WPL == 1) {
        r.v[0] = *reinterpret_cast<const uint64_t *>(p);
    } else if constexpr (WPL == 2) {
        const uint4 a = *reinterpret_cast<const uint4 *>(p);
        r.v[0] = ((uint64_t)a.y << 32) | a.x;
        r.v[1] = ((uint64_t)a.w << 32) | a.z;
    } else {
        const uint4 a = *reinterpret_cast<const uint4 *>(p);
        const uint4 b = *reinterpret_cast<const uint4 *>(p + 16);
        r.v[0] = ((uint64_t)a.y << 32) | a.x;
        r.v[1] = ((uint64_t)a.w << 32) | a.z;
        r.v[2] = ((uint64_t)b.y << 32) | b.x;
        r.v[3] = ((uint64_t)b.w << 32) | b.z;
    }
    return r;
}

// One store's clause test for one lane: LPC lanes per clause, WPL words per lane,
// a plane row of RW = LPC * WPL words.  MODE 0 = falsified, 1 = trigger.
template <int LPC, int WPL, int MODE, bool HOT, bool AGG = false, bool WIDE = false>
struct Tester {
    static constexpr uint32_t kGroup = kGroupOf<AGG>;
    static constexpr uint32_t T = 64 / LPC;                 // clauses per wavefront (and per tile)
    static constexpr uint32_t RW = LPC * WPL;               // words per plane row
    static constexpr uint32_t ROW_SHIFT = ilog2<RW>() + 3;  // bytes per plane row
    // a row's aggregate bits (one per word), as stored by the context
    using AggT = std::conditional_t<(RW <= 16), uint16_t, std::conditional_t<(RW <= 32), uint32_t, uint64_t>>;

    using Tile = TileRef;

    uint32_t j;    // clause of this lane within the tile
    uint32_t w0;   // first word of this lane within a chunk
    uint32_t W;    // words in use
    uint32_t hot_rows;
    uint32_t sched_run;
    uint32_t G;    // chunks of a row (super-groups of 64 words); 1 up to 64 words
    uint64_t act[WPL];  // active words of this lane in chunk 0
    const uint64_t *active;
    const char *pbase;
    uint64_t chunk_bytes;
    const uint64_t *lds;
    const AggT *agg;   // AGG: per chunk and literal code, words with an F slot ([G][n_rows])
    const AggT *aggu;  // AGG in trigger mode: per chunk and variable, words with an active U slot
    const uint64_t *sagg;   // G > 1: per code, super-groups with an F slot
    const uint64_t *saggu;  // G > 1, trigger mode: per variable, super-groups with an active U slot
    uint64_t n_rows;

    __device__ Tester(uint32_t lane, const uint64_t *planes, const uint64_t *active_, uint32_t W_, uint32_t hot_rows_,
                      const uint64_t *lds_, uint32_t sched_run_, const void *agg_, const void *aggu_, uint32_t G_ = 1,
                      uint64_t chunk_elems = 0, uint64_t n_rows_ = 0, const uint64_t *sagg_ = nullptr,
                      const uint64_t *saggu_ = nullptr)
        : j(lane / LPC), w0((lane % LPC) * WPL), W(W_), hot_rows(hot_rows_), sched_run(sched_run_), G(G_),
          active(active_), chunk_bytes(chunk_elems * 8), lds(lds_), agg(static_cast<const AggT *>(agg_)),
          aggu(static_cast<const AggT *>(aggu_)), sagg(sagg_), saggu(saggu_), n_rows(n_rows_) {
#pragma unroll
        for (int i = 0; i < WPL; ++i) act[i] = (w0 + i < W) ? active[w0 + i] : 0;
        pbase = reinterpret_cast<const char *>(planes) + w0 * 8;
    }

    // This lane's words of plane row `code` in the chunk at pb.  Code 0 is the
    // all-ones row, the identity of the AND: literals past a clause's end read it.
    // A hot row is read from LDS through the same generic load: the address is
    // chosen per lane, so a wavefront whose lanes mix hot and cold rows issues one
    // load instead of splitting into an LDS path and a global path.
    __device__ Words<WPL> gather(const char *pb, uint32_t code) const {
        // a one-chunk table stays under 4 GiB: 32-bit row offsets
        const char *p = WIDE ? pb + ((uint64_t)code << ROW_SHIFT) : pb + (code << ROW_SHIFT);
        if constexpr (HOT) {
            if (code < hot_rows) p = reinterpret_cast<const char *>(lds + code * RW + w0);
        }
        return load_words<WPL>(p);
    }

    // cnt.settled += the live words of this wavefront's lanes that `keep` clears
    // (applies: this lane ran the aggregate test); called by every lane alike.
    __device__ static void settled_words(Counts &cnt, const uint64_t *af, const uint64_t *ou, uint32_t keep,
                                         bool applies) {
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            const bool gone = applies && (af[i] | ou[i]) != 0 && !((keep >> i) & 1u);
            cnt.settled += (uint32_t)__builtin_popcountll(__ballot(gone));
        }
    }

    // Locates tile t (bi: bucket cursor, only ever advanced) and issues the loads
    // of this lane's metadata and first four codes.
    __device__ void open(const BucketDesc *descs, uint32_t n_buckets, uint32_t &bi, uint32_t t, Tile &tl) const {
        open_tile(descs, n_buckets, bi, t, j, T, tl);
    }

    // The top level of the aggregate test (G > 1): for this lane's clause, the
    // super-groups (chunks of 64 words) on whose aggregate the clause can be
    // falsified (MODE 0: every literal F in some slot of the super-group) or
    // trigger (MODE 1: the recurrence of Section 4.3 on canBeFalse and
    // canBeUndef), among `groups`.  The lanes of a clause compute the same mask
    // (their loads coincide); the wavefront stops reading literals once every
    // clause's mask is zero.
    __device__ uint64_t super_mask(const Tile &cur, uint64_t groups) const {
        const bool skip = ((cur.lowword >> cur.lowshift) & 1u) && ((sched_run + cur.meta.y) & 3u) != 0;
        const uint32_t len = skip ? 0u : cur.meta.x;
        const uint32_t S = 1u << cur.s_log2;
        uint64_t af = len ? groups : 0ull, ou = 0;
        uint4 c = cur.c0;
        for (uint32_t k = 0;; k += 4) {
            if (!__ballot(k < len && (af | ou) != 0)) break;
            uint4 cn = make_uint4(0, 0, 0, 0);
            if (k + 4 < S) {
                const auto q = __builtin_amdgcn_raw_buffer_load_b128(cur.lits, cur.code_off + ((k + 4) >> 2) * (T * 16u),
                                                                     0, kStream);
                cn = make_uint4(q[0], q[1], q[2], q[3]);
            }
            const uint32_t cs[4] = {c.x, c.y, c.z, c.w};
            // the group's four bit sets are loaded together (past the clause's end,
            // code 0's); once af and ou are zero, further steps keep them zero
            uint64_t cf[4], cu[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t code = k + u < len ? cs[u] : 0u;
                cf[u] = sagg[code];
                if constexpr (MODE == 1) cu[u] = saggu[code >> 1];
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                if (k + u < len) {
                    if constexpr (MODE == 1) ou = (af & cu[u]) | (ou & cf[u]);
                    af &= cf[u];
                }
            }
            c = cn;
        }
        return af | ou;
    }

    // Tests the clauses of an opened tile on chunk g of the rows.  Records go to
    // seg (capacity seg_cap) after the `produced` records already there; returns
    // the new count.  With dense != nullptr, writes each clause's mask row there
    // instead.  sup: the clause's super-group mask (bit g clear: not tested).
    // cnt (when cnt.on): what the wavefront did, added up.
    __device__ uint32_t run(const Tile &cur, gss_report *seg, uint32_t seg_cap, uint32_t produced, uint32_t early_exit,
                            uint64_t *dense, Counts &cnt, uint32_t g = 0, uint64_t sup = ~0ull) const {
        // a low-priority clause sits out the runs where (run + id) % 4 != 0
        const bool skip = ((cur.lowword >> cur.lowshift) & 1u) && ((sched_run + cur.meta.y) & 3u) != 0;
        // chunk g: this lane's words g * RW + w0 .. (a clause whose super-group test
        // was negative for g takes no part)
        const uint32_t len = (skip || !((sup >> g) & 1u)) ? 0u : cur.meta.x;
        const uint32_t S = 1u << cur.s_log2;
        const uint32_t gw0 = WIDE ? g * RW + w0 : w0;
        const bool lane_ok = gw0 < W;
        const char *const pb = WIDE ? pbase + g * chunk_bytes : pbase;
        const AggT *const ag = WIDE ? agg + g * n_rows : agg;
        const AggT *const agu = WIDE ? aggu + g * (n_rows / 2) : aggu;
        uint64_t af[WPL], ou[WPL];  // allFalse, oneUndef (trigger mode)
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            const uint64_t a = WIDE ? (gw0 + i < W ? active[gw0 + i] : 0ull) : act[i];
            af[i] = len ? a : 0;
            ou[i] = 0;
        }
        // aggregate recurrence of the trigger test (Section 4.3), one bit per word of this lane
        uint32_t agg_af = (1u << WPL) - 1u, agg_ou = 0;
        uint4 c = cur.c0;
        for (uint32_t k = 0;; k += 4) {
            {
                uint64_t any = 0;
#pragma unroll
                for (int i = 0; i < WPL; ++i) any |= af[i] | ou[i];
                if (!__ballot(lane_ok && k < len && (!early_exit || any != 0))) break;
            }
            uint4 cn = make_uint4(0, 0, 0, 0);
            if (k + 4 < S) {  // uniform branch: the next four codes, in flight during this group
                // group (k + 4) / 4 of this clause: the tile's groups are T * 16 bytes apart
                const auto q = __builtin_amdgcn_raw_buffer_load_b128(cur.lits, cur.code_off + ((k + 4) >> 2) * (T * 16u),
                                                                     0, kStream);
                cn = make_uint4(q[0], q[1], q[2], q[3]);
            }
            const uint32_t cs[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (uint32_t g0 = 0; g0 < 4; g0 += kGroup) {
                // a lane re-checks its words every kGroup literals; finished lanes issue no loads
                uint64_t any = 0;
#pragma unroll
                for (int i = 0; i < WPL; ++i) any |= af[i] | ou[i];
                bool lane_live = lane_ok && k + g0 < len && (!early_exit || any != 0);
                if constexpr (MODE == 0) {
                    // aggregate pre-test (Section 4): a word where some literal of the
                    // group is F in no slot cannot be falsified; skip the gathers when
                    // that holds for all of this lane's words
                    if (AGG && lane_live) {
                        uint32_t keep = (1u << WPL) - 1u;
#pragma unroll
                        for (uint32_t u = 0; u < kGroup; ++u) {
                            const uint32_t code = (k + g0 + u < len) ? cs[g0 + u] : 0u;
                            keep &= (uint32_t)(ag[code] >> w0);
                        }
                        if (cnt.on) settled_words(cnt, af, af, keep, true);
#pragma unroll
                        for (int i = 0; i < WPL; ++i)
                            if (!((keep >> i) & 1u)) af[i] = 0;
                        lane_live = keep != 0;
                    } else if (AGG && cnt.on) {
                        settled_words(cnt, af, af, 0u, false);  // a lane with no test: every lane joins the ballots
                    }
                } else {
                    // trigger mode: the same recurrence over the group aggregates
                    // (canBeFalse of the literal, canBeUndef of its variable) decides
                    // which words can still trigger (Theorem 1: no false negatives)
                    if (AGG && lane_live) {
#pragma unroll
                        for (uint32_t u = 0; u < kGroup; ++u) {
                            const uint32_t code = (k + g0 + u < len) ? cs[g0 + u] : 0u;
                            const uint32_t cf = (uint32_t)(ag[code] >> w0), cu = (uint32_t)(agu[code >> 1] >> w0);
                            agg_ou = (agg_af & cu) | (agg_ou & cf);
                            agg_af &= cf;
                        }
                        const uint32_t keep = (agg_af | agg_ou) & ((1u << WPL) - 1u);
                        if (cnt.on) settled_words(cnt, af, ou, keep, true);
#pragma unroll
                        for (int i = 0; i < WPL; ++i)
                            if (!((keep >> i) & 1u)) {
                                af[i] = 0;
                                ou[i] = 0;
                            }
                        lane_live = keep != 0;
                    } else if (AGG && cnt.on) {
                        settled_words(cnt, af, ou, 0u, false);
                    }
                }
                if (cnt.on) cnt.gathers += kGroup * (uint32_t)__builtin_popcountll(__ballot(lane_live));
                if (lane_live) {
                    Words<WPL> gf[kGroup], gt[kGroup];
#pragma unroll
                    for (uint32_t u = 0; u < kGroup; ++u) {
                        const uint32_t code = (k + g0 + u < len) ? cs[g0 + u] : 0u;
                        gf[u] = gather(pb, code);
                        if constexpr (MODE == 1) gt[u] = gather(pb, code ^ 1u);
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kGroup; ++u) {
#pragma unroll
                        for (int i = 0; i < WPL; ++i) {
                            if constexpr (MODE == 1) {
                                const uint64_t is_set = gf[u].v[i] | gt[u].v[i];
                                ou[i] = (af[i] & ~is_set) | (ou[i] & gf[u].v[i]);
                            }
                            af[i] &= gf[u].v[i];
                        }
                    }
                }
            }
            c = cn;
        }

        if (dense) {
            if (len) {
#pragma unroll
                for (int i = 0; i < WPL; ++i)
                    if (gw0 + i < W) dense[(uint64_t)cur.meta.y * W + gw0 + i] = af[i] | ou[i];
            }
            return produced;
        }
#pragma unroll
        for (int i = 0; i < WPL; ++i) {
            const uint64_t res = af[i] | ou[i];
            const bool has = res != 0;
            const uint64_t bal = __ballot(has);
            if (has) {
                const uint32_t pos = produced + lanes_below(bal);
                if (pos < seg_cap) {
                    const u32x4 rec = {cur.meta.y, gw0 + i, (uint32_t)res, (uint32_t)(res >> 32)};
                    __builtin_nontemporal_store(rec, reinterpret_cast<u32x4 *>(seg) + pos);
                }
            }
            produced += (uint32_t)__builtin_popcountll(bal);
        }
        return produced;
    }
};

// Called by one workgroup of 1024 threads: exclusive prefix of the records each
// segment kept (min(count, cap)) into offsets[0..n], and summary = {total count,
// largest count, records kept}.  Thread t takes a contiguous share of the
// segments; the shares are combined within each wavefront by shuffles and across
// the 16 wavefronts through LDS (two barriers).
__device__ inline void finalize_segments(const uint32_t *counts, uint32_t n, uint32_t cap, uint64_t *offsets,
                                         unsigned long long *summary) {
    __shared__ unsigned long long wkept[16], wall[16];
    __shared__ unsigned int wmax[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t lo = min(n, tid * per), hi = min(n, lo + per);
    // Up to kHeld counts a thread (16384 segments) are loaded all at once, from
    // addresses clamped into the array, and kept for the second pass; beyond that
    // the thread walks its range twice.
    constexpr uint32_t kHeld = 16;
    const bool held = per <= kHeld;
    uint32_t v[kHeld];
#pragma unroll
    for (uint32_t k = 0; k < kHeld; ++k) v[k] = (held && n) ? counts[min(lo + k, n - 1)] : 0u;
    unsigned long long kept = 0, all = 0;
    unsigned int m = 0;
    if (held) {
#pragma unroll
        for (uint32_t k = 0; k < kHeld; ++k) {
            const uint32_t c = lo + k < hi ? v[k] : 0u;
            kept += min(c, cap);
            all += c;
            m = max(m, c);
        }
    } else {
        for (uint32_t i = lo; i < hi; ++i) {
            const uint32_t c = counts[i];
            kept += min(c, cap);
            all += c;
            m = max(m, c);
        }
    }
    // inclusive scan of kept within the wavefront; sum and max over it
    unsigned long long x = kept, a = all;
    unsigned int mm = m;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const unsigned long long y = __shfl_up(x, d);
        if (lane >= d) x += y;
        a += __shfl_xor(a, d);
        mm = max(mm, (unsigned int)__shfl_xor(mm, d));
    }
    if (lane == 63) wkept[wave] = x;
    if (lane == 0) {
        wall[wave] = a;
        wmax[wave] = mm;
    }
    __syncthreads();
    unsigned long long before = 0, total_kept = 0, total = 0;
    unsigned int mx = 0;
#pragma unroll
    for (uint32_t w = 0; w < 16; ++w) {
        before += w < wave ? wkept[w] : 0ull;
        total_kept += wkept[w];
        total += wall[w];
        mx = max(mx, wmax[w]);
    }
    unsigned long long base = before + x - kept;
    if (held) {
#pragma unroll
        for (uint32_t k = 0; k < kHeld; ++k) {
            if (lo + k < hi) offsets[lo + k] = base;
            base += lo + k < hi ? min(v[k], cap) : 0u;
        }
    } else {
        for (uint32_t i = lo; i < hi; ++i) {
            offsets[i] = base;
            base += min(counts[i], cap);
        }
    }
    if (tid == 0) {
        offsets[n] = total_kept;
        summary[0] = total;
        summary[1] = mx;
        summary[2] = total_kept;
    }
}

}  // namespace gss
