// Assignment bitplanes (Section 3.4): N assignments of a variable as two N-bit
// words.  The paper keeps (isTrue, isSet); this library keeps, per literal code,
// the word of slots where that literal is F:
//   row 2v   = slots where v = F   (isSet & ~isTrue)
//   row 2v+1 = slots where v = T   (isSet &  isTrue)
// so a clause's falsified mask is the AND of one gathered row per literal, and
// the Undef slots of v are the complement of (row 2v | row 2v+1).  The value of
// the isTrue bit for an Undef slot, which the paper leaves open, never enters.
//
// One 64-bit word holds 64 slots, one per lane of a wavefront: the pack kernels
// build each word with two wavefront ballots.
#include "gss_internal.h"

#include <algorithm>
#include <cstring>

namespace gss {

// ---- aggregate bits (Section 4): per row and chunk, bit w = some slot of word
//      w of the chunk has the row's literal F (element g * n_rows + row).  Packed
//      word deltas keep them in step; bulk updates (full sets, var-major deltas,
//      cleared slots) mark them stale, and the next aggregate test rebuilds them.
//      Above them, with more than one chunk, one bit per row and chunk (the
//      super-group: the aggregate of the chunk's word aggregates), rebuilt from
//      the word bits before an aggregate test when they changed.

__device__ inline uint64_t agg_get(const void *agg, uint32_t RWc, uint64_t i) {
    if (RWc <= 16) return reinterpret_cast<const uint16_t *>(agg)[i];
    if (RWc <= 32) return reinterpret_cast<const uint32_t *>(agg)[i];
    return reinterpret_cast<const uint64_t *>(agg)[i];
}

__device__ inline void agg_put(void *agg, uint32_t RWc, uint64_t i, uint64_t bits) {
    if (RWc <= 16)
        reinterpret_cast<uint16_t *>(agg)[i] = (uint16_t)bits;
    else if (RWc <= 32)
        reinterpret_cast<uint32_t *>(agg)[i] = (uint32_t)bits;
    else
        reinterpret_cast<uint64_t *>(agg)[i] = bits;
}

// bit w = word w of chunk g of the row is nonzero
__device__ inline uint64_t row_nonzero_words(const uint64_t *planes, uint32_t RWc, uint64_t chunk, uint32_t g,
                                             uint64_t row) {
    const uint64_t *p = planes + g * chunk + row * RWc;
    uint64_t bits = 0;
    for (uint32_t w = 0; w < RWc; ++w) bits |= (uint64_t)(p[w] != 0) << w;
    return bits;
}

// Thread per (chunk, row) of rows [lo, hi).  Aggregates are stored [G][n_rows].
__global__ void k_agg_rows(const uint64_t *planes, uint32_t RWc, uint64_t chunk, uint32_t G, uint64_t n_rows, void *agg,
                           uint64_t lo, uint64_t hi) {
    const uint64_t span = hi - lo, total = span * G;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t g = (uint32_t)(x / span);
        const uint64_t r = lo + x % span;
        agg_put(agg, RWc, g * n_rows + r, row_nonzero_words(planes, RWc, chunk, g, r));
    }
}

// Trigger-mode aggregate of each variable: bit w = some active slot of word w
// has the variable U (neither row set there); thread per (chunk, variable),
// stored [G][n_vars + 1].
__global__ void k_aggu_rows(const uint64_t *planes, uint32_t RWc, uint64_t chunk, uint32_t G, const uint64_t *active,
                            uint32_t W, void *aggu, uint64_t n_vars1) {
    const uint64_t total = n_vars1 * G;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t g = (uint32_t)(x / n_vars1);
        const uint64_t v = x % n_vars1;
        const uint64_t *pf = planes + g * chunk + (2 * v) * RWc, *pt = pf + RWc;
        uint64_t bits = 0;
        for (uint32_t w = 0; w < RWc; ++w) {
            const uint32_t gw = g * RWc + w;
            const uint64_t act = gw < W ? active[gw] : 0ull;
            bits |= (uint64_t)(((pf[w] | pt[w]) & act) != act) << w;
        }
        agg_put(aggu, RWc, g * n_vars1 + v, bits);
    }
}

// Super-group bits (G > 1): bit g of out[i] = the 64-word aggregate in[g][i] is nonzero.
__global__ void k_super_bits(const uint64_t *in, uint32_t G, uint64_t n, uint64_t *out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t bits = 0;
        for (uint32_t g = 0; g < G; ++g) bits |= (uint64_t)(in[g * n + i] != 0) << g;
        out[i] = bits;
    }
}

void aggu_rebuild(Ctx &c) {
    const uint64_t n = (uint64_t)c.cfg.num_vars + 1;
    if (!c.aggu) c.aggu = c.dalloc((uint64_t)c.G * n * agg_elem_bytes(c.RWc));
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n * c.G + 255) / 256, 65536));
    hipLaunchKernelGGL(k_aggu_rows, dim3(grid), dim3(256), 0, c.stream, c.planes, c.RWc, c.chunk_elems, c.G, c.active,
                       c.W, c.aggu, n);
    GSS_HIP(hipGetLastError());
    c.aggu_valid = true;
    c.saggu_valid = false;
}

void agg_rebuild(Ctx &c, uint64_t lo, uint64_t hi) {
    if (hi <= lo) return;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(((hi - lo) * c.G + 255) / 256, 65536));
    hipLaunchKernelGGL(k_agg_rows, dim3(grid), dim3(256), 0, c.stream, c.planes, c.RWc, c.chunk_elems, c.G, c.n_rows,
                       c.agg, lo, hi);
    GSS_HIP(hipGetLastError());
    c.sagg_valid = false;
}

void super_rebuild(Ctx &c, bool with_u) {
    if (c.G == 1) return;
    if (!c.sagg_valid) {
        hipLaunchKernelGGL(k_super_bits, dim3(fill_grid(c.n_rows)), dim3(256), 0, c.stream,
                           (const uint64_t *)c.agg, c.G, c.n_rows, c.sagg);
        GSS_HIP(hipGetLastError());
        c.sagg_valid = true;
    }
    if (with_u && !c.saggu_valid) {
        const uint64_t n = (uint64_t)c.cfg.num_vars + 1;
        if (!c.saggu) c.saggu = (uint64_t *)c.dalloc(n * 8);
        hipLaunchKernelGGL(k_super_bits, dim3(fill_grid(n)), dim3(256), 0, c.stream, (const uint64_t *)c.aggu, c.G, n,
                           c.saggu);
        GSS_HIP(hipGetLastError());
        c.saggu_valid = true;
    }
}

// Packs the slots of word w from a slot-major staging block.  One wavefront per
// 64 variables; lane b reads slot 64*w + b.  Staging row r holds slot s_lo + r,
// `pitch` bytes per row (a multiple of 64), byte v-1 = value of variable v.
__global__ __launch_bounds__(64) void k_pack_word(uint64_t *planes, uint32_t RWc, uint64_t chunk, uint32_t w,
                                                  uint32_t num_vars,
                                                  const int8_t *stage, uint64_t pitch, uint32_t s_lo, uint32_t s_hi,
                                                  const uint32_t *bad, const uint32_t *perm) {
    if (*bad) return;  // the inputs failed validation: apply nothing
    const uint32_t lane = threadIdx.x;
    const uint32_t v0 = 1 + 64 * blockIdx.x;
    const uint32_t slot = 64 * w + lane;
    const bool in = slot >= s_lo && slot < s_hi;
    uint4 q[4] = {};
    if (in) {
        const uint4 *src = reinterpret_cast<const uint4 *>(stage + (uint64_t)(slot - s_lo) * pitch + (v0 - 1));
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = src[i];
    }
    const uint32_t r[16] = {q[0].x, q[0].y, q[0].z, q[0].w, q[1].x, q[1].y, q[1].z, q[1].w,
                            q[2].x, q[2].y, q[2].z, q[2].w, q[3].x, q[3].y, q[3].z, q[3].w};
    const uint64_t sm = __ballot(in);
    uint64_t f = 0, t = 0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        const uint32_t byte = (r[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        const uint64_t bf = __ballot(byte == 0xFFu);  // -1: F
        const uint64_t bt = __ballot(byte == 0x01u);  // +1: T
        if (lane == (uint32_t)j) {
            f = bf;
            t = bt;
        }
    }
    const uint32_t v = v0 + lane;
    if (v <= num_vars) {
        const uint64_t r0 = plane_index(2ull * internal_var(perm, v), w, RWc, chunk), r1 = r0 + RWc;
        if (sm != ~0ull) {
            f = (planes[r0] & ~sm) | (f & sm);
            t = (planes[r1] & ~sm) | (t & sm);
        }
        planes[r0] = f;
        planes[r1] = t;
    }
}

// Delta update: thread per (variable, 64-slot word), the words of one variable
// on neighbouring lanes, so that a variable's plane rows are written as whole
// lines and its values read as one contiguous run.  The thread reads the word's
// 64 values of its variable (four 16-byte loads when the word is whole and
// aligned) and builds the F and T words; a word only partly inside
// [first, first + n_slots) keeps its other slots.  vals is var-major
// [n_vars][n_slots]; nw = words touched.
// With clear_bits != null, the thread of each variable's first word also clears
// the variable's word of the duplicate bitmap (left zero for the next check).
__global__ __launch_bounds__(256) void k_set_vars(uint64_t *planes, uint32_t RWc, uint64_t chunk, const uint32_t *vars,
                                                  uint32_t n_vars,
                                                  const int8_t *vals, uint32_t first, uint32_t n_slots, uint32_t nw,
                                                  const uint32_t *bad, uint32_t *clear_bits, const uint32_t *perm) {
    const uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (x >= (uint64_t)n_vars * nw) return;
    const uint32_t i = (uint32_t)(x / nw);
    const uint32_t wi = (uint32_t)(x - (uint64_t)i * nw);
    if (clear_bits && wi == 0) clear_bits[vars[i] >> 5] = 0;
    if (*bad) return;  // the inputs failed validation: apply nothing
    const uint32_t w = first / 64 + wi;
    const uint32_t lo = max(first, 64 * w), hi = min(first + n_slots, 64 * w + 64);
    const int8_t *src = vals + (uint64_t)i * n_slots + (lo - first);
    uint64_t f = 0, t = 0;
    if (hi - lo == 64 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 v = reinterpret_cast<const uint4 *>(src)[q];
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t b = (u[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                f |= (uint64_t)(b == 0xFFu) << (16 * q + k);
                t |= (uint64_t)(b == 0x01u) << (16 * q + k);
            }
        }
    } else {
        for (uint32_t s = lo; s < hi; ++s) {
            const int8_t x = src[s - lo];
            f |= (uint64_t)(x == -1) << (s - 64 * w);
            t |= (uint64_t)(x == 1) << (s - 64 * w);
        }
    }
    const uint64_t r0 = plane_index(2ull * internal_var(perm, vars[i]), w, RWc, chunk), r1 = r0 + RWc;
    if (hi - lo != 64) {
        const uint64_t sm = ((1ull << (hi - lo)) - 1) << (lo - 64 * w);  // hi - lo < 64 here
        f = (planes[r0] & ~sm) | (f & sm);
        t = (planes[r1] & ~sm) | (t & sm);
    }
    planes[r0] = f;
    planes[r1] = t;
}

// Packed delta: new plane words of listed variables in one 64-slot word.  Thread
// per variable; f = slots where the variable is F, t = slots where it is T.
// The variables of one launch are distinct, so each thread owns its two rows'
// aggregate bits (bit `word` of the word's chunk), updated in place.
__global__ void k_set_words(uint64_t *planes, uint32_t RWc, uint64_t chunk, uint64_t n_rows, uint32_t word,
                            const uint32_t *vars, const uint64_t *f, const uint64_t *t, uint32_t n, void *agg,
                            const uint32_t *perm) {
    const uint64_t a_base = (uint64_t)(word / kChunkWords) * n_rows;
    const uint64_t bit = 1ull << (word % kChunkWords);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t row = 2ull * internal_var(perm, vars[i]);
        const uint64_t r0 = plane_index(row, word, RWc, chunk);
        planes[r0] = f[i];
        planes[r0 + RWc] = t[i];
        const uint64_t a0 = agg_get(agg, RWc, a_base + row), a1 = agg_get(agg, RWc, a_base + row + 1);
        agg_put(agg, RWc, a_base + row, f[i] ? (a0 | bit) : (a0 & ~bit));
        agg_put(agg, RWc, a_base + row + 1, t[i] ? (a1 | bit) : (a1 & ~bit));
    }
}

// Clears slots [first, first+n) in every row of real variables (rows >= 2).
__global__ void k_clear_slots(uint64_t *planes, uint32_t RWc, uint64_t chunk, uint64_t n_rows, uint32_t first,
                              uint32_t n_slots) {
    const uint32_t w_lo = first / 64, w_hi = (first + n_slots - 1) / 64, nw = w_hi - w_lo + 1;
    const uint64_t total = (n_rows - 2) * nw;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t row = 2 + x / nw;
        const uint32_t w = w_lo + (uint32_t)(x % nw);
        const uint32_t a = std::max(first, 64 * w), b = std::min(first + n_slots, 64 * w + 64);
        const uint64_t sm = (b - a == 64) ? ~0ull : (((1ull << (b - a)) - 1) << (a - 64 * w));
        planes[plane_index(row, w, RWc, chunk)] &= ~sm;
    }
}

void launch_set_words(Ctx &c, uint32_t word, const uint32_t *vars, const uint64_t *f, const uint64_t *t, uint32_t n) {
    if (n == 0) return;
    c.aggu_valid = false;
    c.sagg_valid = false;
    const unsigned grid = std::max<uint32_t>(1, std::min<uint32_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_set_words, dim3(grid), dim3(256), 0, c.stream, c.planes, c.RWc, c.chunk_elems, c.n_rows, word,
                       vars, f, t, n, c.agg, c.d_perm);
    GSS_HIP(hipGetLastError());
    c.mutations++;
}

static uint64_t slot_mask(uint32_t first, uint32_t n, uint32_t w) {
    const uint32_t a = std::max(first, 64 * w), b = std::min(first + n, 64 * w + 64);
    if (b <= a) return 0;
    return (b - a == 64) ? ~0ull : (((1ull << (b - a)) - 1) << (a - 64 * w));
}

__global__ void k_copy_words(const uint64_t *src, uint64_t *dst, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// The active words go up by a kernel reading the pinned ring slot: a queued DMA
// copy would start only after the test before it and then hold up the next one.
static void upload_active(Ctx &c) {
    c.aggu_valid = false;  // U counts active slots only
    const Ctx::Staged st = c.stage_upload(c.W * 8);
    std::memcpy(st.h, c.h_active.data(), c.W * 8);
    hipLaunchKernelGGL(k_copy_words, dim3((c.W + 255) / 256), dim3(256), 0, c.stream, (const uint64_t *)st.hd, c.active,
                       c.W);
    GSS_HIP(hipGetLastError());
    c.stage_done(st);
}

// Range and distinctness of a variable list, O(n) with a bitmap that is cleared
// again afterwards.
static void check_vars(Ctx &c, const uint32_t *vars, uint32_t n_vars) {
    std::vector<uint64_t> &seen = c.var_seen;
    if (seen.size() < (uint64_t)c.cfg.num_vars / 64 + 1) seen.assign((uint64_t)c.cfg.num_vars / 64 + 1, 0);
    uint32_t bad = 0;  // 1: out of range, 2: repeated
    uint32_t i = 0;
    for (; i < n_vars; ++i) {
        const uint32_t v = vars[i];
        if (v < 1 || v > c.cfg.num_vars) { bad = 1; break; }
        uint64_t &word = seen[v >> 6];
        const uint64_t bit = 1ull << (v & 63);
        if (word & bit) { bad = 2; break; }
        word |= bit;
    }
    for (uint32_t k = 0; k < i; ++k) seen[vars[k] >> 6] = 0;
    GSS_REQUIRE(bad != 1, GSS_ERR_BAD_LITERAL, "variable out of range");
    GSS_REQUIRE(bad != 2, GSS_ERR_INVALID_ARG, "variable listed twice");
}

// Every listed variable in 1..num_vars (the cheap half of check_vars).
static void check_var_range(const Ctx &c, const uint32_t *vars, uint32_t n_vars) {
    uint32_t bad = 0;
    const uint32_t V = c.cfg.num_vars;
    for (uint32_t i = 0; i < n_vars; ++i) bad |= (uint32_t)(vars[i] - 1u >= V);
    GSS_REQUIRE(!bad, GSS_ERR_BAD_LITERAL, "variable out of range");
}

// Device half of the variable check: a variable listed twice sets bit 2 of
// *bad (one bitmap bit per variable, cleared again by k_set_vars).
__global__ void k_check_vars(const uint32_t *vars, uint32_t n, uint32_t *bits, uint32_t *bad) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = vars[i], m = 1u << (v & 31);
    if (atomicOr(&bits[v >> 5], m) & m) atomicOr(bad, 2u);
}

// Both checks of a queued delta in one launch: the first var_blocks workgroups
// take the variable list (already on the device), marking repeats (bit 2 of
// *bad); the others check the truth values (bit 1).
__global__ __launch_bounds__(256) void k_check_delta(const int8_t *vals, uint64_t n_vals, uint32_t var_blocks,
                                                     const uint32_t *vars, uint32_t n, uint32_t *bits, uint32_t *bad) {
    if (blockIdx.x >= var_blocks) {
        const uint32_t b = blockIdx.x - var_blocks, value_blocks = gridDim.x - var_blocks;
        if (values_invalid(vals, n_vals, b * (uint64_t)blockDim.x + threadIdx.x, (uint64_t)value_blocks * blockDim.x))
            atomicOr(bad, 1u);
        return;
    }
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = vars[i], m = 1u << (v & 31);
    if (atomicOr(&bits[v >> 5], m) & m) atomicOr(bad, 2u);
}


static void launch_set_vars(Ctx &c, const uint32_t *d_vars, uint32_t n_vars, const int8_t *d_vals, uint32_t first_slot,
                            uint32_t n_slots, const uint32_t *bad, uint32_t *clear_bits) {
    const uint32_t nw = (first_slot + n_slots - 1) / 64 - first_slot / 64 + 1;
    const uint64_t threads = (uint64_t)n_vars * nw;
    hipLaunchKernelGGL(k_set_vars, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, c.stream, c.planes, c.RWc,
                       c.chunk_elems, d_vars, n_vars, d_vals, first_slot, n_slots, nw, bad, clear_bits, c.d_perm);
    GSS_HIP(hipGetLastError());
}

// Checks shared by both forms of gss_set_var_values: the slot range and its activity.
static void check_delta_slots(const Ctx &c, uint32_t first_slot, uint32_t n_slots) {
    GSS_REQUIRE((uint64_t)first_slot + n_slots <= c.cfg.max_slots, GSS_ERR_CAPACITY, "slot range beyond max_slots");
    for (uint32_t w = first_slot / 64; w <= (first_slot + n_slots - 1) / 64; ++w) {
        const uint64_t sm = slot_mask(first_slot, n_slots, w);
        GSS_REQUIRE((c.h_active[w] & sm) == sm, GSS_ERR_INVALID_ARG, "slot range includes inactive slots");
    }
}

static void check_values_host(const int8_t *v, uint64_t n) {
    uint8_t bad = 0;
    for (uint64_t i = 0; i < n; ++i) bad |= (uint8_t)((uint8_t)(v[i] + 1) > 2);
    GSS_REQUIRE(!bad, GSS_ERR_INVALID_ARG, "truth values must be -1, 0 or +1");
}

}  // namespace gss

using namespace gss;

extern "C" gss_status gss_set_assignments(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots, const int8_t *values) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;  // a test in flight no longer sees the current state
    Ctx &c = *c_;
    if (n_slots == 0) return GSS_OK;
    GSS_REQUIRE(values != nullptr, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE((uint64_t)first_slot + n_slots <= c.cfg.max_slots, GSS_ERR_CAPACITY, "slot range beyond max_slots");
    const uint64_t V = c.cfg.num_vars;
    const bool dev = is_device_pointer(values);
    const uint32_t *bad = c.dsmall + 1;  // always zero
    if (dev)
        bad = queue_value_check(c, values, (uint64_t)n_slots * V);
    else
        check_values_host(values, (uint64_t)n_slots * V);

    const uint64_t pitch = (V + 63) / 64 * 64;
    const uint32_t last = first_slot + n_slots;
    int8_t *stage = (int8_t *)c.device_stage(64 * pitch);
    for (uint32_t w = first_slot / 64; w <= (last - 1) / 64; ++w) {
        const uint32_t s_lo = std::max(first_slot, 64 * w), s_hi = std::min(last, 64 * w + 64);
        const int8_t *src = values + (uint64_t)(s_lo - first_slot) * V;
        GSS_HIP(hipMemcpy2DAsync(stage, pitch, src, V, V, s_hi - s_lo,
                                 dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c.stream));
        hipLaunchKernelGGL(k_pack_word, dim3((unsigned)((V + 63) / 64)), dim3(64), 0, c.stream, c.planes, c.RWc,
                           c.chunk_elems, w, (uint32_t)V, stage, pitch, s_lo, s_hi, bad, c.d_perm);
        GSS_HIP(hipGetLastError());
    }
    if (dev) check_flag(c);  // throws, having applied nothing, if a value was invalid
    c.agg_valid = false;
    c.aggu_valid = false;
    for (uint32_t w = first_slot / 64; w <= (last - 1) / 64; ++w) c.h_active[w] |= slot_mask(first_slot, n_slots, w);
    upload_active(c);
    c.sync();  // host inputs are read by the copies above: done before returning
    GSS_API_END
}

extern "C" gss_status gss_set_var_values(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots, uint32_t n_vars,
                                         const uint32_t *vars, const int8_t *values) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;  // a test in flight no longer sees the current state
    Ctx &c = *c_;
    if (n_slots == 0 || n_vars == 0) return GSS_OK;
    GSS_REQUIRE(vars && values, GSS_ERR_INVALID_ARG, "null argument");
    check_delta_slots(c, first_slot, n_slots);
    const uint64_t nv = (uint64_t)n_vars * n_slots;
    const bool dev = is_device_pointer(values);
    const uint32_t *bad = c.dsmall + 1;  // always zero
    if (dev) {
        // device values are checked on the device, and so are repeated variables:
        // one synchronisation at the end reports either
        check_var_range(c, vars, n_vars);
        bad = queue_value_check(c, values, nv);
        if (!c.var_bits) {
            c.var_bits = (uint32_t *)c.dalloc(((uint64_t)c.cfg.num_vars / 32 + 1) * 4);
            launch_fill_u32(c, c.var_bits, (uint64_t)c.cfg.num_vars / 32 + 1, 0);
        }
    } else {
        check_vars(c, vars, n_vars);
        check_values_host(values, nv);
    }

    const size_t vars_bytes = ((size_t)n_vars * 4 + 255) / 256 * 256;
    const size_t bytes = vars_bytes + (dev ? 0 : nv);
    const Ctx::Staged st = c.stage_upload(bytes);
    char *h = st.h, *d = st.d;
    std::memcpy(h, vars, (size_t)n_vars * 4);
    if (!dev) std::memcpy(h + vars_bytes, values, nv);
    GSS_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c.stream));
    const int8_t *dvals = dev ? values : (const int8_t *)(d + vars_bytes);
    if (dev) {
        hipLaunchKernelGGL(k_check_vars, dim3((n_vars + 255) / 256), dim3(256), 0, c.stream, (const uint32_t *)d, n_vars,
                           c.var_bits, c.dsmall);
        GSS_HIP(hipGetLastError());
    }
    launch_set_vars(c, (const uint32_t *)d, n_vars, dvals, first_slot, n_slots, bad, dev ? c.var_bits : nullptr);
    c.agg_valid = false;
    c.aggu_valid = false;
    c.stage_done(st);
    if (dev) check_flag(c);  // one synchronisation: device inputs are fully read when the call returns
    GSS_API_END
}

extern "C" gss_status gss_set_var_values_async(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots, uint32_t n_vars,
                                               const uint32_t *vars, const int8_t *values) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;  // a test in flight no longer sees the current state
    Ctx &c = *c_;
    if (n_slots == 0 || n_vars == 0) return GSS_OK;
    GSS_REQUIRE(vars && values, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(is_device_pointer(values), GSS_ERR_INVALID_ARG, "values must be device memory");
    check_delta_slots(c, first_slot, n_slots);
    check_var_range(c, vars, n_vars);
    if (!c.var_bits) {
        c.var_bits = (uint32_t *)c.dalloc(((uint64_t)c.cfg.num_vars / 32 + 1) * 4);
        launch_fill_u32(c, c.var_bits, (uint64_t)c.cfg.num_vars / 32 + 1, 0);
    }
    // the list goes up through a pinned ring slot on the copy stream, which runs
    // while the test ahead of it executes (on the context stream, a copy would
    // start only when that test ends); the checking kernel waits for it
    if (!c.copy_stream) {
        GSS_HIP(hipStreamCreateWithFlags(&c.copy_stream, hipStreamNonBlocking));
        GSS_HIP(hipEventCreateWithFlags(&c.ev_copy, hipEventDisableTiming));
    }
    const size_t bytes = (size_t)n_vars * 4;
    const Ctx::Staged st = c.stage_upload(bytes);
    std::memcpy(st.h, vars, bytes);
    uint32_t *dv = (uint32_t *)st.d;
    GSS_HIP(hipMemcpyAsync(dv, st.h, bytes, hipMemcpyHostToDevice, c.copy_stream));
    GSS_HIP(hipEventRecord(c.ev_copy, c.copy_stream));
    GSS_HIP(hipStreamWaitEvent(c.stream, c.ev_copy, 0));
    uint32_t *bad = deferred_flag(c);  // sticky: set by this check or an earlier one not yet reported
    const uint64_t nv = (uint64_t)n_vars * n_slots;
    const uint32_t var_blocks = (n_vars + 255) / 256;
    hipLaunchKernelGGL(k_check_delta, dim3(var_blocks + fill_grid((nv + 15) / 16)), dim3(256), 0, c.stream, values, nv,
                       var_blocks, dv, n_vars, c.var_bits, bad);
    GSS_HIP(hipGetLastError());
    launch_set_vars(c, dv, n_vars, values, first_slot, n_slots, bad, c.var_bits);
    c.agg_valid = false;
    c.aggu_valid = false;
    c.stage_done(st);
    GSS_API_END
}

extern "C" gss_status gss_clear_slots(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;  // a test in flight no longer sees the current state
    Ctx &c = *c_;
    if (n_slots == 0) return GSS_OK;
    GSS_REQUIRE((uint64_t)first_slot + n_slots <= c.cfg.max_slots, GSS_ERR_CAPACITY, "slot range beyond max_slots");
    const uint64_t n_rows = 2ull * ((uint64_t)c.cfg.num_vars + 1);
    const uint64_t nw = (first_slot + n_slots - 1) / 64 - first_slot / 64 + 1;
    const uint64_t total = (n_rows - 2) * nw;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((total + 255) / 256, 16384));
    hipLaunchKernelGGL(k_clear_slots, dim3(grid), dim3(256), 0, c.stream, c.planes, c.RWc, c.chunk_elems, n_rows,
                       first_slot, n_slots);
    GSS_HIP(hipGetLastError());
    c.agg_valid = false;
    c.aggu_valid = false;
    for (uint32_t w = first_slot / 64; w <= (first_slot + n_slots - 1) / 64; ++w)
        c.h_active[w] &= ~slot_mask(first_slot, n_slots, w);
    upload_active(c);
    GSS_API_END
}

extern "C" gss_status gss_update_words(gss_ctx *ctx, uint32_t word, uint32_t n_vars, const uint32_t *vars,
                                       const uint64_t *f_words, const uint64_t *t_words) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;  // a test in flight no longer sees the current state
    Ctx &c = *c_;
    if (n_vars == 0) return GSS_OK;
    GSS_REQUIRE(vars && f_words && t_words, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(word < c.W, GSS_ERR_CAPACITY, "word beyond max_slots / 64");
    check_vars(c, vars, n_vars);
    for (uint32_t i = 0; i < n_vars; ++i)
        GSS_REQUIRE((f_words[i] & t_words[i]) == 0, GSS_ERR_INVALID_ARG, "a slot cannot be both F and T");
    const size_t vb = ((size_t)n_vars * 4 + 255) / 256 * 256, wb = ((size_t)n_vars * 8 + 255) / 256 * 256;
    const Ctx::Staged st = c.stage_upload(vb + 2 * wb);
    char *h = st.h, *d = st.d;
    std::memcpy(h, vars, (size_t)n_vars * 4);
    std::memcpy(h + vb, f_words, (size_t)n_vars * 8);
    std::memcpy(h + vb + wb, t_words, (size_t)n_vars * 8);
    GSS_HIP(hipMemcpyAsync(d, h, vb + 2 * wb, hipMemcpyHostToDevice, c.stream));
    launch_set_words(c, word, (const uint32_t *)d, (const uint64_t *)(d + vb), (const uint64_t *)(d + vb + wb), n_vars);
    c.stage_done(st);
    GSS_API_END
}

extern "C" gss_status gss_set_active(gss_ctx *ctx, const uint64_t *active) {
    GSS_API_BEGIN(ctx)
    c_->mutations++;  // a test in flight no longer sees the current state
    Ctx &c = *c_;
    GSS_REQUIRE(active != nullptr, GSS_ERR_INVALID_ARG, "null argument");
    std::memcpy(c.h_active.data(), active, c.W * 8);
    upload_active(c);
    GSS_API_END
}

extern "C" gss_status gss_update_vars(gss_ctx *ctx, uint32_t word, uint32_t n_vars, const uint32_t *vars,
                                      const uint64_t *fp_words, const uint64_t *fn_words) {
    return gss_update_words(ctx, word, n_vars, vars, fp_words, fn_words);
}
