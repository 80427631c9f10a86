// Hot-variable ranking for LDS staging.  The Conclusion (Section 7) proposes
// keeping the values of some variables in shared memory; which ones pays is a
// property of the clauses, not of how the caller numbered its variables.  The
// library therefore counts, on the device, how often each variable occurs in
// the live clauses and renumbers its variables internally so that the most
// frequent ones own the lowest plane rows, the rows the test kernel stages in
// LDS.  The renumbering is invisible at the ABI: callers keep their variable
// numbers and clause ids; codes and plane rows use internal numbers, and every
// entry point that names variables maps them (`perm`, external -> internal).
//
// A ranking moves as little as it can: the H most frequent variables take
// internal numbers 1..H in order of frequency, the variables they displace take
// the numbers left free, and every other variable keeps its number.  Only the
// plane rows of moved variables are copied; the stored codes are rewritten in
// one pass over each length class.
#include "gss_internal.h"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace gss {

// Thread per stored code position of one length class: counts the variables
// of the live clauses' literals (length 0 = removed; positions past a clause's
// length hold padding).
__global__ void k_count_vars(const uint32_t *lits, const uint2 *meta, uint32_t s_log2, uint32_t t_log2,
                             uint64_t n_slots, uint32_t *counts) {
    const uint64_t total = n_slots << s_log2;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t slot = x >> s_log2;
        const uint32_t k = (uint32_t)(x & ((1ull << s_log2) - 1));
        if (k < meta[slot].x) atomicAdd(&counts[lits[code_index(slot, k, s_log2, t_log2)] >> 1], 1u);
    }
}

// Rewrites every code of a length class through remap (internal variable old ->
// new; remap[0] = 0 keeps the padding code).
__global__ void k_remap_codes(uint32_t *lits, uint64_t n, const uint32_t *remap) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = lits[x];
        lits[x] = (remap[c >> 1] << 1) | (c & 1u);
    }
}

// The two plane rows of each moved variable, all chunks: out = rows of
// vars[i] (to = 0), or rows of vars[i] = in (to = 1).  tmp holds [n][G][2][RWc].
__global__ void k_move_rows(uint64_t *planes, uint32_t RWc, uint64_t chunk, uint32_t G, const uint32_t *vars,
                            uint32_t n, uint64_t *tmp, uint32_t to) {
    const uint64_t per = (uint64_t)G * 2 * RWc;
    const uint64_t total = (uint64_t)n * per;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total; x += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = x / per, r = x % per;
        const uint32_t g = (uint32_t)(r / (2 * RWc)), h = (uint32_t)(r % (2 * RWc));
        uint64_t *p = planes + g * chunk + 2ull * vars[i] * RWc + h;
        if (to)
            *p = tmp[x];
        else
            tmp[x] = *p;
    }
}

bool rank_vars(Ctx &c) {
    if (c.hot_rows < 4 || c.G != 1) return false;  // nothing is staged
    const uint32_t V = c.cfg.num_vars;
    const uint32_t H = std::min<uint32_t>(c.hot_rows / 2 - 1, V);  // variables 1..H are staged
    uint64_t lits = 0;
    for (const Bucket &B : c.buckets) lits += B.n_lits;
    c.ranked_lits = lits;
    if (lits == 0) return false;

    // ---- occurrences per internal variable, on the device
    const size_t counts_bytes = ((size_t)V + 1) * 4;
    uint32_t *d_counts = (uint32_t *)c.device_stage(counts_bytes);
    launch_fill_u32(c, d_counts, (uint64_t)V + 1, 0);
    uint32_t t_log2 = 0;
    while ((1u << t_log2) < c.T) ++t_log2;
    for (const Bucket &B : c.buckets) {
        if (B.n_slots == 0 || B.n_dead == B.n_slots) continue;
        hipLaunchKernelGGL(k_count_vars, dim3(fill_grid(B.n_slots << B.stride_log2)), dim3(256), 0, c.stream, B.lits,
                           B.meta, B.stride_log2, t_log2, B.n_slots, d_counts);
        GSS_HIP(hipGetLastError());
    }
    std::vector<uint32_t> counts((size_t)V + 1);
    GSS_HIP(hipMemcpyAsync(counts.data(), d_counts, counts_bytes, hipMemcpyDeviceToHost, c.stream));
    c.sync();

    // ---- the H most frequent (the lower internal number among equals) take 1..H
    std::vector<uint32_t> order(V);
    std::iota(order.begin(), order.end(), 1u);
    std::partial_sort(order.begin(), order.begin() + H, order.end(), [&](uint32_t a, uint32_t b) {
        return counts[a] != counts[b] ? counts[a] > counts[b] : a < b;
    });
    c.hot_lits = 0;
    for (uint32_t r = 0; r < H; ++r) c.hot_lits += counts[order[r]];
    std::vector<uint32_t> moved_from, moved_to;  // internal old -> new, moved variables only
    std::vector<char> hot((size_t)V + 1, 0);
    for (uint32_t r = 0; r < H; ++r) hot[order[r]] = 1;
    std::vector<uint32_t> vacant, displaced;  // numbers above H freed by hot variables; cold variables in 1..H
    for (uint32_t r = 0; r < H; ++r) {
        const uint32_t v = order[r];
        if (v != r + 1) {
            moved_from.push_back(v);
            moved_to.push_back(r + 1);
        }
        if (v > H) vacant.push_back(v);
    }
    for (uint32_t v = 1; v <= H; ++v)
        if (!hot[v]) displaced.push_back(v);
    std::sort(vacant.begin(), vacant.end());
    for (size_t i = 0; i < displaced.size(); ++i) {  // as many as vacant
        moved_from.push_back(displaced[i]);
        moved_to.push_back(vacant[i]);
    }
    if (moved_from.empty()) return false;  // already ranked

    // ---- the host map, then the device: remap table, codes, plane rows
    std::vector<uint32_t> remap((size_t)V + 1);
    std::iota(remap.begin(), remap.end(), 0u);
    for (size_t i = 0; i < moved_from.size(); ++i) remap[moved_from[i]] = moved_to[i];
    const uint32_t n_mv = (uint32_t)moved_from.size();
    const uint64_t per = (uint64_t)c.G * 2 * c.RWc;
    const size_t remap_bytes = ((size_t)V + 1) * 4;
    const size_t list_bytes = ((size_t)n_mv * 4 + 255) / 256 * 256;
    const size_t tmp_bytes = (size_t)n_mv * per * 8;
    // one staging block: remap | old numbers | new numbers | row copies
    const size_t remap_pad = (remap_bytes + 255) / 256 * 256;
    char *d = (char *)c.device_stage(remap_pad + 2 * list_bytes + tmp_bytes);
    uint32_t *d_remap = (uint32_t *)d;
    uint32_t *d_from = (uint32_t *)(d + remap_pad), *d_to = (uint32_t *)(d + remap_pad + list_bytes);
    uint64_t *d_tmp = (uint64_t *)(d + remap_pad + 2 * list_bytes);
    char *h = (char *)c.host_stage(2 * remap_pad + 2 * list_bytes);  // the map, the lists, then the new perm
    std::memcpy(h, remap.data(), remap_bytes);
    if (n_mv) {  // (empty lists may hold no storage at all)
        std::memcpy(h + remap_pad, moved_from.data(), (size_t)n_mv * 4);
        std::memcpy(h + remap_pad + list_bytes, moved_to.data(), (size_t)n_mv * 4);
    }
    GSS_HIP(hipMemcpyAsync(d, h, remap_pad + 2 * list_bytes, hipMemcpyHostToDevice, c.stream));
    for (Bucket &B : c.buckets) {
        if (B.cap_slots == 0) continue;
        const uint64_t n = B.cap_slots << B.stride_log2;
        hipLaunchKernelGGL(k_remap_codes, dim3(fill_grid(n)), dim3(256), 0, c.stream, B.lits, n, d_remap);
        GSS_HIP(hipGetLastError());
    }
    const unsigned rows_grid = fill_grid((uint64_t)n_mv * per);
    hipLaunchKernelGGL(k_move_rows, dim3(rows_grid), dim3(256), 0, c.stream, c.planes, c.RWc, c.chunk_elems, c.G,
                       d_from, n_mv, d_tmp, 0u);
    GSS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_move_rows, dim3(rows_grid), dim3(256), 0, c.stream, c.planes, c.RWc, c.chunk_elems, c.G,
                       d_to, n_mv, d_tmp, 1u);
    GSS_HIP(hipGetLastError());

    // external -> internal: compose with the remap
    if (c.h_perm.empty()) {
        c.h_perm.resize((size_t)V + 1);
        std::iota(c.h_perm.begin(), c.h_perm.end(), 0u);
        c.d_perm = (uint32_t *)c.dalloc(((size_t)V + 1) * 4);
    }
    for (uint32_t &p : c.h_perm) p = remap[p];
    c.h_iperm.resize((size_t)V + 1);
    for (uint32_t v = 0; v <= V; ++v) c.h_iperm[c.h_perm[v]] = v;
    char *hp = h + remap_pad + 2 * list_bytes;  // not the part still being copied
    std::memcpy(hp, c.h_perm.data(), ((size_t)V + 1) * 4);
    GSS_HIP(hipMemcpyAsync(c.d_perm, hp, ((size_t)V + 1) * 4, hipMemcpyHostToDevice, c.stream));
    c.sync();  // the staging buffers are free again
    // the lead-first order of the stored codes is gone (a performance matter only);
    // the aggregate bits are per row and variable: rebuilt by the next aggregate test
    c.agg_valid = false;
    c.aggu_valid = false;
    c.sagg_valid = false;
    c.saggu_valid = false;
    c.rankings++;
    c.version++;
    c.mutations++;
    return true;
}

}  // namespace gss

using namespace gss;

extern "C" gss_status gss_rank_vars(gss_ctx *ctx, uint64_t *out_hot_lits, uint64_t *out_lits) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    GSS_REQUIRE(!c.serving, GSS_ERR_STATE, "a server owns the context");
    rank_vars(c);
    if (out_hot_lits) *out_hot_lits = c.hot_lits;
    if (out_lits) *out_lits = c.ranked_lits;
    GSS_API_END
}
