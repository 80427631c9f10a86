// Ordered reports (GSS_TEST_SORTED): the kept records of a test, sorted by
// (clause id, word) with a least-significant-digit radix sort written for this
// library.  The key packs clause id and word ((id << word_bits) | word); each
// pass orders the 16-byte records stably by one 8-bit digit of it:
//
//   1. per workgroup tile of 4096 records, the count of each digit (LDS);
//   2. one exclusive scan over the counts, digit-major, so that the records of
//      digit d from tile b start after every smaller digit and after digit d of
//      the tiles before b;
//   3. per tile, every record's rank among the equal digits before it: within a
//      wavefront from the lanes below it that share its digit (eight ballots),
//      across the tile's wavefronts and rounds from counts kept in LDS.
//
// A pass whose digit is the same for every record (the high bits of small ids)
// is skipped; a first read of the records counts every pass's digits at once.
#include "gss_internal.h"

#include <algorithm>

namespace gss {
namespace {

constexpr uint32_t kSortThreads = 256;                   // four wavefronts
constexpr uint32_t kSortRounds = 16;                     // records per thread per tile
constexpr uint32_t kSortTile = kSortThreads * kSortRounds;
constexpr uint32_t kRadix = 256;
constexpr uint32_t kMaxPasses = 8;                       // keys of up to 64 bits

__device__ inline uint64_t record_key(const gss_report &r, uint32_t word_bits) {
    return ((uint64_t)r.clause_id << word_bits) | r.word;
}

__device__ inline uint32_t lanes_below_mask(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// counts[p][d]: records whose digit p is d.
__global__ __launch_bounds__(kSortThreads) void k_sort_digits(const gss_report *r, uint64_t n, uint32_t word_bits,
                                                              uint32_t n_passes, unsigned long long *counts) {
    __shared__ uint32_t h[kMaxPasses][kRadix];
    for (uint32_t i = threadIdx.x; i < kMaxPasses * kRadix; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = record_key(r[i], word_bits);
        for (uint32_t p = 0; p < n_passes; ++p) atomicAdd(&h[p][(k >> (8 * p)) & 0xFF], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_passes * kRadix; i += blockDim.x)
        if ((&h[0][0])[i]) atomicAdd(&counts[i], (unsigned long long)(&h[0][0])[i]);
}

// hist[d * n_tiles + b]: records of tile b whose digit (at `shift`) is d.
__global__ __launch_bounds__(kSortThreads) void k_sort_tile_counts(const gss_report *r, uint64_t n, uint32_t word_bits,
                                                                   uint32_t shift, uint32_t *hist, uint32_t n_tiles) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * kSortTile, hi = min(n, lo + kSortTile);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kSortThreads)
        atomicAdd(&h[(record_key(r[i], word_bits) >> shift) & 0xFF], 1u);
    __syncthreads();
    hist[(uint64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// In-place exclusive scan of m counts by one workgroup of 1024 threads, each
// taking a contiguous share (also the store's compaction offsets).
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *x, uint64_t m) {
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x;
    const uint64_t per = (m + 1023) / 1024, lo = t * per, hi = min(m, lo + per);
    uint32_t sum = 0;
    for (uint64_t i = lo; i < hi; ++i) sum += x[i];
    part[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t ? part[t - 1] : 0u;
    for (uint64_t i = lo; i < hi; ++i) {
        const uint32_t v = x[i];
        x[i] = run;
        run += v;
    }
}

// Stable scatter of one digit: the tile's records go in rounds of 256 (record
// lo + 256 * round + thread), so that index order is (round, wavefront, lane).
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const gss_report *in, gss_report *out, uint64_t n,
                                                               uint32_t word_bits, uint32_t shift,
                                                               const uint32_t *offsets, uint32_t n_tiles) {
    constexpr uint32_t kWaves = kSortThreads / 64;
    __shared__ uint32_t base[kRadix];           // where the tile's records of each digit start, plus those placed
    __shared__ uint32_t per_wave[kWaves][kRadix];
    const uint32_t t = threadIdx.x, wave = t / 64;
    base[t] = offsets[(uint64_t)t * n_tiles + blockIdx.x];
    const uint64_t lo = (uint64_t)blockIdx.x * kSortTile, hi = min(n, lo + kSortTile);
    for (uint32_t round = 0; round < kSortRounds; ++round) {
        for (uint32_t w = 0; w < kWaves; ++w) per_wave[w][t] = 0;
        __syncthreads();
        const uint64_t i = lo + (uint64_t)round * kSortThreads + t;
        const bool valid = i < hi;
        gss_report rec{};
        uint32_t d = 0;
        if (valid) {
            rec = in[i];
            d = (uint32_t)((record_key(rec, word_bits) >> shift) & 0xFF);
        }
        // the lanes of this wavefront holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = lanes_below_mask(peers);  // peers in lower lanes
        if (valid && rank == 0) per_wave[wave][d] = (uint32_t)__builtin_popcountll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (uint32_t w = 0; w < wave; ++w) pos += per_wave[w][d];
            out[pos] = rec;
        }
        __syncthreads();
        uint32_t placed = 0;
        for (uint32_t w = 0; w < kWaves; ++w) placed += per_wave[w][t];
        base[t] += placed;
        __syncthreads();
    }
}

unsigned grid_of(uint64_t n) { return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 16384)); }

}  // namespace

void launch_scan_u32(Ctx &c, uint32_t *x, uint64_t m) {
    if (m == 0) return;
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, c.stream, x, m);
    GSS_HIP(hipGetLastError());
}

void sort_records(Ctx &c, gss_report *src, uint64_t n, gss_report *dst) {
    if (n == 0) return;
    GSS_REQUIRE(n < (1ull << 32) - kSortTile, GSS_ERR_CAPACITY, "too many records to sort");
    uint32_t word_bits = 1;
    while ((1u << word_bits) < c.W) ++word_bits;
    const uint32_t n_passes = (32 + word_bits + 7) / 8;
    const uint32_t n_tiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
    const uint64_t hist_n = (uint64_t)kRadix * n_tiles;
    const size_t counts_bytes = kMaxPasses * kRadix * sizeof(unsigned long long);
    char *buf = (char *)c.dalloc(counts_bytes + hist_n * 4);
    unsigned long long *counts = (unsigned long long *)buf;
    uint32_t *hist = (uint32_t *)(buf + counts_bytes);
    try {
        launch_fill_u64(c, (uint64_t *)counts, kMaxPasses * kRadix, 0);
        hipLaunchKernelGGL(k_sort_digits, dim3(std::min<unsigned>(grid_of(n), 1024)), dim3(kSortThreads), 0, c.stream,
                           src, n, word_bits, n_passes, counts);
        GSS_HIP(hipGetLastError());
        std::vector<unsigned long long> h(kMaxPasses * kRadix);
        GSS_HIP(hipMemcpyAsync(h.data(), counts, counts_bytes, hipMemcpyDeviceToHost, c.stream));
        c.sync();
        // every non-trivial digit, least significant first; src and dst take turns
        gss_report *from = src, *to = dst;
        for (uint32_t p = 0; p < n_passes; ++p) {
            if (*std::max_element(h.begin() + p * kRadix, h.begin() + (p + 1) * kRadix) == n) continue;
            const uint32_t shift = 8 * p;
            hipLaunchKernelGGL(k_sort_tile_counts, dim3(n_tiles), dim3(kSortThreads), 0, c.stream, from, n, word_bits,
                               shift, hist, n_tiles);
            GSS_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, c.stream, hist, hist_n);
            GSS_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_sort_scatter, dim3(n_tiles), dim3(kSortThreads), 0, c.stream, from, to, n, word_bits,
                               shift, hist, n_tiles);
            GSS_HIP(hipGetLastError());
            std::swap(from, to);
        }
        if (from != dst)
            GSS_HIP(hipMemcpyAsync(dst, from, n * sizeof(gss_report), hipMemcpyDeviceToDevice, c.stream));
        c.sync();
    } catch (...) {
        (void)hipStreamSynchronize(c.stream);
        c.dfree(buf);
        throw;
    }
    c.dfree(buf);
}

}  // namespace gss
