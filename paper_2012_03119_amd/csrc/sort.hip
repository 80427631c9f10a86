// Ordered reports (GSS_TEST_SORTED): the kept records of a test, sorted by
// (clause id, word) with a device radix sort (hipCUB / rocPRIM) on a key that
// packs both, the mask carried as the value.
#include "gss_internal.h"

#include <hipcub/hipcub.hpp>

namespace gss {
namespace {

__global__ void k_split_records(const gss_report *r, uint64_t n, uint32_t word_bits, uint64_t *keys, uint64_t *vals) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const gss_report x = r[i];
        keys[i] = ((uint64_t)x.clause_id << word_bits) | x.word;
        vals[i] = x.mask;
    }
}

__global__ void k_join_records(const uint64_t *keys, const uint64_t *vals, uint64_t n, uint32_t word_bits,
                               gss_report *out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        out[i] = gss_report{(uint32_t)(k >> word_bits), (uint32_t)(k & ((1ull << word_bits) - 1)), vals[i]};
    }
}

unsigned grid_of(uint64_t n) { return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 16384)); }

}  // namespace

void sort_records(Ctx &c, const gss_report *src, uint64_t n, gss_report *dst) {
    if (n == 0) return;
    GSS_REQUIRE(n < (1ull << 31), GSS_ERR_CAPACITY, "too many records to sort");
    uint32_t word_bits = 1;
    while ((1u << word_bits) < c.W) ++word_bits;
    const int end_bit = 32 + (int)word_bits;
    size_t temp_bytes = 0;
    GSS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                              (const uint64_t *)nullptr, (uint64_t *)nullptr, (int)n, 0, end_bit,
                                              c.stream));
    // keys and masks, in and out, then the sort's own storage (all within the budget)
    char *buf = (char *)c.dalloc(4 * n * 8 + temp_bytes + 256);
    uint64_t *kin = (uint64_t *)buf, *kout = kin + n, *vin = kout + n, *vout = vin + n;
    void *temp = (void *)(((uintptr_t)(vout + n) + 255) & ~(uintptr_t)255);
    try {
        hipLaunchKernelGGL(k_split_records, dim3(grid_of(n)), dim3(256), 0, c.stream, src, n, word_bits, kin, vin);
        GSS_HIP(hipGetLastError());
        GSS_HIP(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, kin, kout, vin, vout, (int)n, 0, end_bit,
                                                  c.stream));
        hipLaunchKernelGGL(k_join_records, dim3(grid_of(n)), dim3(256), 0, c.stream, kout, vout, n, word_bits, dst);
        GSS_HIP(hipGetLastError());
        c.sync();
    } catch (...) {
        (void)hipStreamSynchronize(c.stream);
        c.dfree(buf);
        throw;
    }
    c.dfree(buf);
}

}  // namespace gss
