// Layout of a length class's literal codes, shared by the host and the kernels.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define GSS_HD __host__ __device__
#else
#define GSS_HD
#endif

namespace gss {

// Position (in codes) of code k of slot `slot` in a length class of stride
// 2^s_log2 whose tiles hold 2^t_log2 clauses.  Each tile takes T * S consecutive
// codes; inside it the codes come in groups of four, group g of every clause of
// the tile side by side (clause j's group at (g * T + j) * 4).  The wavefront
// testing a tile then reads each group of its clauses as one contiguous run:
// whole cache lines, where a slot-major layout would touch one line per clause
// to read its first few codes.
GSS_HD inline uint64_t code_index(uint64_t slot, uint32_t k, uint32_t s_log2, uint32_t t_log2) {
    const uint64_t tile = slot >> t_log2, j = slot & ((1ull << t_log2) - 1);
    return ((tile << t_log2) << s_log2) + ((((uint64_t)(k >> 2)) << t_log2) + j) * 4 + (k & 3);
}

}  // namespace gss
