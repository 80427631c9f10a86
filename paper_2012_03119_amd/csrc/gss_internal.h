// Internal declarations of libgss: the context, the clause store, the assignment
// planes and the launchers of the device kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <new>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/gss.h"
#include "layout.h"

namespace gss {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

struct Error : std::runtime_error {
    gss_status code;
    Error(gss_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define GSS_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw ::gss::Error(GSS_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define GSS_REQUIRE(cond, code, msg)            \
    do {                                        \
        if (!(cond))                            \
            throw ::gss::Error((code), (msg));  \
    } while (0)

// ---------------------------------------------------------------------------
// encodings shared by host and device code of the library
// ---------------------------------------------------------------------------

// A literal is stored as code = 2*v + neg (v >= 1; neg = 1 for -v).  Plane row
// `code` holds, per slot, whether that literal is F: row 2v has the slots where
// v = F, row 2v+1 the slots where v = T.  Variable 0 is reserved: row 0 is all
// ones (a literal that is always F) and row 1 all zeros (never F).
__host__ __device__ inline uint32_t lit_code(int32_t lit) {
    return lit > 0 ? 2u * (uint32_t)lit : 2u * (uint32_t)(-lit) + 1u;
}

// Plane rows wider than 64 words (4096 slots) are stored in chunks of 64 words:
// chunk g holds words [64g, 64g + 64) of every row, one row after the other, so
// that every chunk has the layout of a 64-word table.  A chunk's slots form a
// super-group (the aggregate of up to 64 word aggregates).  With at most 64
// words there is one chunk and word w of row r sits at r * RW + w.
constexpr uint32_t kChunkWords = 64;
constexpr uint32_t kMaxSlots = 64u * 64u * 64u;  // 64 super-groups of 64 words

__host__ __device__ inline uint64_t plane_index(uint64_t row, uint32_t w, uint32_t RWc, uint64_t chunk_elems) {
    return (uint64_t)(w / kChunkWords) * chunk_elems + row * RWc + (w % kChunkWords);
}

// Plane row variable of external variable v (identity until a ranking moved it).
__host__ __device__ inline uint32_t internal_var(const uint32_t *perm, uint32_t v) { return perm ? perm[v] : v; }

constexpr int kMaxBuckets = 17;              // length classes 4, 8, ..., 65536 (classes 0-1 unused)
constexpr int kMinClass = 2;                 // strides start at 4 codes: one 16-byte load
constexpr uint32_t kMaxClauseLen = 65536;
constexpr uint32_t kDeadId = 0xFFFFFFFFu;
constexpr uint64_t kNoLoc = ~0ull;

// test kernel launch shape: persistent workgroups of 4 wavefronts, up to 8 per CU
constexpr uint32_t kTestWavesPerBlock = 4;
constexpr uint32_t kTestBlocksPerCU = 8;
constexpr uint32_t kMinSegment = 16;   // smallest report segment per wavefront (grown on demand)
constexpr uint64_t kScratchBytes = 64ull << 20;  // gss_test_noalloc's segments, per GPU
constexpr int kMaxDevices = 64;

// length class: smallest c >= kMinClass with 2^c >= len
inline int length_class(uint32_t len) {
    int c = kMinClass;
    while ((1u << c) < len) ++c;
    return c;
}

// ---------------------------------------------------------------------------
// device-side descriptors
// ---------------------------------------------------------------------------

// One length class of the clause store as the test kernel sees it.  Slot s holds
// its clause's codes at lits[s * S + k] (k < S, lead first, padded with code 0), so a
// lane reads four codes with one 16-byte load.  A tile is T consecutive slots
// (T = 64 / lanes-per-clause): the clauses one wavefront tests together.
struct BucketDesc {
    const uint32_t *lits;
    const uint2 *meta;     // per slot: (length, clause id); length 0 = empty or removed
    uint64_t lits_bytes;   // sizes of the two arrays (the kernel's buffer-load bounds)
    uint64_t meta_bytes;
    uint32_t stride_log2;  // S = 1 << stride_log2 codes per slot
    uint32_t tile_begin;   // global index of the bucket's first tile
    const uint32_t *low;   // schedule: bit per slot, set for low-priority clauses (null: no schedule)
    uint64_t low_bytes;
    // scheduled test: the slots this run tests (a list built on the device) and
    // their number (null: every slot, the tile order)
    const uint32_t *list;
    const uint32_t *list_count;
};

struct TestArgs {
    BucketDesc b[kMaxBuckets];
    uint32_t n_buckets;
    uint32_t n_tiles;
    const uint64_t *planes;   // [G][2 * (num_vars + 1)][RWc], RWc = min(RW, 64), RW = lanes per clause >= W
    const uint64_t *active;   // [W]
    uint32_t W;
    uint32_t G;               // chunks (super-groups) of a plane row: 1, or RW / 64
    uint64_t chunk_elems;     // words of one chunk: 2 * (num_vars + 1) * RWc
    uint32_t hot_rows;        // rows [0, hot_rows) are staged in LDS (0 = off)
    gss_report *reports;      // n_waves segments of seg_cap records, one per wavefront
    uint32_t *seg_counts;     // [n_waves]: records produced by each wavefront (beyond seg_cap: counted only)
    uint32_t seg_cap;
    uint64_t *dense;          // GSS_TEST_DENSE: [n_ids][W]
    uint32_t sched_run;       // schedule: a low-priority clause is tested when (sched_run + id) % 4 == 0
    const void *agg;          // aggregate bits per row (element of 2, 4 or 8 bytes by RWc; [G][rows]); null: no pre-test
    const void *aggu;         // trigger mode: per variable, bit w = word w has an active slot where it is U ([G][vars])
    const uint64_t *sagg;     // G > 1: per row, bit g = the row's literal is F in some slot of super-group g
    const uint64_t *saggu;    // G > 1, trigger mode: per variable, bit g = U in some active slot of super-group g
    uint64_t n_rows;          // rows of the plane table (the stride of the aggregate chunks)
    uint64_t gmask;           // super-groups holding an active slot (bit g: words 64g .. 64g + 63)
    uint32_t *wave_stats;     // GSS_TEST_COUNT: [n_waves][2] gathers, pre-test settled words; null: not counted
};

// ---------------------------------------------------------------------------
// host-side state
// ---------------------------------------------------------------------------

struct Bucket {
    uint32_t stride_log2 = 0;
    uint64_t n_slots = 0;    // slots in use, live or removed (the append tail)
    uint64_t n_dead = 0;
    uint64_t cap_slots = 0;  // allocated slots, a multiple of T
    uint64_t n_lits = 0;     // literals of the live clauses
    uint32_t *lits = nullptr;
    uint2 *meta = nullptr;        // per slot (length, id)
    std::vector<uint32_t> h_ids;  // mirror of ids (kDeadId = removed)
    std::vector<uint32_t> h_len;  // mirror of len
    uint32_t *low = nullptr;      // schedule bits (one per slot), built from the priority scores
    uint64_t low_words = 0;
};

struct MlpWork;
struct Priority;

struct Ctx {
    gss_config cfg{};
    int device = 0;
    int n_cu = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t W = 0;     // 64-slot words in use per plane row
    uint32_t RW = 0;    // stored words per plane row (power of two >= W; words >= W stay zero)
    uint32_t RWc = 0;   // words of a row in one chunk: min(RW, 64)
    uint32_t G = 1;     // chunks (super-groups) of a row: RW / RWc
    uint64_t n_rows = 0;       // plane rows: 2 * (num_vars + 1)
    uint64_t chunk_elems = 0;  // words of one chunk: n_rows * RWc
    uint32_t LPC = 0;   // lanes per clause in the test kernel (RWc / words per lane)
    uint32_t T = 0;     // clauses per tile = 64 / LPC
    uint32_t hot_rows = 0;

    uint64_t device_bytes = 0;
    std::unordered_map<void *, size_t> allocs;

    uint64_t *planes = nullptr;
    void *agg = nullptr;  // per row: bit w set when word w of the row is nonzero (see agg_elem_bytes)
    bool agg_valid = true;  // false after bulk plane updates: rebuilt by the next aggregate test
    void *aggu = nullptr;   // per variable: bit w set when some active slot of word w has it U
    bool aggu_valid = false;
    uint64_t *sagg = nullptr;   // G > 1: per row, one bit per super-group (from agg)
    uint64_t *saggu = nullptr;  // G > 1: per variable, one bit per super-group (from aggu)
    bool sagg_valid = false;    // sagg reflects agg
    bool saggu_valid = false;   // saggu reflects aggu
    uint64_t *active = nullptr;
    std::vector<uint64_t> h_active;
    std::vector<uint64_t> var_seen;  // scratch bitmap for argument checks (kept all-zero)
    uint32_t *var_bits = nullptr;    // device twin of var_seen for device-input checks (kept all-zero)

    Bucket buckets[kMaxBuckets];
    std::vector<uint64_t> id_loc;  // per id: bucket << 40 | slot, or kNoLoc
    uint64_t live = 0;
    uint64_t version = 0;  // bumped whenever store arrays or report segments move (batch graphs check it)

    // reports: one segment of seg_cap records per wavefront of the test kernel
    gss_report *reports = nullptr;
    uint32_t max_waves = 0;                  // wavefronts of the largest test launch
    uint32_t seg_cap = 0;
    uint32_t last_waves = 0;                 // wavefronts of the last launch
    uint32_t *seg_counts = nullptr;          // [max_waves]
    uint64_t *seg_offsets = nullptr;         // [max_waves + 1] exclusive prefix of the kept records
    unsigned long long *d_summary = nullptr;  // device {total, max, kept, deferred verdict}
    unsigned long long *h_summary = nullptr;  // pinned host copy, written by the finalize kernel
    unsigned long long *hd_summary = nullptr; // h_summary as kernels address it
    const void *occ_fn = nullptr;             // the test kernel whose occupancy is cached
    size_t occ_lds = 0;
    int occ_fit = 0;
    uint32_t *dsmall = nullptr;              // 256 B device scratch for flags
    uint32_t *hsmall = nullptr;              // 256 B pinned host
    void *d_desc = nullptr;                  // device copy of the test kernel's bucket descriptors
    std::vector<BucketDesc> desc_shadow;     // what the device copy holds (uploaded again only when it differs)
    void *hsmall_desc = nullptr;             // pinned host staging of the same
    uint64_t test_serial = 0;  // tests completed by this context
    uint64_t n_reports = 0;  // records found by the last test
    uint64_t n_kept = 0;     // records stored (fewer on overflow)
    bool tested = false;
    uint32_t last_flags = 0;

    // internal variable numbers (hot-variable ranking): external v -> perm[v];
    // empty / null until the first ranking that moves a variable (identity)
    std::vector<uint32_t> h_perm;
    std::vector<uint32_t> h_iperm;  // internal -> external
    uint32_t *d_perm = nullptr;
    uint64_t ranked_lits = 0;  // literals stored at the last ranking
    uint64_t hot_lits = 0;     // of them, on the staged variables
    uint64_t rankings = 0;
    bool serving = false;      // a server owns the context (no ranking then)
    const uint32_t *perm() const { return h_perm.empty() ? nullptr : h_perm.data(); }
    uint32_t external_var(uint32_t v) const { return h_iperm.empty() ? v : h_iperm[v]; }

    uint32_t *wave_stats = nullptr;  // [max_waves][2], allocated by the first counted test
    uint32_t *sched_list = nullptr;  // scheduled test: slots tested this run, per length class
    uint64_t sched_list_cap = 0;
    uint32_t *sched_counts = nullptr;  // [kMaxBuckets]: their number

    uint64_t *dense = nullptr;
    uint64_t dense_rows = 0;
    uint64_t dense_ids = 0;  // ids issued when the last dense test ran: the rows it wrote

    // staging for uploads (device) and pinned host staging
    void *dstage = nullptr;
    size_t dstage_bytes = 0;
    void *hstage = nullptr;
    size_t hstage_bytes = 0;

    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    bool timed = false;  // the last launched test kernel has timing events
    hipEvent_t ev_stage = nullptr;  // recorded after the last queued use of the staging buffers
    // queued deltas: their variable lists go up on a copy stream of their own while
    // the test ahead of them runs (created by the first gss_set_var_values_async)
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_copy = nullptr;
    uint64_t tests_launched = 0;    // serial of the last queued test (its finalize kernel writes it to h_summary[4])
    uint64_t tests_completed = 0;   // serial of the last test seen complete (or of all, after a sync)
    bool pending = false;           // gss_test_async issued, gss_test_wait not yet called (or a batched test
                                    // of which the context is a member, gss_batch_wait not yet called)
    bool batch_pending = false;     // the test in flight is a batch's
    bool pending_launched = false;
    uint32_t pending_flags = 0;
    bool stage_pending = false;
    uint64_t mutations = 0;         // calls that changed the store, the planes or the active set
    uint64_t launch_mutations = 0;  // the same counter when the last test was launched
    gss_stats stats{};
    std::string last_error;
    MlpWork *mlp = nullptr;    // workspace of the priority network's kernels
    Priority *prio = nullptr;  // learned clause priority (null until enabled)

    // device memory within the budget
    void *dalloc(size_t bytes);
    void dfree(void *p);
    // Bulk staging (large uploads and downloads that synchronise): the returned
    // memory is free to write (queued work that read it has finished).  A call
    // that leaves work reading it queued calls stage_release().
    void *device_stage(size_t bytes);
    void *host_stage(size_t bytes);
    void stage_release();
    void sync();
    void mark_idle();  // bookkeeping of sync() after the stream was synchronised elsewhere
    // Device memory that queued work may still read: freed once the test queued
    // after that work has completed (or at the next synchronisation).
    void defer_free(void *p);
    void release_deferred();  // frees what the completed tests no longer need
    // true when `bytes` more fit the HBM budget, after releasing deferred frees
    // (which synchronises) if that is what it takes
    bool fits(uint64_t bytes);
    std::vector<std::pair<void *, uint64_t>> deferred_frees;

    // Upload ring: small uploads (deltas, inserts, removals, activity) take a slot
    // of pinned host + device memory; the kernels that read it are queued before
    // the next test, so the slot is free once that test has completed (or after a
    // synchronisation).  A caller can queue uploads behind a test still running
    // without waiting for it, and no event is recorded between the kernels.
    struct Staged {
        char *h;
        char *d;
        int slot;
        const char *hd;  // h as kernels address it (pinned host memory read over the bus)
    };
    static constexpr int kRing = 8;
    struct RingSlot {
        char *h = nullptr;
        char *hd = nullptr;
        char *d = nullptr;
        size_t hbytes = 0;  // pinned host bytes
        size_t dbytes = 0;  // device bytes (may be fewer: slots taken host-only)
        uint64_t free_after = 0;  // free once this test serial has completed
        bool busy = false;
    } ring[kRing];
    int ring_next = 0;
    // A free slot of at least `bytes`.  host_only: only its pinned host memory is
    // used (kernels read it over the bus), so taking it allocates no device memory
    // and cannot fail on the HBM budget (.d may then be smaller or null).
    Staged stage_upload(size_t bytes, bool host_only = false);
    void stage_done(const Staged &s);            // its consumers are queued
};

// True when this thread's share (grid-stride: first item tid, step stride) of the
// n truth values at v holds a byte outside {-1, 0, +1}.  Sixteen bytes per load;
// a byte x is valid iff (x + 1) as an unsigned byte is at most 2.
__device__ inline bool values_invalid(const int8_t *v, uint64_t n, uint64_t tid, uint64_t stride) {
    unsigned found = 0;
    const uint64_t head = (16 - ((uintptr_t)v & 15)) & 15;  // bytes before the first aligned block
    for (uint64_t i = tid; i < head && i < n; i += stride) found |= (uint8_t)(v[i] + 1) > 2;
    const uint64_t n16 = n > head ? (n - head) / 16 : 0;
    const uint4 *q = reinterpret_cast<const uint4 *>(v + head);
    for (uint64_t i = tid; i < n16; i += stride) {
        const uint4 x = q[i];
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int s = 0; s < 4; ++s) found |= (((w[k] >> (8 * s)) + 1) & 0xFFu) > 2;
    }
    for (uint64_t i = head + n16 * 16 + tid; i < n; i += stride) found |= (uint8_t)(v[i] + 1) > 2;
    return found != 0;
}

// Bytes of one row's aggregate bits in one chunk: 2 up to 16 words, 4 up to 32, else 8.
inline uint32_t agg_elem_bytes(uint32_t RWc) { return RWc <= 16 ? 2u : RWc <= 32 ? 4u : 8u; }
// recomputes the aggregate bits of rows [lo, hi) in every chunk
void agg_rebuild(Ctx &c, uint64_t lo, uint64_t hi);
// recomputes the per-variable U bits (trigger-mode aggregates) of every variable
void aggu_rebuild(Ctx &c);
// G > 1: recomputes the super-group bits from the word bits (sagg, and saggu when
// the trigger-mode bits are wanted)
void super_rebuild(Ctx &c, bool with_u);

// kernels / launchers (defined in the .hip files)
void launch_fill_u64(Ctx &c, uint64_t *p, uint64_t n, uint64_t value);
void launch_fill_u32(Ctx &c, uint32_t *p, uint64_t n, uint32_t value);
bool is_device_pointer(const void *p);
unsigned fill_grid(uint64_t n);  // workgroups of 256 for a grid-stride pass over n items
const uint32_t *queue_value_check(Ctx &c, const int8_t *values, uint64_t n);
void queue_value_check_into(Ctx &c, const int8_t *values, uint64_t n, uint32_t *verdict);
void check_flag(Ctx &c);
// Queues a kernel copy of `bytes` (a multiple of 16, 16-byte aligned) from pinned
// host memory (as kernels address it, Staged::hd) into device memory.
void copy_in(Ctx &c, void *dst, const void *src_hd, size_t bytes);
// Queues the copy of the last test's first n kept records, as one list, into
// device memory dst (on the context's stream).
void queue_stitch(Ctx &c, gss_report *dst, uint64_t n);
void scratch_setup(int device);  // once per device, from gss_create
// Activity (learned priority enabled): state for ids below n_ids (validate
// before an insert changes anything); bump the clauses with a record in the
// last test; remove the least active live clauses until `keep` remain, returning
// their ids (may run while a test is in flight: it synchronises the stream).
void priority_reserve(Ctx &c, uint64_t n_ids);
void priority_bump_hits(Ctx &c);
std::vector<uint32_t> priority_evict(Ctx &c, uint64_t keep);
// Ranks the variables by occurrences in the live clauses and renumbers them so
// that the most frequent own the LDS-staged rows; false when nothing moved.
bool rank_vars(Ctx &c);
// Writes the n records at src (device) into dst (device) ordered by (clause id,
// word); synchronises the stream.
void sort_records(Ctx &c, gss_report *src, uint64_t n, gss_report *dst);  // src is overwritten
void launch_scan_u32(Ctx &c, uint32_t *x, uint64_t m);  // in place, exclusive, on c.stream
uint32_t *deferred_flag(Ctx &c);
uint32_t read_deferred(Ctx &c);
void report_deferred(Ctx &c, uint32_t verdict);
// Clause ingest in two parts.  prepare_clauses validates DIMACS clauses and
// encodes them (codes 2v+neg of the internal variable number perm[v], or v
// without a map; the lead -- smallest code -- first; the length class and lead
// of each clause); it touches no context and may run on any thread.  commit_clauses assigns ids in batch order and uploads the batch, laid
// out by length class and lead.  Both throw Error.
struct Prepared {
    std::vector<uint32_t> codes;
    std::vector<uint64_t> offs{0};
    std::vector<uint32_t> lead;
    std::vector<uint8_t> cls;
    uint32_t size() const { return (uint32_t)lead.size(); }
    void clear() {
        codes.clear();
        offs.assign(1, 0);
        lead.clear();
        cls.clear();
    }
    void append(const Prepared &o);
};
void prepare_clauses(int64_t num_vars, const int32_t *lits, const uint64_t *offsets, uint32_t n, Prepared &out,
                     const uint32_t *perm);
void commit_clauses(Ctx &c, const Prepared &p, uint32_t *out_ids);

// learned priority hooks: clauses added (ids first..first+n, lengths from offsets),
// clauses removed (host ids), the schedule bits of every class (for a scheduled
// test; returns the run number), and release of everything
void priority_added(Ctx &c, uint64_t first, uint32_t n, const uint64_t *offsets);
void priority_removed(Ctx &c, const uint32_t *ids, uint32_t n);
uint32_t priority_schedule(Ctx &c);
void priority_release(Ctx &c);
void mlp_release(Ctx &c);
// queues new plane words of n variables of one 64-slot word (device arrays, checked by the caller)
void launch_set_words(Ctx &c, uint32_t word, const uint32_t *vars, const uint64_t *f, const uint64_t *t, uint32_t n);

// Wrapper of every ABI entry point taking a context: converts exceptions into
// status codes and records the message for gss_last_error.
#define GSS_API_BEGIN(ctxp)                                  \
    ::gss::Ctx *c_ = reinterpret_cast<::gss::Ctx *>(ctxp);   \
    if (!c_) return GSS_ERR_INVALID_ARG;                     \
    try {                                                    \
        c_->last_error.clear();
#define GSS_API_END                                          \
    }                                                        \
    catch (const ::gss::Error &e) {                          \
        c_->last_error = e.what();                           \
        return e.code;                                       \
    }                                                        \
    catch (const std::bad_alloc &) {                         \
        c_->last_error = "host out of memory";               \
        return GSS_ERR_CAPACITY;                             \
    }                                                        \
    catch (const std::exception &e) {                        \
        c_->last_error = e.what();                           \
        return GSS_ERR_DEVICE;                               \
    }                                                        \
    return GSS_OK;

}  // namespace gss
