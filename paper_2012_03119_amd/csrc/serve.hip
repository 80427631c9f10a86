// Served clause test: a GPU-manager thread fed by solver threads.
//
// Section 5 of the paper runs one CPU thread besides the solver threads to drive
// the GPU; Section 3.6 has the solvers send it their assignments and export their
// learned clauses, and get back the clauses that fire.  Here producer p owns the
// 64 slots of word p and sends snapshots of its 64 assignments as packed deltas.
//
// Data path of one snapshot:
//   producer thread: merges the delta into its open mailbox (pinned host memory;
//     a variable sent twice keeps its last value)
//   manager: takes the mailbox (swapping in a free one) and copies it to the
//     device on a copy stream while the current run still executes; once that
//     run has completed, it queues the copy of the run's records to the host (on
//     a fetch stream), then the plane update (behind the upload) and the next run
//   next run: tests every word with a new snapshot; while the run after it
//     executes, its records are routed by word to the producers' queues, which
//     is when the snapshot is notified.  A queue holds ranges of the pinned
//     buffer the records came back in, not copies: each producer copies its own
//     records when it polls, on its own thread.
//
// Runs are launched back to back (continuous batching): while run k executes,
// the manager routes the records of run k-1 and admits snapshots, inserts and
// removals for run k+1.
#include "gss_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>

namespace gss {
namespace {

using Clock = std::chrono::steady_clock;

// Staged delta of one word: vars[cap] | f[cap] | t[cap] in pinned host memory,
// mirrored by a device buffer of the same layout for the plane update kernel.
struct Mail {
    char *h = nullptr;
    uint32_t cap = 0;
    uint32_t n = 0;
    char *d = nullptr;
    uint32_t dcap = 0;
    uint64_t free_after = 0;    // the test queued behind the kernel that read d
    bool busy = false;          // uploaded or applied, until that test completes
    bool queued = false;        // uploaded, plane update not queued yet
    const char *hd = nullptr;   // h as kernels address it, when the device buffer could not be had (else null)

    static size_t vbytes(uint32_t cap) { return ((size_t)cap * 4 + 255) / 256 * 256; }
    static size_t bytes(uint32_t cap) { return vbytes(cap) + (size_t)cap * 16; }
    uint32_t *vars() const { return (uint32_t *)h; }
    uint64_t *f() const { return (uint64_t *)(h + vbytes(cap)); }
    uint64_t *t() const { return (uint64_t *)(h + vbytes(cap)) + cap; }
};

constexpr int kMails = 3;  // the open one, and up to two queued behind runs

// The records of one run in pinned host memory, shared by the producers that
// still hold a range of them; reused once none does.
struct RecBlock {
    gss_report *h = nullptr;
    uint64_t cap = 0;
    uint64_t used_run = 0;  // the last run fetched into it
    RecBlock() = default;
    RecBlock(const RecBlock &) = delete;
    RecBlock &operator=(const RecBlock &) = delete;
    ~RecBlock() {
        if (h) (void)hipHostFree(h);
    }
};

// Pending records of a producer: a range of a shared block, or (once the block
// had to be reused before the producer polled) records of its own.
struct OutChunk {
    std::shared_ptr<RecBlock> blk;
    std::vector<gss_report> own;
    const gss_report *p = nullptr;
    uint64_t n = 0;
};

constexpr size_t kMaxRecBlocks = 8;  // beyond this, a producer that does not poll gets copies

struct Producer {
    std::mutex mu;
    Mail mail[kMails];
    int open = 0;
    std::vector<uint32_t> pos;  // variable -> its index in the open mailbox (checked against vars[])
    uint64_t snaps = 0;         // snapshots merged into the open mailbox
    double arrival = -1.0;      // send time of the newest of them

    std::mutex omu;
    std::deque<OutChunk> outbox;
    uint64_t out_n = 0;  // records in the outbox
    uint64_t last_run = UINT64_MAX;
};

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)std::llround(p * (double)(v.size() - 1)));
    std::nth_element(v.begin(), v.begin() + (ptrdiff_t)k, v.end());
    return v[k];
}

// Splitmix64 step: the random removals.
uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Grows a producer's open mailbox (not queued, so its memory is free to move).
void ensure_host(Mail &m, uint32_t need, uint32_t limit) {
    if (need <= m.cap) return;
    uint32_t cap = (uint32_t)std::max<uint64_t>(need, std::min<uint64_t>(limit, 2ull * m.cap));
    cap = std::min(cap, limit);
    char *h = nullptr;
    if (hipHostMalloc((void **)&h, Mail::bytes(cap), hipHostMallocDefault) != hipSuccess)
        throw Error(GSS_ERR_DEVICE, "hipHostMalloc failed for a delta mailbox");
    Mail old = m;
    m.h = h;
    m.cap = cap;
    if (old.h) {
        std::memcpy(m.vars(), old.vars(), (size_t)m.n * 4);
        std::memcpy(m.f(), old.f(), (size_t)m.n * 8);
        std::memcpy(m.t(), old.t(), (size_t)m.n * 8);
        (void)hipHostFree(old.h);
    }
}

// ---- records routed by word on the device: a counting sort of the run's kept
//      records by their 64-slot word (a served producer owns one word), so that
//      the host hands each producer one contiguous block.

// counts[w] += records of word w (counts zeroed before).
__global__ __launch_bounds__(256) void k_route_count(const gss_report *reports, const uint32_t *seg_counts,
                                                     uint32_t seg_cap, uint32_t n_segments, uint32_t *counts) {
    __shared__ uint32_t h[kChunkWords];
    if (threadIdx.x < kChunkWords) h[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t s = blockIdx.x; s < n_segments; s += gridDim.x) {
        const uint32_t n = min(seg_counts[s], seg_cap);
        const gss_report *seg = reports + (uint64_t)s * seg_cap;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&h[seg[i].word], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kChunkWords && h[threadIdx.x]) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

// One wavefront: offsets[w] = records of the words before w (offsets[W] = all),
// and the placement cursors start there.
__global__ void k_route_scan(const uint32_t *counts, uint32_t W, uint32_t *cursor, unsigned long long *offsets) {
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (uint32_t w = 0; w < W; ++w) {
            offsets[w] = run;
            cursor[w] = (uint32_t)run;
            run += counts[w];
        }
        offsets[W] = run;
    }
}

// Every kept record to its word's block (order inside a block unspecified).  A
// workgroup counts its segments' records per word in LDS, claims one range per
// word with one atomic each, then places its records with LDS cursors: the
// global counters see one atomic per (workgroup, word), not one per record.
__global__ __launch_bounds__(256) void k_route_place(const gss_report *reports, const uint32_t *seg_counts,
                                                     uint32_t seg_cap, uint32_t n_segments, uint32_t *cursor,
                                                     gss_report *out) {
    __shared__ uint32_t h[kChunkWords];
    if (threadIdx.x < kChunkWords) h[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t s = blockIdx.x; s < n_segments; s += gridDim.x) {
        const uint32_t n = min(seg_counts[s], seg_cap);
        const gss_report *seg = reports + (uint64_t)s * seg_cap;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&h[seg[i].word], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kChunkWords) h[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]) : 0u;
    __syncthreads();
    for (uint32_t s = blockIdx.x; s < n_segments; s += gridDim.x) {
        const uint32_t n = min(seg_counts[s], seg_cap);
        const gss_report *seg = reports + (uint64_t)s * seg_cap;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const gss_report r = seg[i];
            out[atomicAdd(&h[r.word], 1u)] = r;
        }
    }
}

}  // namespace
}  // namespace gss

using namespace gss;

struct gss_server {
    Ctx *c = nullptr;
    gss_server_config cfg{};
    uint32_t V = 0, P = 0;
    Clock::time_point t0;
    std::vector<Producer> prod;
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_copied = nullptr;
    // records of a finished run travel to the host on their own stream while the
    // next run executes: routed into fdev[k], copied into a pinned block
    hipStream_t fetch_stream = nullptr;
    hipEvent_t ev_stitched = nullptr;
    hipEvent_t ev_fetched[2] = {nullptr, nullptr};
    FILE *log = nullptr;

    // inserts waiting for admission, already validated and encoded by the
    // producer threads that sent them
    std::mutex imu;
    Prepared queue;
    uint64_t q_limit = 0;

    std::atomic<bool> stop{false};
    std::atomic<bool> failed{false};
    std::thread manager;
    gss_status status = GSS_OK;
    std::string error;
    std::string manager_error;
    mutable std::mutex emu;

    std::atomic<uint64_t> n_snapshots{0}, n_refused{0};
    gss_serve_result res{};
    std::vector<double> lat;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void fail(gss_status code, const std::string &msg) {
        std::lock_guard<std::mutex> g(emu);
        if (status == GSS_OK) {
            status = code;
            error = msg;
            manager_error = msg;  // kept: later calls refused by the failed server overwrite `error`
        }
        failed = true;
    }
    void run();
};

void gss_server::run() {
    Ctx &C = *c;
    gss_ctx *ctx = reinterpret_cast<gss_ctx *>(c);
    std::vector<uint32_t> live;  // ids of live clauses, for random removal
    live.reserve(C.live + 1024);
    for (uint64_t id = 0; id < C.id_loc.size(); ++id)
        if (C.id_loc[id] != kNoLoc) live.push_back((uint32_t)id);
    uint64_t rng = cfg.seed * 0x2545F4914F6CDD1Dull + 11;
    std::vector<double> staged(P, -1.0), inflight(P, -1.0);  // arrival of the untested / tested snapshot
    // two device lists, used in turn, the records are routed into; pinned blocks
    // they are copied to (they come back at full link speed), shared with the
    // producers' outboxes
    gss_report *fdev[2] = {nullptr, nullptr};
    uint64_t fdev_cap[2] = {0, 0};
    std::vector<std::shared_ptr<RecBlock>> pool;
    // routing by word: device counts, cursors and offsets; pinned copies of the offsets
    uint32_t *route_dev = nullptr;  // counts [64] | cursor [64] | offsets [65] (u64)
    unsigned long long *roff[2] = {nullptr, nullptr};
    int next_k = 0;
    struct Fetch {  // the records of a finished run on their way to the host (at most one)
        bool active = false;
        uint64_t run = 0, n = 0;
        int k = 0;
        std::shared_ptr<RecBlock> blk;
        std::vector<double> arrivals;  // per producer: the tested snapshot's send time, or -1
    } fq;
    std::vector<uint64_t> act(C.W, 0);
    struct Taken {
        uint32_t p;
        Mail *m;
    };
    std::vector<Taken> taken;
    Prepared ins;
    std::vector<uint32_t> ids;
    bool held = false;  // inserts held back by the HBM budget until something is removed
    bool evict_spent = false;
    bool pending = false;
    uint64_t run_id = 0;
    double del_due = 0.0, last = now();
    const double kernel_ms0 = C.stats.total_kernel_ms;
    const char *phase = "start";  // what the manager was doing (named in an error)
    auto timed = [&](double &acc, auto &&fn) {
        const double a = now();
        fn();
        acc += (now() - a) * 1e3;
    };

    auto admit = [&]() {
        // ---- snapshots: take every producer's open mailbox that holds any and
        //      start its upload (the plane update itself waits for the next launch)
        for (uint32_t p = 0; p < P; ++p) {
            Producer &pr = prod[p];
            Mail *m = nullptr;
            uint64_t snaps = 0;
            double arrival = -1.0;
            {
                // a producer merging a snapshot holds its lock: take its mailbox next time
                std::unique_lock<std::mutex> g(pr.mu, std::try_to_lock);
                if (!g.owns_lock() || pr.snaps == 0) continue;
                int free_k = -1;
                for (int k = 0; k < kMails && free_k < 0; ++k) {
                    if (k == pr.open) continue;
                    Mail &x = pr.mail[k];
                    if (x.queued) continue;
                    if (x.busy) {
                        // free once the run queued behind its plane update has completed,
                        // or once the stream is idle (a run that launched nothing)
                        if (C.tests_completed < x.free_after) {
                            const hipError_t e = hipStreamQuery(C.stream);
                            if (e == hipErrorNotReady) continue;
                            GSS_HIP(e);
                        }
                        x.busy = false;
                    }
                    free_k = k;
                }
                if (free_k < 0) continue;  // both in use: keep merging into the open one
                m = &pr.mail[pr.open];
                pr.open = free_k;
                pr.mail[free_k].n = 0;
                snaps = pr.snaps;
                arrival = pr.arrival;
                pr.snaps = 0;
            }
            res.dropped += snaps - 1 + (staged[p] >= 0 ? 1 : 0);
            staged[p] = arrival;
            if (m->n == 0) continue;
            m->hd = nullptr;
            if (m->n > m->dcap) {  // the device mirror is idle: the mailbox was open
                C.dfree(m->d);
                m->d = nullptr;
                m->dcap = 0;
                try {
                    m->d = (char *)C.dalloc(Mail::bytes(m->cap));
                    m->dcap = m->cap;
                } catch (const Error &e) {
                    if (e.code != GSS_ERR_CAPACITY) throw;
                    // no room in the HBM budget: the plane update reads the mailbox
                    // from pinned host memory over the bus instead (the delta must
                    // be applied: the producer's next one builds on it)
                    void *hd = nullptr;
                    GSS_HIP(hipHostGetDevicePointer(&hd, m->h, 0));
                    m->hd = (const char *)hd;
                }
            }
            if (!m->hd) {
                const size_t vb = Mail::vbytes(m->dcap);
                GSS_HIP(hipMemcpyAsync(m->d, m->h, (size_t)m->n * 4, hipMemcpyHostToDevice, copy_stream));
                GSS_HIP(hipMemcpyAsync(m->d + vb, m->f(), (size_t)m->n * 8, hipMemcpyHostToDevice, copy_stream));
                GSS_HIP(hipMemcpyAsync(m->d + vb + (size_t)m->dcap * 8, m->t(), (size_t)m->n * 8,
                                       hipMemcpyHostToDevice, copy_stream));
            }
            res.delta_bytes += (uint64_t)m->n * 20;
            m->busy = true;
            m->queued = true;
            taken.push_back({p, m});
        }
    };

    // Plane updates of the uploaded deltas, queued right before a launch: queued
    // earlier, they would sit behind the copies between the running test and the
    // fetch of its records.
    auto apply_deltas = [&]() {
        if (!taken.empty()) {
            GSS_HIP(hipEventRecord(ev_copied, copy_stream));
            GSS_HIP(hipStreamWaitEvent(C.stream, ev_copied, 0));
            for (const Taken &x : taken) {
                Mail &m = *x.m;
                if (m.hd) {  // read from pinned host memory (same layout, capacity m.cap)
                    const size_t vb = Mail::vbytes(m.cap);
                    launch_set_words(C, x.p, (const uint32_t *)m.hd, (const uint64_t *)(m.hd + vb),
                                     (const uint64_t *)(m.hd + vb) + m.cap, m.n);
                } else {
                    const size_t vb = Mail::vbytes(m.dcap);
                    launch_set_words(C, x.p, (const uint32_t *)m.d, (const uint64_t *)(m.d + vb),
                                     (const uint64_t *)(m.d + vb) + m.dcap, m.n);
                }
                m.free_after = C.tests_launched + 1;  // the run launched right after this
                m.queued = false;
                if (log) {
                    std::fprintf(log, "W %u %u\n", x.p, m.n);
                    const uint32_t *v = m.vars();
                    const uint64_t *f = m.f(), *t = m.t();
                    for (uint32_t i = 0; i < m.n; ++i)
                        std::fprintf(log, "%u %llx %llx\n", v[i], (unsigned long long)f[i], (unsigned long long)t[i]);
                }
            }
            taken.clear();
        }
    };

    // Activity eviction: removes the least active live clauses until evict_keep
    // of them are left; logged as a "V n" line followed by the removal.
    auto evict = [&]() {
        const uint64_t keep = (uint64_t)std::floor(cfg.evict_keep * (double)C.live);
        const std::vector<uint32_t> out = priority_evict(C, keep);
        if (out.empty()) return;
        res.evicted += out.size();
        res.evictions++;
        if (log) {
            std::fprintf(log, "V %zu\nR %zu", out.size(), out.size());
            for (uint32_t id : out) std::fprintf(log, " %u", id);
            std::fputc('\n', log);
        }
        live.clear();  // rebuilt from the store: evictions are rare
        for (uint64_t id = 0; id < C.id_loc.size(); ++id)
            if (C.id_loc[id] != kNoLoc) live.push_back((uint32_t)id);
    };

    // Store changes are queued once per run, behind the run just launched, so
    // their host work overlaps it (and the upload ring is not drained).
    auto change_store = [&]() {
        // ---- removals: a fraction of the live clauses per second
        const double t = now();
        del_due += cfg.delete_fraction * (double)live.size() * std::max(0.0, t - last);
        last = t;
        const uint32_t n_del = (uint32_t)std::min<double>(std::floor(del_due), (double)live.size());
        if (n_del) {
            del_due -= n_del;
            ids.resize(n_del);
            for (uint32_t i = 0; i < n_del; ++i) {
                const uint64_t k = splitmix(rng) % live.size();
                ids[i] = live[k];
                live[k] = live.back();
                live.pop_back();
            }
            const gss_status rc = gss_remove_clauses(ctx, ids.data(), n_del);
            if (rc != GSS_OK) throw Error(rc, C.last_error);
            res.deleted += n_del;
            held = false;
            if (log) {
                std::fprintf(log, "R %u", n_del);
                for (uint32_t id : ids) std::fprintf(log, " %u", id);
                std::fputc('\n', log);
            }
        }
        // ---- inserts, admitted within the HBM budget
        if (!held) {
            {
                std::lock_guard<std::mutex> g(imu);
                std::swap(ins, queue);
                queue.clear();
            }
            const uint32_t n = ins.size();
            if (n) {
                ids.resize(n);
                // with eviction, the store also leaves room for the manager's own
                // buffers (records, mailboxes, report segments): a budget that is
                // nearly used up evicts before the insert
                const uint64_t budget = C.cfg.hbm_budget_bytes;
                const uint64_t reserve = cfg.evict_keep > 0 ? budget / 32 : 0;
                if (cfg.evict_keep > 0 && !evict_spent && budget && C.device_bytes + reserve > budget) evict();
                // the store may not take the reserve (the budget is lowered during the insert)
                auto commit = [&]() -> bool {
                    C.cfg.hbm_budget_bytes = budget - reserve;
                    try {
                        commit_clauses(C, ins, ids.data());
                    } catch (const Error &e) {
                        C.cfg.hbm_budget_bytes = budget;
                        if (e.code != GSS_ERR_CAPACITY) throw;
                        return false;
                    } catch (...) {
                        C.cfg.hbm_budget_bytes = budget;
                        throw;
                    }
                    C.cfg.hbm_budget_bytes = budget;
                    return true;
                };
                bool admitted = commit();
                if (!admitted && cfg.evict_keep > 0 && !evict_spent) {
                    // Section 3.7: the least active clauses leave to make room (the
                    // activities of the runs completed so far), then the insert is retried
                    evict();
                    admitted = commit();
                }
                // an eviction that made no room is not repeated until an insert is admitted
                evict_spent = !admitted && cfg.evict_keep > 0;
                if (admitted) {
                    res.inserted += n;
                    live.insert(live.end(), ids.begin(), ids.end());
                    if (log) {
                        for (uint32_t i = 0; i < n; ++i) {
                            std::fprintf(log, "A %u %llu", ids[i], (unsigned long long)(ins.offs[i + 1] - ins.offs[i]));
                            for (uint64_t k = ins.offs[i]; k < ins.offs[i + 1]; ++k) {
                                const uint32_t code = ins.codes[k];
                                // the caller's variable numbers, not the internal ones
                                const int32_t v = (int32_t)C.external_var(code >> 1);
                                std::fprintf(log, " %d", (code & 1) ? -v : v);
                            }
                            std::fputc('\n', log);
                        }
                    }
                    ins.clear();
                } else {
                    // budget full: back in front of what arrived since, until a removal
                    held = true;
                    std::lock_guard<std::mutex> g(imu);
                    ins.append(queue);
                    std::swap(ins, queue);
                    ins.clear();
                }
            }
        }
    };

    // Routes the records of the fetched run to the producers' queues (which is when
    // their snapshots are notified).  With wait false, returns false while the copy
    // is still on its way.  Runs on the manager thread while the next run executes
    // (a thread of its own measured slower: the host cores are shared with the
    // solver threads).
    auto route_fetch = [&](bool wait) -> bool {
        if (!fq.active) return false;
        if (wait) {
            timed(res.fetch_ms, [&] { GSS_HIP(hipEventSynchronize(ev_fetched[fq.k])); });
        } else {
            const hipError_t e = hipEventQuery(ev_fetched[fq.k]);
            if (e == hipErrorNotReady) return false;
            GSS_HIP(e);
        }
        const double route_t0 = now();
        const gss_report *r = fq.blk->h;
        const unsigned long long *off = roff[fq.k];  // producer p's records: r[off[p] .. off[p + 1])
        const uint64_t got = fq.n;
        if (log) {
            for (uint64_t i = 0; i < got; ++i)
                std::fprintf(log, "P %llu %u %u %llx\n", (unsigned long long)fq.run, r[i].clause_id, r[i].word,
                             (unsigned long long)r[i].mask);
            std::fprintf(log, "E %llu %llu\n", (unsigned long long)fq.run, (unsigned long long)got);
        }
        const double t = now();
        for (uint32_t p = 0; p < P; ++p) {
            if (fq.arrivals[p] < 0) continue;
            {
                Producer &pr = prod[p];
                std::lock_guard<std::mutex> g(pr.omu);
                const uint64_t m = got ? off[p + 1] - off[p] : 0;
                if (m) {
                    OutChunk ch;
                    ch.blk = fq.blk;
                    ch.p = r + off[p];
                    ch.n = m;
                    pr.outbox.push_back(std::move(ch));
                    pr.out_n += m;
                }
                pr.last_run = fq.run;
            }
            lat.push_back((t - fq.arrivals[p]) * 1e3);
            res.tested++;
        }
        res.reports += got;
        res.route_ms += (now() - route_t0) * 1e3;
        fq.active = false;
        fq.blk.reset();
        return true;
    };

    // A pinned block for a run's records: a free one (no producer holds a range of
    // it; the smallest that fits, else the largest, grown), a new one while the
    // pool is small, else the least recently used one, whose holders are given
    // copies of their ranges first.
    auto take_block = [&](uint64_t need) -> std::shared_ptr<RecBlock> {
        auto better = [need](const RecBlock &a, const RecBlock &b) {
            const bool fa = a.cap >= need, fb = b.cap >= need;
            if (fa != fb) return fa;
            return fa ? a.cap < b.cap : a.cap > b.cap;
        };
        std::shared_ptr<RecBlock> pick;
        for (const auto &b : pool)
            if (b.use_count() == 1 && (!pick || better(*b, *pick))) pick = b;
        if (!pick && pool.size() >= kMaxRecBlocks) {
            pick = *std::min_element(pool.begin(), pool.end(),
                                     [](const auto &a, const auto &b) { return a->used_run < b->used_run; });
            for (uint32_t p = 0; p < P; ++p) {
                Producer &pr = prod[p];
                std::lock_guard<std::mutex> g(pr.omu);
                for (OutChunk &ch : pr.outbox)
                    if (ch.blk == pick) {
                        ch.own.assign(ch.p, ch.p + ch.n);
                        ch.p = ch.own.data();
                        ch.blk.reset();
                    }
            }
        }
        if (!pick) {
            pool.push_back(std::make_shared<RecBlock>());
            pick = pool.back();
        }
        // the last holder released it (a release decrement): its reads are over
        std::atomic_thread_fence(std::memory_order_acquire);
        if (pick->cap < need) {
            if (pick->h) (void)hipHostFree(pick->h);
            pick->h = nullptr;
            pick->cap = 0;
            const uint64_t want = need + need / 4 + 1024;
            GSS_HIP(hipHostMalloc((void **)&pick->h, want * sizeof(gss_report), hipHostMallocDefault));
            pick->cap = want;
        }
        pick->used_run = run_id;
        return pick;
    };

    auto finish = [&]() {
        uint64_t n = 0;
        gss_status rc = GSS_OK;
        timed(res.wait_ms, [&] { rc = gss_test_wait(ctx, &n); });
        pending = false;
        const bool overflow = rc == GSS_ERR_REPORT_OVERFLOW;
        if (rc != GSS_OK && !overflow) throw Error(rc, C.last_error);
        const uint64_t this_run = run_id - 1;
        res.runs++;
        if (overflow) {
            // records were lost (the segments are grown now): the words are tested
            // again, with a newer snapshot where one is staged
            res.overflowed_runs++;
            if (log) std::fprintf(log, "X %llu %llu\n", (unsigned long long)this_run, (unsigned long long)n);
            for (uint32_t p = 0; p < P; ++p)
                if (inflight[p] >= 0) {
                    if (staged[p] < 0)
                        staged[p] = inflight[p];
                    else
                        res.dropped++;
                    inflight[p] = -1.0;
                }
            return;
        }
        // activities (Section 3.7): every clause with a record in this run is
        // bumped, queued before the next run overwrites the segments
        if (cfg.evict_keep > 0) {
            priority_bump_hits(C);
            if (log) std::fprintf(log, "B %llu\n", (unsigned long long)this_run);
        }
        // routes the records of the run fetched before this one, then starts this
        // run's fetch; the next run is launched without waiting for it
        if (fq.active) route_fetch(true);
        const int k = next_k;
        next_k ^= 1;
        std::shared_ptr<RecBlock> blk = take_block(n);
        gss_report *place = nullptr;  // where the routing kernel writes the records
        if (n > fdev_cap[k]) {
            C.dfree(fdev[k]);
            fdev[k] = nullptr;
            fdev_cap[k] = 0;
            const uint64_t want = n + n / 4 + 1024;
            try {
                fdev[k] = (gss_report *)C.dalloc(want * sizeof(gss_report));
                fdev_cap[k] = want;
            } catch (const Error &e) {
                if (e.code != GSS_ERR_CAPACITY) throw;
                // no room in the HBM budget: the records go straight into the pinned
                // host buffer (written over the bus)
                void *hd = nullptr;
                GSS_HIP(hipHostGetDevicePointer(&hd, blk->h, 0));
                place = (gss_report *)hd;
            }
        }
        timed(res.fetch_ms, [&] {
            if (n) {  // the records sorted by word on the device, then to the host with the word offsets
                uint32_t *counts = route_dev, *cursor = route_dev + kChunkWords;
                unsigned long long *offs = (unsigned long long *)(route_dev + 2 * kChunkWords);
                launch_fill_u32(C, counts, kChunkWords, 0);
                const unsigned grid = std::max<uint32_t>(1, std::min<uint32_t>(C.last_waves, 1024));
                hipLaunchKernelGGL(k_route_count, dim3(grid), dim3(256), 0, C.stream, C.reports, C.seg_counts,
                                   C.seg_cap, C.last_waves, counts);
                GSS_HIP(hipGetLastError());
                hipLaunchKernelGGL(k_route_scan, dim3(1), dim3(64), 0, C.stream, counts, C.W, cursor, offs);
                GSS_HIP(hipGetLastError());
                hipLaunchKernelGGL(k_route_place, dim3(grid), dim3(256), 0, C.stream, C.reports, C.seg_counts,
                                   C.seg_cap, C.last_waves, cursor, place ? place : fdev[k]);
                GSS_HIP(hipGetLastError());
                GSS_HIP(hipEventRecord(ev_stitched, C.stream));
                GSS_HIP(hipStreamWaitEvent(fetch_stream, ev_stitched, 0));
                if (!place)
                    GSS_HIP(hipMemcpyAsync(blk->h, fdev[k], n * sizeof(gss_report), hipMemcpyDeviceToHost,
                                           fetch_stream));
                GSS_HIP(hipMemcpyAsync(roff[k], offs, (C.W + 1) * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                       fetch_stream));
            }
            GSS_HIP(hipEventRecord(ev_fetched[k], fetch_stream));
        });
        fq.active = true;
        fq.run = this_run;
        fq.n = n;
        fq.k = k;
        fq.blk = std::move(blk);
        fq.arrivals = inflight;
        std::fill(inflight.begin(), inflight.end(), -1.0);
    };

    try {
        GSS_HIP(hipSetDevice(C.device));
        route_dev = (uint32_t *)C.dalloc(2 * kChunkWords * 4 + (kChunkWords + 1) * 8);
        for (auto &o : roff)
            GSS_HIP(hipHostMalloc((void **)&o, (kChunkWords + 1) * sizeof(unsigned long long), hipHostMallocDefault));
        double last_change = now();
        for (;;) {
            const bool stopping = stop.load();
            phase = "taking snapshots";
            if (!stopping) timed(res.admit_ms, admit);
            if (pending) {
                int done = 0;
                const gss_status rq = gss_test_query(ctx, &done);
                if (rq != GSS_OK) throw Error(rq, C.last_error);
                if (!done && !stopping) {
                    // the previous run's records, while this one executes
                    if (!route_fetch(false)) std::this_thread::sleep_for(std::chrono::microseconds(20));
                    continue;
                }
                phase = "completing a run";
                finish();
            }
            if (stopping) {
                route_fetch(true);
                break;
            }
            // ---- next run: every word with an untested snapshot
            uint32_t n_act = 0;
            std::fill(act.begin(), act.end(), 0);
            for (uint32_t p = 0; p < P; ++p)
                if (staged[p] >= 0) {
                    act[p] = ~0ull;
                    inflight[p] = staged[p];
                    staged[p] = -1.0;
                    ++n_act;
                }
            if (!n_act) {
                route_fetch(false);
                if (now() - last_change > 0.005) {
                    phase = "changing the store";
                    timed(res.store_ms, change_store);
                    last_change = now();
                }
                std::this_thread::sleep_for(std::chrono::microseconds(50));
                continue;
            }
            const double launch_t0 = now();
            phase = "launching a run";
            apply_deltas();
            gss_status rc = gss_set_active(ctx, act.data());
            if (rc != GSS_OK) throw Error(rc, C.last_error);
            if (log) {
                std::fprintf(log, "T %llu", (unsigned long long)run_id);
                for (uint64_t x : act) std::fprintf(log, " %llx", (unsigned long long)x);
                std::fputc('\n', log);
            }
            res.pairs += C.live * 64ull * n_act;
            rc = gss_test_async(ctx, cfg.test_flags);
            if (rc != GSS_OK) throw Error(rc, C.last_error);
            pending = true;
            run_id++;
            res.launch_ms += (now() - launch_t0) * 1e3;
            phase = "changing the store";
            timed(res.store_ms, change_store);
            last_change = now();
        }
    } catch (const Error &e) {
        fail(e.code, std::string(phase) + ": " + e.what() + " (device bytes " + std::to_string(C.device_bytes) +
                         ", live clauses " + std::to_string(C.live) + ")");
    } catch (const std::bad_alloc &) {
        fail(GSS_ERR_CAPACITY, "host out of memory");
    } catch (const std::exception &e) {
        fail(GSS_ERR_DEVICE, e.what());
    }
    if (pending) {  // an error left a run in flight: complete it so the context is usable
        uint64_t n = 0;
        (void)gss_test_wait(ctx, &n);
    }
    (void)hipStreamSynchronize(C.stream);
    (void)hipStreamSynchronize(fetch_stream);
    for (int k = 0; k < 2; ++k) {
        C.dfree(fdev[k]);
        if (roff[k]) (void)hipHostFree(roff[k]);
    }
    C.dfree(route_dev);
    res.gpu_ms = C.stats.total_kernel_ms - kernel_ms0;
}

extern "C" gss_status gss_server_start(gss_ctx *ctx, const gss_server_config *cfg, gss_server **out) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(cfg && out, GSS_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    GSS_REQUIRE(c.G == 1, GSS_ERR_INVALID_ARG, "a server takes a context of at most 4096 slots");
    GSS_REQUIRE(cfg->n_producers >= 1 && cfg->n_producers <= c.W, GSS_ERR_INVALID_ARG,
                "n_producers must be in 1..max_slots/64 (one 64-slot word each)");
    const uint32_t known = GSS_TEST_TRIGGER | GSS_TEST_NO_EARLY_EXIT | GSS_TEST_NO_HOT | GSS_TEST_AGGREGATE;
    GSS_REQUIRE((cfg->test_flags & ~known) == 0, GSS_ERR_INVALID_ARG, "test flag not allowed for served runs");
    GSS_REQUIRE(cfg->delete_fraction >= 0 && cfg->delete_fraction <= 1, GSS_ERR_INVALID_ARG,
                "delete_fraction must be in [0, 1]");
    GSS_REQUIRE(cfg->evict_keep >= 0 && cfg->evict_keep < 1, GSS_ERR_INVALID_ARG, "evict_keep must be in [0, 1)");
    GSS_REQUIRE(!c.pending, GSS_ERR_STATE, "a test is in flight");
    if (cfg->evict_keep > 0 && !c.prio) {  // activities live in the priority state
        gss_priority_config pc{};
        pc.n_sources = cfg->n_producers;
        pc.seed = cfg->seed;
        const gss_status rc = gss_priority_enable(ctx, &pc);
        if (rc != GSS_OK) throw Error(rc, c.last_error);
    }
    auto s = std::make_unique<gss_server>();
    s->c = &c;
    s->cfg = *cfg;
    s->cfg.log_path = nullptr;
    s->V = c.cfg.num_vars;
    s->P = cfg->n_producers;
    s->q_limit = cfg->max_queued_lits ? cfg->max_queued_lits : (1ull << 26);
    if (cfg->log_path) {
        s->log = std::fopen(cfg->log_path, "w");
        GSS_REQUIRE(s->log, GSS_ERR_INVALID_ARG, std::string("cannot open the log file ") + cfg->log_path);
    }
    s->prod = std::vector<Producer>(s->P);
    try {
        GSS_HIP(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
        GSS_HIP(hipEventCreateWithFlags(&s->ev_copied, hipEventDisableTiming));
        GSS_HIP(hipStreamCreateWithFlags(&s->fetch_stream, hipStreamNonBlocking));
        GSS_HIP(hipEventCreateWithFlags(&s->ev_stitched, hipEventDisableTiming));
        for (hipEvent_t &e : s->ev_fetched) GSS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        const uint32_t first = std::min<uint32_t>(s->V, 1u << 16);
        for (Producer &p : s->prod) {
            p.pos.assign((size_t)s->V + 1, 0);
            for (Mail &m : p.mail) ensure_host(m, first, s->V);
        }
        // every word starts untested and inactive
        std::vector<uint64_t> none(c.W, 0);
        const gss_status rc = gss_set_active(ctx, none.data());
        if (rc != GSS_OK) throw Error(rc, c.last_error);
        c.sync();
    } catch (...) {
        for (Producer &p : s->prod)
            for (Mail &m : p.mail)
                if (m.h) (void)hipHostFree(m.h);
        if (s->ev_copied) (void)hipEventDestroy(s->ev_copied);
        if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
        for (hipEvent_t e : s->ev_fetched)
            if (e) (void)hipEventDestroy(e);
        if (s->ev_stitched) (void)hipEventDestroy(s->ev_stitched);
        if (s->fetch_stream) (void)hipStreamDestroy(s->fetch_stream);
        if (s->log) std::fclose(s->log);
        throw;
    }
    s->t0 = Clock::now();
    c.serving = true;
    gss_server *raw = s.release();
    raw->manager = std::thread([raw] { raw->run(); });
    *out = raw;
    GSS_API_END
}

// Wrapper of the server entry points: exceptions become status codes.
#define GSS_SRV_BEGIN(sp)                     \
    if (!(sp)) return GSS_ERR_INVALID_ARG;    \
    try {
#define GSS_SRV_END(sp)                       \
    }                                         \
    catch (const ::gss::Error &e) {           \
        std::lock_guard<std::mutex> g_((sp)->emu); \
        (sp)->error = e.what();               \
        return e.code;                        \
    }                                         \
    catch (const std::bad_alloc &) {          \
        return GSS_ERR_CAPACITY;              \
    }                                         \
    catch (const std::exception &e) {         \
        std::lock_guard<std::mutex> g_((sp)->emu); \
        (sp)->error = e.what();               \
        return GSS_ERR_DEVICE;                \
    }                                         \
    return GSS_OK;

extern "C" gss_status gss_server_send(gss_server *s, uint32_t producer, uint32_t n_vars, const uint32_t *vars,
                                      const uint64_t *f_words, const uint64_t *t_words) {
    GSS_SRV_BEGIN(s)
    GSS_REQUIRE(!s->failed.load(), GSS_ERR_STATE, "the server's manager stopped on an error");
    GSS_REQUIRE(producer < s->P, GSS_ERR_INVALID_ARG, "producer out of range");
    GSS_REQUIRE(n_vars == 0 || (vars && f_words && t_words), GSS_ERR_INVALID_ARG, "null argument");
    for (uint32_t i = 0; i < n_vars; ++i) {
        GSS_REQUIRE(vars[i] >= 1 && vars[i] <= s->V, GSS_ERR_BAD_LITERAL, "variable out of range");
        GSS_REQUIRE((f_words[i] & t_words[i]) == 0, GSS_ERR_INVALID_ARG, "a slot cannot be both F and T");
    }
    Producer &p = s->prod[producer];
    std::lock_guard<std::mutex> g(p.mu);
    Mail &m = p.mail[p.open];
    ensure_host(m, (uint32_t)std::min<uint64_t>((uint64_t)m.n + n_vars, s->V), s->V);
    uint32_t *mv = m.vars();
    uint64_t *mf = m.f(), *mt = m.t();
    for (uint32_t i = 0; i < n_vars; ++i) {
        const uint32_t v = vars[i];
        uint32_t q = p.pos[v];
        if (!(q < m.n && mv[q] == v)) {
            q = m.n++;
            mv[q] = v;
            p.pos[v] = q;
        }
        mf[q] = f_words[i];
        mt[q] = t_words[i];
    }
    p.snaps++;
    p.arrival = s->now();
    s->n_snapshots++;
    GSS_SRV_END(s)
}

extern "C" gss_status gss_server_insert(gss_server *s, uint32_t producer, const int32_t *lits, const uint64_t *offsets,
                                        uint32_t n) {
    GSS_SRV_BEGIN(s)
    GSS_REQUIRE(!s->failed.load(), GSS_ERR_STATE, "the server's manager stopped on an error");
    GSS_REQUIRE(producer < s->P, GSS_ERR_INVALID_ARG, "producer out of range");
    if (n == 0) return GSS_OK;
    GSS_REQUIRE(lits && offsets, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(offsets[0] == 0, GSS_ERR_INVALID_ARG, "offsets[0] must be 0");
    const int64_t V = s->V;
    Prepared p;  // validation and encoding here, on the producer's thread
    prepare_clauses(V, lits, offsets, n, p, s->c->perm());
    std::lock_guard<std::mutex> g(s->imu);
    if (s->queue.codes.size() + p.codes.size() > s->q_limit) {
        s->n_refused += n;
        throw Error(GSS_ERR_CAPACITY, "insert queue full");
    }
    s->queue.append(p);
    GSS_SRV_END(s)
}

extern "C" gss_status gss_server_poll(gss_server *s, uint32_t producer, gss_report *out, uint64_t cap, uint64_t *out_n,
                                      uint64_t *out_run) {
    GSS_SRV_BEGIN(s)
    GSS_REQUIRE(producer < s->P, GSS_ERR_INVALID_ARG, "producer out of range");
    GSS_REQUIRE(out_n, GSS_ERR_INVALID_ARG, "null argument");
    Producer &p = s->prod[producer];
    std::lock_guard<std::mutex> g(p.omu);
    if (out_run) *out_run = p.last_run;
    if (!out) {
        *out_n = p.out_n;
        p.outbox.clear();
        p.out_n = 0;
        return GSS_OK;
    }
    // copied here, on the caller's thread, from the pinned blocks
    uint64_t k = 0;
    while (k < cap && !p.outbox.empty()) {
        OutChunk &ch = p.outbox.front();
        const uint64_t m = std::min<uint64_t>(cap - k, ch.n);
        std::memcpy(out + k, ch.p, m * sizeof(gss_report));
        k += m;
        ch.p += m;
        ch.n -= m;
        if (ch.n == 0) p.outbox.pop_front();
    }
    p.out_n -= k;
    *out_n = k;
    GSS_SRV_END(s)
}

extern "C" gss_status gss_server_stop(gss_server *s, gss_serve_result *out) {
    if (!s) return GSS_ERR_INVALID_ARG;
    s->stop = true;
    if (s->manager.joinable()) s->manager.join();
    Ctx &c = *s->c;
    c.serving = false;
    gss_serve_result r = s->res;
    r.snapshots = s->n_snapshots.load();
    r.refused = s->n_refused.load();
    r.live_end = c.live;
    r.wall_s = s->now();
    double sum = 0;
    for (double x : s->lat) sum += x;
    r.mean_ms = s->lat.empty() ? 0.0 : sum / (double)s->lat.size();
    r.p50_ms = percentile(s->lat, 0.50);
    r.p99_ms = percentile(s->lat, 0.99);
    r.max_ms = s->lat.empty() ? 0.0 : *std::max_element(s->lat.begin(), s->lat.end());
    (void)hipStreamSynchronize(s->copy_stream);
    (void)hipStreamSynchronize(c.stream);
    for (Producer &p : s->prod)
        for (Mail &m : p.mail) {
            if (m.h) (void)hipHostFree(m.h);
            c.dfree(m.d);
        }
    r.device_bytes_end = c.device_bytes;
    (void)hipEventDestroy(s->ev_copied);
    (void)hipStreamDestroy(s->copy_stream);
    (void)hipStreamSynchronize(s->fetch_stream);
    for (hipEvent_t e : s->ev_fetched) (void)hipEventDestroy(e);
    (void)hipEventDestroy(s->ev_stitched);
    (void)hipStreamDestroy(s->fetch_stream);
    if (s->log) std::fclose(s->log);
    if (out) *out = r;
    const gss_status st = s->status;
    c.last_error = st != GSS_OK ? "the server's manager stopped: " + s->manager_error : s->error;
    delete s;
    return st;
}

extern "C" const char *gss_server_last_error(const gss_server *s) {
    if (!s) return "";
    std::lock_guard<std::mutex> g(s->emu);
    return s->error.c_str();
}
