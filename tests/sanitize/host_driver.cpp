// Host-side sanitizer run of the library (test infrastructure).
//
// The library is built a second time with its host code under AddressSanitizer
// and UndefinedBehaviorSanitizer (the device code is unchanged); this program,
// built with the same sanitizers, drives the C ABI on small inputs: ingest,
// full and partial value updates (host, device, packed, queued), every test mode
// and fetch, removals with compaction, hot-variable ranking, the allocation-free
// test, the learned priority, a batch of two stores and a served session with
// late polls.  Every plain test is compared with the C oracle, bit for bit.  A
// host access out of bounds, a use of freed memory or undefined behaviour in the
// library's host code aborts the run.
#include "gss.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <thread>
#include <vector>

extern "C" {
int oracle_falsified(int64_t n_clauses, const int64_t *offsets, const int32_t *lits, int64_t n_vars, int64_t n_slots,
                     const int8_t *values_vm, const uint8_t *active, uint64_t *out);
int oracle_trigger(int64_t n_clauses, const int64_t *offsets, const int32_t *lits, int64_t n_vars, int64_t n_slots,
                   const int8_t *values_vm, const uint8_t *active, uint64_t *out);
}

namespace {

[[noreturn]] void fail(const char *file, int line, const char *what, const char *detail) {
    std::fprintf(stderr, "FAIL %s:%d: %s %s\n", file, line, what, detail ? detail : "");
    std::exit(1);
}

#define CHECK(cond, detail) \
    do {                                         \
        if (!(cond)) fail(__FILE__, __LINE__, #cond, detail); \
    } while (0)
#define OK(ctx, call)                                                      \
    do {                                                                   \
        const gss_status rc_ = (call);                                     \
        if (rc_ != GSS_OK) fail(__FILE__, __LINE__, #call, gss_last_error(ctx)); \
    } while (0)

using Clauses = std::map<uint32_t, std::vector<int32_t>>;  // live clauses by id

struct Store {
    uint32_t V = 0, S = 0;       // variables, slots (max_slots)
    std::vector<int8_t> values;  // slot-major [S][V]
    std::vector<uint8_t> active; // [S]
    Clauses live;
    uint32_t next_id = 0;
};

std::vector<int32_t> random_clause(std::mt19937_64 &rng, uint32_t V) {
    std::uniform_real_distribution<double> u(0.0, 1.0);
    const uint32_t len = u(rng) < 0.8 ? 1 + (uint32_t)(rng() % 5) : 6 + (uint32_t)(rng() % 60);
    std::vector<int32_t> c(len);
    for (auto &l : c) {
        const int32_t v = 1 + (int32_t)(rng() % V);
        l = (rng() & 1) ? v : -v;
    }
    return c;
}

// Adds n random clauses through gss_add_clauses and into the model.
void add_clauses(gss_ctx *ctx, Store &st, std::mt19937_64 &rng, uint32_t n) {
    std::vector<int32_t> lits;
    std::vector<uint64_t> offs{0};
    std::vector<std::vector<int32_t>> cs;
    for (uint32_t i = 0; i < n; ++i) {
        cs.push_back(random_clause(rng, st.V));
        lits.insert(lits.end(), cs.back().begin(), cs.back().end());
        offs.push_back(lits.size());
    }
    std::vector<uint32_t> ids(n);
    OK(ctx, gss_add_clauses(ctx, lits.data(), offs.data(), n, ids.data()));
    for (uint32_t i = 0; i < n; ++i) {
        CHECK(ids[i] == st.next_id + i, "ids are issued in order");
        st.live[ids[i]] = cs[i];
    }
    st.next_id += n;
}

// The oracle's masks, one row of W words per issued id (zero rows for removed ids).
std::vector<uint64_t> expected(const Store &st, bool trigger) {
    const uint32_t W = st.S / 64;
    std::vector<int64_t> offs{0};
    std::vector<int32_t> lits;
    std::vector<uint32_t> ids;
    for (const auto &kv : st.live) {
        ids.push_back(kv.first);
        lits.insert(lits.end(), kv.second.begin(), kv.second.end());
        offs.push_back((int64_t)lits.size());
    }
    std::vector<int8_t> vm((size_t)st.V * st.S);
    for (uint32_t s = 0; s < st.S; ++s)
        for (uint32_t v = 0; v < st.V; ++v) vm[(size_t)v * st.S + s] = st.values[(size_t)s * st.V + v];
    std::vector<uint64_t> rows(ids.size() * W);
    const int rc = (trigger ? oracle_trigger : oracle_falsified)((int64_t)ids.size(), offs.data(), lits.data(), st.V,
                                                                 st.S, vm.data(), st.active.data(), rows.data());
    CHECK(rc == 0, "oracle");
    std::vector<uint64_t> out((size_t)st.next_id * W, 0);
    for (size_t i = 0; i < ids.size(); ++i)
        std::memcpy(&out[(size_t)ids[i] * W], &rows[i * W], W * 8);
    return out;
}

// Records into dense rows; each (clause, word) at most once, never an empty mask.
std::vector<uint64_t> dense_of(const std::vector<gss_report> &r, uint32_t n_ids, uint32_t W) {
    std::vector<uint64_t> d((size_t)n_ids * W, 0);
    for (const gss_report &x : r) {
        CHECK(x.clause_id < n_ids && x.word < W && x.mask != 0, "record in range");
        uint64_t &cell = d[(size_t)x.clause_id * W + x.word];
        CHECK(cell == 0, "record repeated");
        cell = x.mask;
    }
    return d;
}

std::vector<gss_report> fetch(gss_ctx *ctx, uint64_t n) {
    std::vector<gss_report> r(std::max<uint64_t>(n, 1));
    uint64_t got = 0;
    OK(ctx, gss_fetch_reports(ctx, r.data(), n, &got));
    CHECK(got == n, "fetched every record");
    r.resize(got);
    return r;
}

void check_test(gss_ctx *ctx, const Store &st, uint32_t flags, const char *what) {
    uint64_t n = 0;
    OK(ctx, gss_test(ctx, flags, &n));
    const std::vector<gss_report> r = fetch(ctx, n);
    if (flags & GSS_TEST_SORTED)
        for (size_t i = 1; i < r.size(); ++i)
            CHECK(r[i - 1].clause_id < r[i].clause_id ||
                      (r[i - 1].clause_id == r[i].clause_id && r[i - 1].word < r[i].word),
                  what);
    CHECK(dense_of(r, st.next_id, st.S / 64) == expected(st, flags & GSS_TEST_TRIGGER), what);
    std::printf("  %s: %llu records\n", what, (unsigned long long)n);
}

void random_values(std::mt19937_64 &rng, int8_t *v, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        const uint64_t x = rng() % 10;
        v[i] = x < 4 ? -1 : x < 7 ? 1 : 0;
    }
}

void single_store(hipStream_t stream) {
    std::puts("single store");
    std::mt19937_64 rng(11);
    Store st;
    st.V = 2500;
    st.S = 256;
    st.values.assign((size_t)st.S * st.V, 0);
    st.active.assign(st.S, 0);
    gss_config cfg{};
    cfg.num_vars = st.V;
    cfg.max_slots = st.S;
    cfg.report_capacity = 4096;  // small: the first tests grow the segments
    cfg.stream = stream;
    cfg.hot_vars = 32;
    cfg.timing_interval = 2;
    gss_ctx *ctx = nullptr;
    OK(nullptr, gss_create(&cfg, &ctx));
    add_clauses(ctx, st, rng, 20000);

    // assignments in slots 0..199; slots 200..255 stay inactive
    const uint32_t n_act = 200;
    random_values(rng, st.values.data(), (size_t)n_act * st.V);
    std::fill(st.active.begin(), st.active.begin() + n_act, 1);
    OK(ctx, gss_set_assignments(ctx, 0, n_act, st.values.data()));
    check_test(ctx, st, GSS_TEST_FALSIFIED, "falsified");
    check_test(ctx, st, GSS_TEST_TRIGGER, "trigger");
    check_test(ctx, st, GSS_TEST_AGGREGATE, "aggregate");
    check_test(ctx, st, GSS_TEST_TRIGGER | GSS_TEST_AGGREGATE, "trigger aggregate");
    check_test(ctx, st, GSS_TEST_NO_EARLY_EXIT | GSS_TEST_NO_HOT, "no early exit, no staging");
    check_test(ctx, st, GSS_TEST_SORTED, "sorted");
    check_test(ctx, st, GSS_TEST_COUNT, "counted");
    {  // dense masks of every id
        uint64_t n = 0;
        OK(ctx, gss_test(ctx, GSS_TEST_DENSE, &n));
        std::vector<uint32_t> ids(st.next_id);
        for (uint32_t i = 0; i < st.next_id; ++i) ids[i] = i;
        std::vector<uint64_t> m((size_t)st.next_id * (st.S / 64));
        OK(ctx, gss_fetch_masks(ctx, ids.data(), st.next_id, m.data()));
        CHECK(m == expected(st, false), "dense masks");
    }

    // a host delta of 300 variables on slots 10..189
    {
        std::vector<uint32_t> vars;
        for (uint32_t v = 1; v <= st.V; v += 8) vars.push_back(v);
        const uint32_t first = 10, ns = 180;
        std::vector<int8_t> vm(vars.size() * ns);
        random_values(rng, vm.data(), vm.size());
        for (size_t i = 0; i < vars.size(); ++i)
            for (uint32_t s = 0; s < ns; ++s) st.values[(size_t)(first + s) * st.V + vars[i] - 1] = vm[i * ns + s];
        OK(ctx, gss_set_var_values(ctx, first, ns, (uint32_t)vars.size(), vars.data(), vm.data()));
        check_test(ctx, st, 0, "after a host delta");
    }
    // a packed delta of word 1
    {
        std::vector<uint32_t> vars;
        std::vector<uint64_t> f, t;
        for (uint32_t v = 3; v <= st.V; v += 5) {
            const uint64_t r = rng();
            vars.push_back(v);
            f.push_back(r & 0x5555555555555555ull);
            t.push_back(r & 0xAAAAAAAAAAAAAAAAull);
            for (uint32_t b = 0; b < 64; ++b)
                st.values[(size_t)(64 + b) * st.V + v - 1] = (f.back() >> b) & 1 ? -1 : (t.back() >> b) & 1 ? 1 : 0;
        }
        OK(ctx, gss_update_words(ctx, 1, (uint32_t)vars.size(), vars.data(), f.data(), t.data()));
        check_test(ctx, st, 0, "after a packed delta");
    }
    // a queued delta from device memory, then an asynchronous test
    {
        std::vector<uint32_t> vars;
        for (uint32_t v = 2; v <= st.V; v += 7) vars.push_back(v);
        const uint32_t ns = n_act;
        std::vector<int8_t> vm(vars.size() * ns);
        random_values(rng, vm.data(), vm.size());
        for (size_t i = 0; i < vars.size(); ++i)
            for (uint32_t s = 0; s < ns; ++s) st.values[(size_t)s * st.V + vars[i] - 1] = vm[i * ns + s];
        int8_t *d = nullptr;
        CHECK(hipMalloc((void **)&d, vm.size()) == hipSuccess, "hipMalloc");
        CHECK(hipMemcpy(d, vm.data(), vm.size(), hipMemcpyHostToDevice) == hipSuccess, "hipMemcpy");
        OK(ctx, gss_set_var_values_async(ctx, 0, ns, (uint32_t)vars.size(), vars.data(), d));
        OK(ctx, gss_test_async(ctx, 0));
        uint64_t n = 0;
        OK(ctx, gss_test_wait(ctx, &n));
        CHECK(dense_of(fetch(ctx, n), st.next_id, st.S / 64) == expected(st, false), "after a queued delta");
        CHECK(hipFree(d) == hipSuccess, "hipFree");
        std::puts("  queued delta and asynchronous test: ok");
    }
    // removals of 45% (compaction), more inserts, ranking
    {
        std::vector<uint32_t> ids;
        for (const auto &kv : st.live)
            if (rng() % 100 < 45) ids.push_back(kv.first);
        std::shuffle(ids.begin(), ids.end(), rng);
        OK(ctx, gss_remove_clauses(ctx, ids.data(), (uint32_t)ids.size()));
        for (uint32_t id : ids) st.live.erase(id);
        CHECK(gss_remove_clauses(ctx, ids.data(), 1) == GSS_ERR_UNKNOWN_ID, "removed twice");
        check_test(ctx, st, 0, "after removals");
        add_clauses(ctx, st, rng, 6000);
        uint64_t hot = 0, all = 0;
        OK(ctx, gss_rank_vars(ctx, &hot, &all));
        CHECK(hot <= all && all > 0, "ranking");
        check_test(ctx, st, 0, "after inserts and ranking");
        check_test(ctx, st, GSS_TEST_TRIGGER | GSS_TEST_AGGREGATE, "trigger aggregate after changes");
    }
    // the allocation-free test into a device buffer
    {
        const uint64_t cap = 1 << 20;
        gss_report *d = nullptr;
        CHECK(hipMalloc((void **)&d, cap * sizeof(gss_report)) == hipSuccess, "hipMalloc");
        uint64_t n = 0;
        OK(ctx, gss_test_noalloc(ctx, 0, d, cap, &n));
        std::vector<gss_report> r(n);
        CHECK(hipMemcpy(r.data(), d, n * sizeof(gss_report), hipMemcpyDeviceToHost) == hipSuccess, "hipMemcpy");
        CHECK(dense_of(r, st.next_id, st.S / 64) == expected(st, false), "allocation-free test");
        CHECK(hipFree(d) == hipSuccess, "hipFree");
        std::puts("  allocation-free test: ok");
    }
    // learned priority: samples, training, scoring, a scheduled test, activity reduction
    {
        gss_priority_config pc{};
        pc.n_sources = 1;
        pc.sample_period = 3;
        pc.sample_capacity = 1 << 16;
        pc.seed = 5;
        OK(ctx, gss_priority_enable(ctx, &pc));
        for (int r = 0; r < 4; ++r) {
            uint64_t n = 0;
            OK(ctx, gss_test(ctx, 0, &n));
            OK(ctx, gss_priority_observe(ctx));
        }
        gss_adam_config ac{};
        ac.lr = 1e-3f;
        ac.beta1 = 0.9f;
        ac.beta2 = 0.999f;
        ac.eps = 1e-8f;
        ac.batch = 512;
        float loss = 0.f;
        OK(ctx, gss_priority_train(ctx, 1, &ac, 3, &loss));
        uint64_t n_low = 0;
        OK(ctx, gss_priority_score(ctx, 0.5f, &n_low));
        uint64_t n = 0;
        for (int r = 0; r < 3; ++r) {
            OK(ctx, gss_test(ctx, GSS_TEST_SCHEDULED, &n));
            (void)fetch(ctx, n);
            OK(ctx, gss_priority_observe(ctx));
            OK(ctx, gss_priority_update(ctx, &n_low));
        }
        uint64_t live = 0, removed = 0;
        OK(ctx, gss_store_info(ctx, &live, nullptr, nullptr));
        OK(ctx, gss_priority_reduce(ctx, live / 2, &removed));
        uint64_t live2 = 0;
        OK(ctx, gss_store_info(ctx, &live2, nullptr, nullptr));
        CHECK(live2 + removed == live, "reduce");
        std::printf("  priority: %llu low, %llu removed by activity\n", (unsigned long long)n_low,
                    (unsigned long long)removed);
    }
    gss_stats s{};
    OK(ctx, gss_get_stats(ctx, &s));
    CHECK(s.timed_launches > 0 && s.timed_launches < s.kernel_launches, "timing interval");
    gss_destroy(ctx);
}

void batch_of_two(hipStream_t stream) {
    std::puts("batch");
    std::mt19937_64 rng(12);
    Store st[2];
    gss_ctx *ctx[2] = {nullptr, nullptr};
    for (int k = 0; k < 2; ++k) {
        st[k].V = k ? 900 : 3000;
        st[k].S = k ? 64 : 512;
        st[k].values.assign((size_t)st[k].S * st[k].V, 0);
        st[k].active.assign(st[k].S, 1);
        gss_config cfg{};
        cfg.num_vars = st[k].V;
        cfg.max_slots = st[k].S;
        cfg.report_capacity = 1 << 16;
        cfg.stream = stream;
        OK(nullptr, gss_create(&cfg, &ctx[k]));
        add_clauses(ctx[k], st[k], rng, k ? 5000 : 12000);
        random_values(rng, st[k].values.data(), st[k].values.size());
        OK(ctx[k], gss_set_assignments(ctx[k], 0, st[k].S, st[k].values.data()));
    }
    gss_batch *b = nullptr;
    CHECK(gss_batch_create(ctx, 2, &b) == GSS_OK, gss_batch_last_error(b));
    for (int rep = 0; rep < 3; ++rep) {
        uint64_t n[2] = {0, 0};
        CHECK(gss_batch_test(b, 0, n) == GSS_OK, gss_batch_last_error(b));
        for (int k = 0; k < 2; ++k)
            CHECK(dense_of(fetch(ctx[k], n[k]), st[k].next_id, st[k].S / 64) == expected(st[k], false), "batch");
    }
    // asynchronous: the next round's delta of store 0 queued behind the batch in flight
    {
        Store &s0 = st[0];
        std::vector<uint32_t> vars;
        for (uint32_t v = 1; v <= s0.V; v += 9) vars.push_back(v);
        std::vector<int8_t> vm(vars.size() * s0.S);
        random_values(rng, vm.data(), vm.size());
        int8_t *d = nullptr;
        CHECK(hipMalloc((void **)&d, vm.size()) == hipSuccess, "hipMalloc");
        CHECK(hipMemcpy(d, vm.data(), vm.size(), hipMemcpyHostToDevice) == hipSuccess, "hipMemcpy");
        CHECK(gss_batch_test_async(b, 0) == GSS_OK, gss_batch_last_error(b));
        uint64_t dummy = 0;
        CHECK(gss_test(ctx[0], 0, &dummy) == GSS_ERR_STATE, "a member refuses a test while the batch runs");
        OK(ctx[0], gss_set_var_values_async(ctx[0], 0, s0.S, (uint32_t)vars.size(), vars.data(), d));
        uint64_t n[2] = {0, 0};
        CHECK(gss_batch_wait(b, n) == GSS_OK, gss_batch_last_error(b));
        for (int k = 0; k < 2; ++k)
            CHECK(dense_of(fetch(ctx[k], n[k]), st[k].next_id, st[k].S / 64) == expected(st[k], false), "async batch");
        for (size_t i = 0; i < vars.size(); ++i)
            for (uint32_t s = 0; s < s0.S; ++s) s0.values[(size_t)s * s0.V + vars[i] - 1] = vm[i * s0.S + s];
        CHECK(gss_batch_test(b, 0, n) == GSS_OK, gss_batch_last_error(b));
        for (int k = 0; k < 2; ++k)
            CHECK(dense_of(fetch(ctx[k], n[k]), st[k].next_id, st[k].S / 64) == expected(st[k], false),
                  "batch after the queued delta");
        CHECK(hipFree(d) == hipSuccess, "hipFree");
    }
    gss_batch_destroy(b);
    for (auto *c : ctx) gss_destroy(c);
    std::puts("  two stores, batched tests (one asynchronous, a delta queued behind it): ok");
}

void served(hipStream_t stream) {
    std::puts("served");
    std::mt19937_64 rng(13);
    Store st;
    st.V = 3000;
    st.S = 256;
    gss_config cfg{};
    cfg.num_vars = st.V;
    cfg.max_slots = st.S;
    cfg.report_capacity = 1 << 16;
    cfg.stream = stream;
    gss_ctx *ctx = nullptr;
    OK(nullptr, gss_create(&cfg, &ctx));
    add_clauses(ctx, st, rng, 15000);
    gss_server_config sc{};
    sc.n_producers = 4;
    sc.delete_fraction = 0.2;
    sc.seed = 3;
    gss_server *srv = nullptr;
    OK(ctx, gss_server_start(ctx, &sc, &srv));
    std::vector<uint32_t> vars(st.V);
    for (uint32_t v = 0; v < st.V; ++v) vars[v] = v + 1;
    std::vector<uint64_t> f(st.V), t(st.V);
    std::vector<gss_report> out(777);
    uint64_t got_total = 0;
    for (int round = 0; round < 30; ++round) {
        for (uint32_t p = 0; p < sc.n_producers; ++p) {
            for (uint32_t v = 0; v < st.V; ++v) {
                const uint64_t r = rng();
                f[v] = r & 0x1111111111111111ull;
                t[v] = (r >> 1) & 0x2222222222222222ull;
            }
            CHECK(gss_server_send(srv, p, st.V, vars.data(), f.data(), t.data()) == GSS_OK, gss_server_last_error(srv));
            std::vector<int32_t> lits;
            std::vector<uint64_t> offs{0};
            for (int i = 0; i < 20; ++i) {
                const auto c = random_clause(rng, st.V);
                lits.insert(lits.end(), c.begin(), c.end());
                offs.push_back(lits.size());
            }
            CHECK(gss_server_insert(srv, p, lits.data(), offs.data(), 20) == GSS_OK, gss_server_last_error(srv));
            // producers 0 and 1 poll in small pieces; 2 and 3 only at the end
            if (p < 2) {
                uint64_t n = 0, run = 0;
                CHECK(gss_server_poll(srv, p, out.data(), out.size(), &n, &run) == GSS_OK, gss_server_last_error(srv));
                got_total += n;
            }
        }
        std::this_thread::sleep_for(std::chrono::milliseconds(3));
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(200));
    for (uint32_t p = 0; p < sc.n_producers; ++p)
        for (;;) {
            uint64_t n = 0, run = 0;
            CHECK(gss_server_poll(srv, p, out.data(), out.size(), &n, &run) == GSS_OK, gss_server_last_error(srv));
            got_total += n;
            if (n == 0) break;
        }
    gss_serve_result res{};
    OK(ctx, gss_server_stop(srv, &res));
    CHECK(res.runs > 0 && res.inserted > 0 && got_total <= res.reports, "server results");
    std::printf("  %llu runs, %llu records, %llu collected by the producers\n", (unsigned long long)res.runs,
                (unsigned long long)res.reports, (unsigned long long)got_total);
    // the workload generator on the same context (usable again once the server stopped)
    gss_sim_config sim{};
    sim.n_threads = 4;
    sim.duration_s = 0.5;
    sim.snapshot_rate = 100.0;
    sim.redraw_fraction = 0.05;
    sim.insert_rate = 2000.0;
    sim.delete_fraction = 0.05;
    sim.seed = 9;
    sim.test_flags = GSS_TEST_AGGREGATE;
    OK(ctx, gss_serve_simulate(ctx, &sim, &res));
    std::printf("  generator: %llu runs\n", (unsigned long long)res.runs);
    gss_destroy(ctx);
}

}  // namespace

int main() {
    std::setvbuf(stdout, nullptr, _IOLBF, 0);  // progress survives an abort
    hipStream_t stream = nullptr;
    CHECK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess, "stream");
    single_store(stream);
    batch_of_two(stream);
    served(stream);
    CHECK(hipStreamDestroy(stream) == hipSuccess, "stream");
    std::puts("host sanitizer run: ok");
    std::fflush(stdout);
    // Every check has run.  The HIP runtime's own teardown at exit can trip
    // AddressSanitizer's device-allocator bookkeeping (an assertion inside the
    // sanitizer runtime, in no code of this library), so the process ends here.
    std::_Exit(0);
}
