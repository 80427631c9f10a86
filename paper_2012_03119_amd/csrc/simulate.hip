// Served workload generator: simulated solver threads driving a gss_server.
//
// Each thread stands for one solver thread of the paper's parallel solver: it
// sends snapshots of its 64 assignments and exports learned clauses.  Snapshot
// values follow Table 1 (how often a variable takes each subset of {T, F, U}
// over successive assignments of one thread); successive snapshots of a thread
// differ in a fraction of the variables, so they travel as deltas.
#include "gss_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>

namespace {

using Clock = std::chrono::steady_clock;

// xoshiro256** (Blackman and Vigna), seeded through splitmix64.
struct Rng {
    uint64_t s[4];
    explicit Rng(uint64_t seed) {
        for (auto &x : s) {
            uint64_t z = (seed += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            x = z ^ (z >> 31);
        }
    }
    static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
    uint64_t next() {
        const uint64_t r = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
        s[2] ^= s[0];
        s[3] ^= s[1];
        s[1] ^= s[2];
        s[0] ^= s[3];
        s[2] ^= t;
        s[3] = rotl(s[3], 45);
        return r;
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    uint64_t below(uint64_t n) { return (uint64_t)(uniform() * (double)n); }
};

// Table 1 frequencies, in the order {T} {F} {T,F} {U} {T,U} {F,U} {T,F,U};
// cumulative thresholds out of 2^16.
struct Table1 {
    uint32_t cum[7];
    Table1() {
        const double w[7] = {0.127, 0.064, 0.000, 0.660, 0.060, 0.068, 0.021};
        double acc = 0, tot = 0;
        for (double x : w) tot += x;
        for (int k = 0; k < 7; ++k) cum[k] = (uint32_t)std::llround((acc += w[k] / tot) * 65536.0);
        cum[6] = 65536;
    }
    // The (F-slots, T-slots) words of one variable in one snapshot.
    void draw(Rng &r, uint64_t &f, uint64_t &t) const {
        const uint64_t a = r.next();
        const uint32_t u = (uint32_t)(a & 0xFFFF);
        int k = 0;
        while (u >= cum[k]) ++k;
        const uint64_t x = r.next();
        switch (k) {
        case 0: f = 0; t = ~0ull; break;  // {T}
        case 1: f = ~0ull; t = 0; break;  // {F}
        case 2: f = x; t = ~x; break;     // {T,F}
        case 3: f = 0; t = 0; break;      // {U}
        case 4: f = 0; t = x; break;      // {T,U}
        case 5: f = x; t = 0; break;      // {F,U}
        default: {                        // {T,F,U}: each slot uniform over the three
            f = t = 0;
            uint64_t bits = x;
            int left = 32;
            for (int b = 0; b < 64; ++b) {
                uint64_t v;
                do {
                    if (left == 0) {
                        bits = r.next();
                        left = 32;
                    }
                    v = bits & 3;
                    bits >>= 2;
                    --left;
                } while (v == 3);
                if (v == 1) f |= 1ull << b;
                if (v == 2) t |= 1ull << b;
            }
        }
        }
    }
};

// Learned clause lengths: half in 2..10, 40% in 11..50, 10% in 51..300.
uint32_t draw_length(Rng &r) {
    const double u = r.uniform();
    if (u < 0.5) return 2 + (uint32_t)r.below(9);
    if (u < 0.9) return 11 + (uint32_t)r.below(40);
    return 51 + (uint32_t)r.below(250);
}

struct Shared {
    gss_server *srv;
    gss_sim_config cfg;
    uint32_t V;
    std::atomic<bool> stop{false};
    std::atomic<int> status{GSS_OK};
    Clock::time_point t0;
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

void solver_thread(Shared &sh, uint32_t id) {
    const gss_sim_config &cfg = sh.cfg;
    const uint32_t V = sh.V;
    Rng r(cfg.seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull * (id + 1));
    const Table1 tab;
    std::vector<uint32_t> vars;
    std::vector<uint64_t> f, t;
    auto send = [&]() {
        const gss_status rc = gss_server_send(sh.srv, id, (uint32_t)vars.size(), vars.data(), f.data(), t.data());
        if (rc != GSS_OK) {
            sh.status = rc;
            sh.stop = true;
        }
    };
    // full first snapshot
    vars.resize(V);
    f.resize(V);
    t.resize(V);
    for (uint32_t v = 0; v < V; ++v) {
        vars[v] = v + 1;
        tab.draw(r, f[v], t[v]);
    }
    send();
    // later snapshots redraw runs of 64 consecutive variables
    const uint32_t nb = (V + 63) / 64;
    const uint32_t k_blocks = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(nb, std::llround(cfg.redraw_fraction * nb)));
    std::vector<uint32_t> perm(nb);
    for (uint32_t b = 0; b < nb; ++b) perm[b] = b;
    auto expo = [&](double rate) { return -std::log(1.0 - r.uniform()) / rate; };
    double next_snap = sh.now() + expo(cfg.snapshot_rate);
    const double tick = 0.01;
    double next_ins = sh.now() + tick, ins_due = 0;
    std::vector<int32_t> lits;
    std::vector<uint64_t> offs;
    std::vector<uint32_t> seen(V + 1, 0);  // variables drawn for the current clause (by stamp)
    uint32_t stamp = 0;
    while (!sh.stop.load(std::memory_order_relaxed)) {
        const double now = sh.now();
        if (now >= next_snap) {
            vars.clear();
            f.clear();
            t.clear();
            for (uint32_t i = 0; i < k_blocks; ++i) {  // distinct blocks: partial Fisher-Yates
                const uint32_t j = i + (uint32_t)r.below(nb - i);
                std::swap(perm[i], perm[j]);
                const uint32_t lo = perm[i] * 64 + 1, hi = std::min<uint32_t>(V, lo + 63);
                for (uint32_t v = lo; v <= hi; ++v) {
                    uint64_t fv, tv;
                    tab.draw(r, fv, tv);
                    vars.push_back(v);
                    f.push_back(fv);
                    t.push_back(tv);
                }
            }
            send();
            next_snap += expo(cfg.snapshot_rate);
        }
        if (now >= next_ins) {
            ins_due += cfg.insert_rate * tick;
            const uint32_t n = (uint32_t)ins_due;
            ins_due -= n;
            if (n) {
                lits.clear();
                offs.assign(1, 0);
                for (uint32_t c = 0; c < n; ++c) {
                    const uint32_t L = std::min(draw_length(r), V);
                    const size_t base = lits.size();
                    ++stamp;
                    while (lits.size() - base < L) {  // distinct variables
                        const uint32_t v = 1 + (uint32_t)r.below(V);
                        if (seen[v] == stamp) continue;
                        seen[v] = stamp;
                        lits.push_back((r.next() & 1) ? (int32_t)v : -(int32_t)v);
                    }
                    offs.push_back(lits.size());
                }
                const gss_status rc = gss_server_insert(sh.srv, id, lits.data(), offs.data(), n);
                if (rc != GSS_OK && rc != GSS_ERR_CAPACITY) {
                    sh.status = rc;
                    sh.stop = true;
                }
            }
            next_ins += tick;
        }
        uint64_t got = 0;
        (void)gss_server_poll(sh.srv, id, nullptr, 0, &got, nullptr);  // records are discarded
        const double wait = std::min(next_snap, next_ins) - sh.now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.001)));
    }
}

}  // namespace

using namespace gss;

extern "C" gss_status gss_serve_simulate(gss_ctx *ctx, const gss_sim_config *cfg, gss_serve_result *out) {
    GSS_API_BEGIN(ctx)
    Ctx &c = *c_;
    GSS_REQUIRE(cfg && out, GSS_ERR_INVALID_ARG, "null argument");
    GSS_REQUIRE(cfg->duration_s > 0 && cfg->snapshot_rate > 0 && cfg->insert_rate >= 0, GSS_ERR_INVALID_ARG,
                "duration and snapshot rate must be positive, insert rate non-negative");
    GSS_REQUIRE(cfg->redraw_fraction > 0 && cfg->redraw_fraction <= 1, GSS_ERR_INVALID_ARG,
                "redraw_fraction must be in (0, 1]");
    gss_server_config sc{};
    sc.n_producers = cfg->n_threads;
    sc.test_flags = cfg->test_flags;
    sc.delete_fraction = cfg->delete_fraction;
    sc.seed = cfg->seed;
    sc.log_path = cfg->log_path;
    sc.evict_keep = cfg->evict_keep;
    gss_server *srv = nullptr;
    gss_status rc = gss_server_start(ctx, &sc, &srv);
    if (rc != GSS_OK) return rc;
    Shared sh;
    sh.srv = srv;
    sh.cfg = *cfg;
    sh.V = c.cfg.num_vars;
    sh.t0 = Clock::now();
    std::vector<std::thread> threads;
    try {
        for (uint32_t i = 0; i < cfg->n_threads; ++i) threads.emplace_back(solver_thread, std::ref(sh), i);
    } catch (...) {
        sh.stop = true;
    }
    while (!sh.stop.load() && sh.now() < cfg->duration_s)
        std::this_thread::sleep_for(std::chrono::milliseconds(5));
    sh.stop = true;
    for (auto &x : threads) x.join();
    rc = gss_server_stop(srv, out);  // sets the context's last error
    if (rc != GSS_OK) return rc;
    GSS_REQUIRE(threads.size() == cfg->n_threads, GSS_ERR_DEVICE, "could not start the solver threads");
    if (sh.status != GSS_OK) throw Error((gss_status)sh.status.load(), "a solver thread's call failed");
    GSS_API_END
}
