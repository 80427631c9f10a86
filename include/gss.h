/*
 * gss.h -- C ABI of the MI355X clause-test library (libgss.so).
 *
 * The library keeps a database of clauses and a set of up to `max_slots` partial
 * assignments resident in GPU memory and finds every (clause, assignment) pair in
 * which the clause is falsified: each of its literals is F under the assignment.
 * This is the test at the heart of GpuShareSat (Section 3.4 and its listing of the
 * bitwise trigger test; Section 3.5 for running it on millions of clauses at
 * once), restricted to the conflict half of Definition 1 (Section 3.3); the full
 * trigger predicate is available as a flag.
 *
 * The calls follow the paper's description of the exchange (Section 3.6): solver
 * threads export clauses (gss_add_clauses), send assignments (gss_set_assignments
 * and the delta calls), the GPU tests every clause against every assignment it
 * holds and reports the hits (gss_test, gss_fetch_reports), and clauses leave the
 * GPU again (gss_remove_clauses, Section 3.7 on deleting GPU clauses).
 *
 * Conventions for every call:
 *  - Return value: GSS_OK (0) or a negative gss_status (gss_poll alone may also
 *    return the positive GSS_NOT_READY).  No exception, abort or
 *    longjmp crosses this interface.  After an error, gss_last_error() holds a
 *    message.  Errors detected while validating arguments leave the context
 *    unchanged (validate, then apply).  GSS_ERR_DEVICE means a HIP call failed;
 *    the context may then be unusable and should be destroyed.
 *  - Input arrays are owned by the caller and are not retained after the call
 *    returns (gss_set_var_values_async states its own longer lifetime for its
 *    device values).  Unless a call says otherwise they are host memory.  Calls
 *    marked "host or device" also accept device pointers (detected with
 *    hipPointerGetAttributes); device inputs must stay valid until the call returns.
 *  - A context is not thread-safe: one thread drives it, like the single GPU
 *    manager thread of the paper's solver (Section 5).  Work is issued on the
 *    context's stream; calls that return results synchronise that stream.
 *  - Literals are DIMACS signed int32: variable v in 1..num_vars, -v its negation.
 *  - Truth values are int8: +1 = T, -1 = F, 0 = U (Section 3.1).
 *  - Assignment slots are numbered 0..max_slots-1; slot s is bit s%64 of word s/64.
 */
#ifndef GSS_H
#define GSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gss_status;

#define GSS_OK 0
#define GSS_ERR_INVALID_ARG (-1)     /* null pointer, empty clause, bad value, bad range, bad flag */
#define GSS_ERR_BAD_LITERAL (-2)     /* literal 0 or |literal| > num_vars */
#define GSS_ERR_UNKNOWN_ID (-3)      /* clause id never issued, already removed, or repeated */
#define GSS_ERR_CAPACITY (-4)        /* slot range, id space or HBM budget exhausted */
#define GSS_ERR_REPORT_OVERFLOW (-5) /* more hits than report capacity; count is still exact */
#define GSS_ERR_DEVICE (-6)          /* a HIP runtime call failed */
#define GSS_ERR_STATE (-7)           /* call not valid now (e.g. fetch before any test) */
#define GSS_NOT_READY 1              /* gss_poll: the test is still running (not an error) */

typedef struct gss_ctx gss_ctx;

/* One hit record: clause `clause_id` is falsified by slot 64*word + b for every
 * set bit b of `mask` (Section 4.3 reports a clause to the owner of a group with
 * the mask of hits inside the group; here a group is one 64-slot word).
 * 16 bytes, naturally aligned. */
typedef struct gss_report {
    uint32_t clause_id;
    uint32_t word;
    uint64_t mask;
} gss_report;

/* Device allocator hooks: a caller that manages device memory (for instance a
 * framework's caching allocator) can route every device allocation of the
 * context through them.  Both NULL: the library uses hipMalloc/hipFree.
 * dev_alloc returns NULL on failure. */
typedef void *(*gss_dev_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*gss_dev_free_fn)(void *ptr, void *stream, void *user);

typedef struct gss_config {
    uint32_t num_vars;          /* variables 1..num_vars (>= 1) */
    uint32_t max_slots;         /* assignment capacity: multiple of 64, 64..262144 (W = max_slots/64 words) */
    uint64_t hbm_budget_bytes;  /* cap on the context's device memory; 0 = no cap */
    uint64_t report_capacity;   /* initial report buffer entries, split evenly over the test kernel's
                                   wavefronts (at least 16 each); grown by gss_test unless GSS_TEST_NO_REGROW */
    void *stream;               /* borrowed hipStream_t; NULL = the context creates its own */
    gss_dev_alloc_fn dev_alloc; /* optional, see above */
    gss_dev_free_fn dev_free;
    void *alloc_user;
    uint32_t hot_vars;          /* LDS staging of the rows of the hot_vars most frequent variables (0 = off);
                                   see gss_rank_vars */
    uint32_t timing_interval;   /* the test kernel is timed with HIP events on every timing_interval-th
                                   launch (0 or 1: every launch); the events cost the stream a few
                                   microseconds per launch.  See gss_stats.timed_launches */
} gss_config;

/* Creates a context on the current HIP device.  Planes start all-Undef and no slot
 * is active.  *out receives the context (NULL on error; then use the return code). */
gss_status gss_create(const gss_config *cfg, gss_ctx **out);

/* Releases every device and host resource of the context.  NULL is accepted. */
void gss_destroy(gss_ctx *ctx);

/* Message describing the last error of this context ("" if none).  With ctx NULL,
 * the last error of a failed gss_create on this thread. */
const char *gss_last_error(const gss_ctx *ctx);

/* Adds n clauses (Section 3.6: every learned clause is exported to the GPU).
 * Clause i is lits[offsets[i] .. offsets[i+1]), host memory, offsets has n+1
 * entries and is non-decreasing.  Each clause needs at least one literal
 * (an empty clause is GSS_ERR_INVALID_ARG) and at most 65536.  Repeated literals
 * and tautologies are accepted and kept as given (literal order is not kept).
 * out_ids[i] (host, n entries) receives the clause's id: ids are issued
 * sequentially from 0 and never reused within a context.
 * Errors: INVALID_ARG, BAD_LITERAL, CAPACITY (id space or HBM budget), DEVICE. */
gss_status gss_add_clauses(gss_ctx *ctx, const int32_t *lits, const uint64_t *offsets, uint32_t n,
                           uint32_t *out_ids);

/* Removes n clauses by id (Section 3.7: the GPU deletes clauses as well).  Every
 * id must be live and appear once, else GSS_ERR_UNKNOWN_ID and nothing is
 * removed.  Storage is reclaimed by compaction when a length class holds more
 * than a quarter dead slots. */
gss_status gss_remove_clauses(gss_ctx *ctx, const uint32_t *ids, uint32_t n);

/* Number of live clauses, the next id to be issued, and the context's device bytes. */
gss_status gss_store_info(const gss_ctx *ctx, uint64_t *live_clauses, uint64_t *next_id, uint64_t *device_bytes);

/* Sets assignments into slots first_slot .. first_slot+n_slots-1 and marks them
 * active (Section 3.6: the parent assignment of a conflict is sent to the GPU).
 * values: slot-major int8 [n_slots][num_vars] (entry [s][v-1] is the value of
 * variable v in slot first_slot+s), host or device memory.  Values outside
 * {-1, 0, +1}: INVALID_ARG.  Range beyond max_slots: CAPACITY. */
gss_status gss_set_assignments(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots, const int8_t *values);

/* Delta update: new values of n_vars variables in slots first_slot ..
 * first_slot+n_slots-1; other variables and slots are unchanged.  vars: host
 * array of distinct variable numbers (1..num_vars).  values: var-major int8
 * [n_vars][n_slots], host or device.  The slots must already be active. */
gss_status gss_set_var_values(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots, uint32_t n_vars,
                              const uint32_t *vars, const int8_t *values);

/* The same delta with nothing waited for, so that a loop of deltas and tests
 * keeps the device busy.  values must be device memory, read by kernels queued on
 * the context's stream; it must stay unchanged until the first test begun after
 * this call has completed (the return of that gss_test, of the gss_test_wait of
 * that gss_test_async, or of a gss_batch_test that includes the context).  vars,
 * a host array, is copied before return.  The
 * slot range and the variable range are checked at once (nothing is queued on
 * error); the values and repeated variables are checked on the device.  An update
 * that fails that check applies nothing, nor do the asynchronous updates queued
 * after it, and the completion of that first test reports INVALID_ARG (the test
 * ran on the state without those updates; its records can be fetched). */
gss_status gss_set_var_values_async(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots, uint32_t n_vars,
                                    const uint32_t *vars, const int8_t *values);

/* Packed delta for one 64-slot word (a solver thread that keeps its group of 64
 * assignments as bit words sends only the changed variables): for each listed
 * variable vars[i] (distinct, 1..num_vars), bit b of f_words[i] says slot
 * 64*word+b has the variable F, bit b of t_words[i] that it has it T (both 0 =
 * U; both 1 is INVALID_ARG).  Host arrays.  Other variables and words are
 * unchanged; activity is not changed. */
gss_status gss_update_words(gss_ctx *ctx, uint32_t word, uint32_t n_vars, const uint32_t *vars,
                            const uint64_t *f_words, const uint64_t *t_words);
/* The same call under the name of a delta of variable rows: fp_words are the F
 * words (a positive literal is false), fn_words the T words (a negative literal
 * is false). */
gss_status gss_update_vars(gss_ctx *ctx, uint32_t word, uint32_t n_vars, const uint32_t *vars,
                           const uint64_t *fp_words, const uint64_t *fn_words);

/* Replaces the set of active slots (W words, host): the slots a test reports on.
 * Plane values of inactive slots are kept, so a slot group can be switched off
 * between runs and on again after further deltas. */
gss_status gss_set_active(gss_ctx *ctx, const uint64_t *active);

/* Makes slots first_slot .. first_slot+n_slots-1 inactive and all-Undef.  Tests
 * report nothing for inactive slots (Section 3.5 tests up to a fixed number of
 * assignments per run; a freed slot can take the next assignment). */
gss_status gss_clear_slots(gss_ctx *ctx, uint32_t first_slot, uint32_t n_slots);

/* Flags of gss_test. */
#define GSS_TEST_FALSIFIED 0u         /* default: every literal F */
#define GSS_TEST_TRIGGER 1u           /* Definition 1: no literal T and at most one not F */
#define GSS_TEST_NO_EARLY_EXIT 2u     /* read every literal (no wavefront early exit) */
#define GSS_TEST_SORTED 4u            /* gss_fetch_reports returns records ordered by (clause_id, word) */
#define GSS_TEST_DENSE 8u             /* write one mask row per clause id (see gss_fetch_masks); no reports */
#define GSS_TEST_NO_REGROW 16u        /* on overflow return GSS_ERR_REPORT_OVERFLOW instead of growing */
#define GSS_TEST_NO_HOT 32u           /* do not stage hot-variable rows in LDS */
/* Aggregate pre-test (Section 4): the 64 assignments of a word form a group, and
 * the context keeps, per literal, one bit per word saying whether the literal is
 * F in some slot of it (canBeFalse of the group's aggregate) and, per variable,
 * whether it is U in some active slot (canBeUndef).  A clause can only be
 * falsified in a word where all its literals can be F, and only trigger where the
 * aggregate recurrence of Section 4.3 says so (Theorem 1), so a lane reads a
 * literal's plane words only while the aggregate bits of its words allow it.  The
 * result is the same as without the flag; it is faster when the assignments of a
 * word are similar (as successive assignments of one solver thread are). */
#define GSS_TEST_AGGREGATE 256u
/* Counts what the test kernel did (gss_get_stats, last_* fields below): the
 * plane-row gathers its lanes issued and the (clause, word) pairs the aggregate
 * pre-test settled.  Costs a few instructions per gather and a synchronisation
 * when the test completes. */
#define GSS_TEST_COUNT 512u

/* Tests every live clause against every active slot (Section 3.6: a GPU run tests
 * all clauses against all assignments not yet tested and reports every hit).
 * *out_n_reports receives the number of gss_report records (one per clause and
 * 64-slot word with at least one hit; 0 with GSS_TEST_DENSE).  Each wavefront of
 * the test kernel appends to its own segment of the report buffer; if one is too
 * small the buffer is grown within the HBM budget and the test repeated, unless
 * GSS_TEST_NO_REGROW: then GSS_ERR_REPORT_OVERFLOW is returned, *out_n_reports
 * holds the exact count, and only the records that fit are kept (which ones is
 * unspecified).  Records come in a deterministic order for a given store, slot
 * set and device; with GSS_TEST_SORTED, gss_fetch_reports orders them by clause
 * id, then word (a device radix sort of every kept record at fetch time, which
 * needs 64 bytes of device memory per record; cap takes the first records of
 * that order).  GSS_TEST_SORTED with GSS_TEST_DENSE: INVALID_ARG. */
gss_status gss_test(gss_ctx *ctx, uint32_t flags, uint64_t *out_n_reports);

/* The same test split in two: gss_test_async queues it and returns; the host may
 * prepare the next run meanwhile (calls that change the store or the planes are
 * queued behind the test on the context's stream).  gss_test_query sets *done
 * once the results are in; gss_test_wait waits, then behaves as the end of
 * gss_test, with one difference: when the report segments overflowed and a call
 * changed the store, the planes or the active set after gss_test_async, the
 * segments are grown but the test is not repeated (a rerun would see the new
 * state): GSS_ERR_REPORT_OVERFLOW, with the exact count in *out_n_reports.  Only
 * one test may be in flight; gss_fetch_reports before gss_test_wait is
 * GSS_ERR_STATE. */
gss_status gss_test_async(gss_ctx *ctx, uint32_t flags);
gss_status gss_test_query(gss_ctx *ctx, int *done);
gss_status gss_test_wait(gss_ctx *ctx, uint64_t *out_n_reports);
/* Non-blocking form of the two above: GSS_NOT_READY (a positive status, not an
 * error) while the test in flight runs; once it has completed, exactly
 * gss_test_wait (its status and *out_n_reports).  No test in flight:
 * GSS_ERR_STATE. */
gss_status gss_poll(gss_ctx *ctx, uint64_t *out_n_reports);

/* Copies the records of the last gss_test into out (host or device, room for cap
 * records) as one list.  *out_n receives the number copied: min(cap, records
 * kept).  GSS_ERR_STATE before the first test. */
gss_status gss_fetch_reports(gss_ctx *ctx, gss_report *out, uint64_t cap, uint64_t *out_n);

/* After a gss_test with GSS_TEST_DENSE: copies the mask rows of n clause ids into
 * out (host or device, uint64 [n][W], W = max_slots/64).  Removed ids give zero
 * rows; ids never issued are GSS_ERR_UNKNOWN_ID; ids issued after that test
 * (which has no row for them) are GSS_ERR_STATE.  Both are checked on the host
 * before anything is queued. */
gss_status gss_fetch_masks(gss_ctx *ctx, const uint32_t *ids, uint32_t n, uint64_t *out);

/* Hot variables (Section 7, Conclusion: keep some variables' values in shared
 * memory).  With hot_vars > 0 the test kernel stages the plane rows of hot_vars
 * variables in LDS.  The library picks them: it counts on the device how often
 * each variable occurs in the live clauses and renumbers its variables
 * internally so that the hot_vars most frequent ones own the staged rows.  The
 * renumbering is invisible at this interface (variables keep their numbers in
 * every call, ids and records are unchanged).  gss_test ranks by itself on its
 * first run with staging and whenever the stored literals have doubled since
 * the last ranking (not while a server owns the context); gss_rank_vars ranks
 * now.  *out_hot_lits and *out_lits (either may be NULL) receive the literal
 * occurrences on the staged variables and in the store at the last ranking.
 * No staging (hot_vars 0, or rows of more than 4096 slots): nothing is ranked
 * and both counts are 0.  GSS_ERR_STATE with a test in flight or a server. */
gss_status gss_rank_vars(gss_ctx *ctx, uint64_t *out_hot_lits, uint64_t *out_lits);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): gss_test followed by
 * gss_fetch_reports into device memory, with no hipMalloc, hipFree or
 * allocating library call.  The test kernel's report segments, their counts and
 * offsets live in a 64 MiB scratch array that the library holds once per GPU
 * (from its first context on that GPU until the process ends); the records are
 * then stitched into out (device memory, room for cap records; NULL when cap is
 * 0).  *out_n_reports receives the exact number of records.  flags:
 * GSS_TEST_TRIGGER, GSS_TEST_NO_EARLY_EXIT, GSS_TEST_NO_HOT, GSS_TEST_AGGREGATE
 * (GSS_TEST_NO_REGROW is accepted and changes nothing: nothing is ever grown);
 * other flags are INVALID_ARG.  GSS_TEST_TRIGGER | GSS_TEST_AGGREGATE is
 * GSS_ERR_STATE until one gss_test with those flags has allocated the
 * canBeUndef bits.  Errors:
 *  - CAPACITY: the launch has too many wavefronts for 16 records each in the
 *    scratch array (nothing is run);
 *  - REPORT_OVERFLOW: a wavefront found more records than its share of the
 *    scratch array (the array holds about 4 M records spread evenly over the
 *    wavefronts), or more than cap; out holds min(cap, kept) records and
 *    *out_n_reports the exact count.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (from contexts on different streams or
 * threads) race and must be serialised by the caller.  The call synchronises
 * the context's stream.  Afterwards gss_fetch_reports is GSS_ERR_STATE until the
 * next gss_test (the records went to out only). */
gss_status gss_test_noalloc(gss_ctx *ctx, uint32_t flags, gss_report *out, uint64_t cap, uint64_t *out_n_reports);

/* Counters and timings of the context. */
typedef struct gss_stats {
    uint64_t tests_run;         /* gss_test calls that launched kernels */
    uint64_t last_pairs;        /* live clauses x active slots of the last test */
    uint64_t last_reports;      /* records of the last test */
    uint64_t last_literals;     /* literals stored for the live clauses (sum of lengths) */
    uint64_t live_clauses;
    uint64_t active_slots;
    uint64_t device_bytes;
    uint64_t compactions;
    uint64_t regrows;           /* report-buffer regrowths */
    uint64_t kernel_launches;   /* test kernel launches (reruns included) */
    double last_kernel_ms;      /* duration of the last timed test kernel, from HIP events on the context stream */
    double total_kernel_ms;     /* sum over the timed test kernel launches since the last reset */
    uint64_t timed_launches;    /* launches summed in total_kernel_ms (every gss_config.timing_interval-th) */
    /* the last test, when it ran with GSS_TEST_COUNT (else 0): */
    uint64_t last_gathers;      /* plane-row reads of the kernel's lanes: a lane reads its (up to 4) words of the
                                   row of each literal it tests (with GSS_TEST_AGGREGATE, of each literal of a
                                   group of four, padding past the clause's end included); trigger mode reads the
                                   opposite literal's row beside it, counted once */
    uint64_t last_gather_bytes; /* bytes those reads asked for */
    uint64_t last_agg_settled;  /* (clause, word) pairs the aggregate pre-test settled before the plane words
                                   did: no further gathers for them (GSS_TEST_AGGREGATE) */
} gss_stats;

gss_status gss_get_stats(const gss_ctx *ctx, gss_stats *out);
gss_status gss_reset_stats(gss_ctx *ctx);

/* hipStream_t the context issues work on (borrowed or owned). */
gss_status gss_get_stream(const gss_ctx *ctx, void **stream);

/* ---- Batched test: several independent stores in one persistent launch ----
 *
 * A batch groups n contexts (1..64) created on the same device with the same
 * stream (pass one hipStream_t in every gss_config).  gss_batch_test tests every
 * store against its own active slots in ONE persistent kernel launch; afterwards
 * each context holds its records exactly as after its own gss_test (fetch them
 * with gss_fetch_reports).  The contexts stay usable on their own; a batch only
 * reads them and must be destroyed before them.  This has no counterpart in the
 * paper, whose GPU serves one clause database; it serves several at once. */
typedef struct gss_batch gss_batch;

#define GSS_ORDER_STORE 0u         /* all tiles of store 0, then store 1, ... */
#define GSS_ORDER_INTERLEAVE 1u    /* chunks of chunk_tiles tiles, stores in turn */
#define GSS_ORDER_LONGEST_FIRST 2u /* length classes by decreasing stride across stores, stores in turn */

/* The order in which the stores' tiles are dealt to the wavefronts, and the
 * number of persistent workgroups per compute unit (0 = as many as fit).  Any
 * schedule gives the same results; the autotuner picks the fastest. */
typedef struct gss_schedule {
    uint32_t order;
    uint32_t chunk_tiles;   /* 0 = 64 */
    uint32_t blocks_per_cu; /* 0..8 */
    uint32_t reserved;
} gss_schedule;

/* Flag of gss_batch_test: capture the launch sequence (table uploads, kernels,
 * the copy of the counts) in a hipGraph on first use and replay it while no store
 * changed (clauses added or removed, report segments grown), and the schedule
 * and flags are the same; otherwise capture again. */
#define GSS_TEST_GRAPH 64u

gss_status gss_batch_create(gss_ctx *const *ctxs, uint32_t n, gss_batch **out);
void gss_batch_destroy(gss_batch *batch);
const char *gss_batch_last_error(const gss_batch *batch);
gss_status gss_batch_set_schedule(gss_batch *batch, const gss_schedule *schedule);

/* Tests every store of the batch.  flags: GSS_TEST_TRIGGER, GSS_TEST_NO_EARLY_EXIT,
 * GSS_TEST_NO_REGROW, GSS_TEST_GRAPH, GSS_TEST_AGGREGATE (each store's aggregate
 * bits are brought up to date before the launch; no LDS staging in a batch, whose
 * wavefronts move between stores).  A member with a gss_test_async in flight:
 * GSS_ERR_STATE (nothing queued).  out_n_reports (n entries, may be NULL)
 * receives each store's record count.  A store whose report segments overflow is
 * grown and the whole batch repeated (unless GSS_TEST_NO_REGROW: then
 * GSS_ERR_REPORT_OVERFLOW, with exact counts). */
gss_status gss_batch_test(gss_batch *batch, uint32_t flags, uint64_t *out_n_reports);

/* The same test queued without waiting, so that the next round's updates
 * (gss_set_var_values_async on the members) can be queued while it runs: the
 * host work of those calls then overlaps the batched kernel.  Until
 * gss_batch_wait, the members count as having a test in flight (gss_test on them,
 * gss_fetch_reports and the like: GSS_ERR_STATE; gss_test_wait on a member: STATE,
 * naming gss_batch_wait).  gss_batch_wait returns what gss_batch_test would; a
 * store that overflowed is grown, and the batch repeated only when no member has
 * changed since the launch (else GSS_ERR_REPORT_OVERFLOW with exact counts, and
 * the next test fits). */
gss_status gss_batch_test_async(gss_batch *batch, uint32_t flags);
gss_status gss_batch_wait(gss_batch *batch, uint64_t *out_n_reports);

/* Duration of the last batched launch sequence in ms (HIP events around it),
 * launches and graph captures so far, and the tiles of the last plan. */
gss_status gss_batch_info(const gss_batch *batch, double *last_ms, uint64_t *launches, uint64_t *captures,
                          uint64_t *tiles);

/* ---- Learned clause priority ----
 *
 * The paper measures (Section 3.2) that a clause used recently is likely to be
 * used again soon, and deletes clauses on the GPU by MiniSat-style activity
 * (Section 3.7).  This extension learns a priority instead: a 12 -> 64 -> 64 -> 1
 * perceptron (ReLU, sigmoid output, fp32) scores each clause from its length,
 * LBD, age in runs, source thread and the hit counts (slots where it was
 * falsified) of the last 8 runs that tested it; clauses scoring below a
 * threshold are tested only in runs where (run + id) % 4 == 0.  The plain test
 * stays available and judges what the schedule misses.
 *
 * Network parameters, 5057 floats: W1[12][64] (input major), b1[64], W2[64][64],
 * b2[64], w3[64], b3.  Features, in order: log1p(length), log1p(LBD),
 * log1p(age), source / max(1, n_sources - 1), log1p(hits of the last 8 tested
 * runs), most recent first. */
#define GSS_MLP_FEATURES 12
#define GSS_MLP_PARAMS 5057

/* Flag of gss_test: follow the priority schedule of the current run (needs
 * gss_priority_score first). */
#define GSS_TEST_SCHEDULED 128u

typedef struct gss_adam_config {
    float lr, beta1, beta2, eps; /* Adam (Kingma and Ba): step size, moment decays, epsilon */
    uint32_t batch;              /* samples per step (the last step may be smaller) */
    uint32_t reserved[3];
} gss_adam_config;

/* The network's kernels on their own (for checking them and for other callers).
 * params: host [5057].  x: [n][12] fp32, y: [n] labels in {0, 1}, host or device.
 * out_prob: [n] probabilities, out_grad: [5057] gradient of the mean binary
 * cross-entropy, host or device; out_loss: host scalar. */
gss_status gss_mlp_forward(gss_ctx *ctx, const float *params, const float *x, uint32_t n, float *out_prob);
gss_status gss_mlp_loss_grad(gss_ctx *ctx, const float *params, const float *x, const float *y, uint32_t n,
                             float *out_loss, float *out_grad);
/* Adam from fresh moments over the minibatches order[0..batch), order[batch..2
 * batch), ... (order: host array of row indices < n).  params (host) is updated in
 * place; out_losses (host, may be NULL) receives each step's loss. */
gss_status gss_mlp_train(gss_ctx *ctx, float *params, const float *x, const float *y, uint32_t n,
                         const uint32_t *order, uint64_t n_order, const gss_adam_config *cfg, float *out_losses);

typedef struct gss_priority_config {
    uint32_t n_sources;       /* solver threads that export clauses (>= 1) */
    uint32_t sample_period;   /* a tested clause becomes a training sample of a run when a hash of
                                 (seed, id, run) is 0 modulo the period; 0 = no samples */
    uint64_t sample_capacity; /* rows of the sample buffer */
    uint64_t seed;            /* sampling and weight initialisation */
    double activity_decay;    /* Section 3.7 activity: the bump grows by 1/decay per run; 0 = 0.999 */
    uint64_t reserved[3];
} gss_priority_config;

/* Enables the priority on a context: per-clause state for every issued id (LBD
 * defaults to the length, source to 0), a seeded He-uniform network. */
gss_status gss_priority_enable(gss_ctx *ctx, const gss_priority_config *cfg);
/* LBD (>= 0) and source thread (< n_sources) of n live clauses (host arrays). */
gss_status gss_priority_set_clause_info(gss_ctx *ctx, const uint32_t *ids, uint32_t n, const float *lbd,
                                        const uint32_t *source);
/* After a test (plain or scheduled, not dense, no records lost): counts each
 * clause's hits from the test's records, takes the run's samples (features
 * before the run, label = hit in it), shifts the hit history of every clause the
 * test ran, and advances the run counter.  Once per test. */
gss_status gss_priority_observe(gss_ctx *ctx);
/* Trains the network on the samples taken so far: epochs of seeded shuffles,
 * Adam from fresh moments.  *out_loss (may be NULL): the last step's loss. */
gss_status gss_priority_train(gss_ctx *ctx, uint32_t epochs, const gss_adam_config *cfg, uint64_t seed,
                              float *out_loss);
gss_status gss_priority_clear_samples(gss_ctx *ctx);
/* Changes the sample period (0 stops sampling, for instance once the network is
 * trained; a nonzero period needs the sample capacity given at enable). */
gss_status gss_priority_set_sampling(gss_ctx *ctx, uint32_t period);
/* Scores every live clause; scores below threshold are low priority.
 * *out_n_low (may be NULL): how many. */
gss_status gss_priority_score(gss_ctx *ctx, float threshold, uint64_t *out_n_low);
/* Rescores only the clauses that may have changed side of the threshold since
 * they were last scored: new clauses, new LBD or source, a low clause that hit
 * in a run, a high clause that did not.  The others keep their scores until the
 * next gss_priority_score (their age still grows).  Uses the threshold of the last
 * gss_priority_score, which must have run since the last gss_priority_mark.
 * *out_n_low (may be NULL): low clauses now. */
gss_status gss_priority_update(gss_ctx *ctx, uint64_t *out_n_low);
/* Sets the low flags directly, one byte per issued id (host array of next_id
 * entries; nonzero = low), in place of a scoring: schedules of other policies. */
gss_status gss_priority_mark(gss_ctx *ctx, const uint8_t *low, uint64_t n);
/* Copies the network's parameters out (get) and/or in (set); host [5057] each, either may be NULL. */
gss_status gss_priority_params(gss_ctx *ctx, float *get, const float *set);
/* Features ([n][12]), last scores and low flags of n issued ids (host arrays). */
gss_status gss_priority_fetch(gss_ctx *ctx, const uint32_t *ids, uint32_t n, float *out_features, float *out_scores,
                              uint8_t *out_low);
/* Activity-based deletion (Section 3.7, the GPU deletes clauses like MiniSat
 * on the CPU): every observed run adds the current bump to the activity of each
 * clause with a hit, then the bump grows by 1/activity_decay (activities are
 * rescaled together when it grows large).  gss_priority_reduce removes live
 * clauses, least active first (the older among equals), until `keep` remain;
 * *out_removed (may be NULL) receives how many.  gss_priority_activity copies the
 * activities of n issued ids (host arrays). */
gss_status gss_priority_reduce(gss_ctx *ctx, uint64_t keep, uint64_t *out_removed);
gss_status gss_priority_activity(gss_ctx *ctx, const uint32_t *ids, uint32_t n, float *out_activity);
/* Copies up to cap samples ([cap][12] features, [cap] labels; host, either may be NULL). */
gss_status gss_priority_samples(gss_ctx *ctx, float *out_x, float *out_y, uint64_t cap, uint64_t *out_n);
/* Run counter, samples held, low clauses of the last scoring. */
gss_status gss_priority_info(const gss_ctx *ctx, uint32_t *out_run, uint64_t *out_samples, uint64_t *out_n_low);

/* ---- Served test: a manager thread fed by solver threads ----
 *
 * Section 5 has one CPU thread besides the solver threads manage the GPU; per
 * Section 3.6 the solver threads send it their assignments and export their
 * learned clauses, and learn which clauses fire on their assignments.  A server
 * owns a context and runs that manager in a native thread:
 *
 *  - producer p (0 <= p < n_producers <= W) owns the 64 slots of word p: each
 *    gss_server_send is one snapshot of its 64 assignments, given as a packed
 *    delta to its previous snapshot (as gss_update_words).  Deltas that arrive
 *    while a run is on the GPU are merged and uploaded on a copy stream while
 *    that run still executes; the next run tests every word with a new snapshot
 *    (continuous batching).  A snapshot superseded before a run took it is
 *    dropped, as the paper drops assignments the GPU cannot take.
 *  - gss_server_insert queues learned clauses; they are admitted between runs
 *    within the context's HBM budget: while it is full they are held back, or,
 *    with evict_keep, the least active clauses make room (Section 3.7).
 *  - a fraction of the live clauses is removed each second at random (the
 *    simulated clause-database reduction of the solvers).
 *  - the records of each run are routed by word to their producer, who collects
 *    them with gss_server_poll.  Notify latency: from the send of the snapshot a
 *    run tested until its records are in the producer's queue.
 *
 * While a server runs, its context must not be used directly.  send, insert and
 * poll are thread-safe. */
typedef struct gss_server gss_server;

typedef struct gss_server_config {
    uint32_t n_producers;     /* 1..W (max_slots / 64) */
    uint32_t test_flags;      /* flags of every run: GSS_TEST_TRIGGER, GSS_TEST_NO_EARLY_EXIT, GSS_TEST_NO_HOT,
                                 GSS_TEST_AGGREGATE */
    double delete_fraction;   /* fraction of the live clauses removed per second (0 = none) */
    uint64_t seed;            /* of the removals */
    const char *log_path;     /* NULL, or a text file receiving every change, run and record in the
                                 order the device applies them (for replay against a reference) */
    uint64_t max_queued_lits; /* inserts waiting for admission, in literals (0 = 1 << 26); beyond: refused */
    double evict_keep;        /* activity eviction (Section 3.7): when an insert does not fit the HBM budget,
                                 the least active live clauses are removed until this fraction of them is
                                 left, and the insert is retried (0 = off: inserts wait for removals).
                                 In [0, 1).  Enables the context's learned priority if it is not (its
                                 activities: every run bumps the clauses with a record) */
    uint64_t reserved[2];
} gss_server_config;

typedef struct gss_serve_result {
    uint64_t snapshots;       /* gss_server_send calls */
    uint64_t tested;          /* snapshots whose records reached their producer */
    uint64_t dropped;         /* snapshots superseded before a run took them */
    uint64_t runs;            /* test runs completed */
    uint64_t overflowed_runs; /* runs whose records overflowed (their words are tested again) */
    uint64_t inserted;        /* clauses admitted */
    uint64_t refused;         /* clauses refused (insert queue full) */
    uint64_t deleted;         /* clauses removed */
    uint64_t reports;         /* records routed to producers */
    uint64_t pairs;           /* clause x assignment tests: live clauses x active slots, summed over runs */
    uint64_t live_end;        /* live clauses at the end */
    uint64_t device_bytes_end;
    uint64_t delta_bytes;     /* bytes of deltas uploaded */
    uint64_t evicted;         /* clauses removed by activity eviction */
    uint64_t evictions;       /* activity evictions (each removes down to evict_keep of the live clauses) */
    double wall_s;            /* from start to stop */
    double gpu_ms;            /* test kernel time, summed over runs */
    double mean_ms, p50_ms, p99_ms, max_ms; /* notify latency */
    /* manager thread time by phase, summed over the session (ms): taking and
     * uploading deltas, waiting for runs, fetching records, routing them,
     * inserts and removals, launching runs */
    double admit_ms, wait_ms, fetch_ms, route_ms, store_ms, launch_ms;
} gss_serve_result;

/* Starts the manager thread on ctx (no test may be in flight).  Allocates two
 * pinned host and device delta buffers of num_vars entries per producer. */
gss_status gss_server_start(gss_ctx *ctx, const gss_server_config *cfg, gss_server **out);

/* A snapshot of producer p: n_vars entries (vars 1..num_vars; f_words[i] and
 * t_words[i] disjoint, as gss_update_words; a variable listed twice takes its
 * last entry).  Host arrays, copied before returning. */
gss_status gss_server_send(gss_server *srv, uint32_t producer, uint32_t n_vars, const uint32_t *vars,
                           const uint64_t *f_words, const uint64_t *t_words);

/* Queues n learned clauses of producer p (layout of gss_add_clauses; copied).
 * GSS_ERR_CAPACITY when the admission queue is full (nothing queued). */
gss_status gss_server_insert(gss_server *srv, uint32_t producer, const int32_t *lits, const uint64_t *offsets,
                             uint32_t n);

/* Moves up to cap of producer p's pending records into out (host) and sets
 * *out_n; out NULL discards them all (*out_n = the number discarded).  *out_run
 * (may be NULL) receives the last run whose records were routed to p (or
 * UINT64_MAX if none).  The records wait in the pinned buffers they were
 * fetched into and are copied here, on the caller's thread; a producer that
 * falls several runs behind is given copies, so that those buffers can be
 * reused. */
gss_status gss_server_poll(gss_server *srv, uint32_t producer, gss_report *out, uint64_t cap, uint64_t *out_n,
                           uint64_t *out_run);

/* Stops the manager (the run in flight is completed and routed), fills *out (may
 * be NULL) and releases the server; the context is usable again.  Errors met by
 * the manager thread are returned here. */
gss_status gss_server_stop(gss_server *srv, gss_serve_result *out);

/* Message of the server's last error ("" if none). */
const char *gss_server_last_error(const gss_server *srv);

/* ---- Served workload generator ----
 *
 * Runs a server on ctx for duration_s with n_threads simulated solver threads.
 * Thread i owns word i.  It sends a full snapshot at start, then a Poisson stream
 * of snapshots at snapshot_rate per second, each redrawing redraw_fraction of
 * the variables (in runs of 64 consecutive variables); every variable of a
 * snapshot takes a subset of {T, F, U} with the frequencies of Table 1, then
 * each of its 64 slots a value drawn uniformly from that subset.  It inserts
 * insert_rate clauses per second (lengths: half in 2..10, 40% in 11..50, 10% in
 * 51..300; distinct variables, uniform signs) and discards its records.  Seeded:
 * the drawn values are reproducible, their timing is not. */
typedef struct gss_sim_config {
    uint32_t n_threads;
    uint32_t test_flags;
    double duration_s;
    double snapshot_rate;
    double redraw_fraction;
    double insert_rate;
    double delete_fraction;
    uint64_t seed;
    const char *log_path;
    double evict_keep;        /* as gss_server_config.evict_keep */
    uint64_t reserved[3];
} gss_sim_config;

gss_status gss_serve_simulate(gss_ctx *ctx, const gss_sim_config *cfg, gss_serve_result *out);

#ifdef __cplusplus
}
#endif

#endif /* GSS_H */
