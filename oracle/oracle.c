/*
 * oracle.c -- the reference computation of the clause test, as plain CPU loops.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * do.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (GpuShareSat, Section 3.1 and Section 3.3):
 *   - truth values T, F, U; the negation of U is U;
 *   - the value of a literal under an assignment is the value of its variable,
 *     negated when the literal is negative;
 *   - falsified: a clause is falsified by an assignment when every one of its
 *     literals has the value F (a solver holding that assignment would be in
 *     conflict on it);
 *   - trigger (Definition 1): no literal has the value T and at least s-1 of the
 *     s literals have the value F (the clause is in conflict or would imply its
 *     one Undef literal).  Literals are counted as a multiset, so a repeated
 *     literal counts once per occurrence.
 *
 * The loops run clause -> assignment -> literal and stop scanning a clause's
 * literals as soon as the answer for that assignment is known.  Output is one bit
 * per (clause, assignment slot), packed 64 slots per uint64 word: bit b of word w
 * is slot 64*w + b.  Bits of slots that are not active are 0.
 *
 * Encodings at this interface:
 *   - literals: DIMACS signed int32, variable v in 1..n_vars, -v is its negation;
 *   - truth values: int8, +1 = T, -1 = F, 0 = U;
 *   - clause c occupies lits[offsets[c] .. offsets[c+1]).
 *
 * Every entry point returns 0 on success and a negative number on bad input
 * (a literal 0 or beyond n_vars: -1; a bad size or offset: -2).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TV_T ((int8_t)1)
#define TV_F ((int8_t)-1)
#define TV_U ((int8_t)0)

/* The value of a literal given the value of its variable (Section 3.1). */
static int8_t literal_value(int32_t lit, int8_t var_value)
{
    if (lit > 0)
        return var_value;
    /* negation: T <-> F, U stays U */
    if (var_value == TV_T)
        return TV_F;
    if (var_value == TV_F)
        return TV_T;
    return TV_U;
}

/*
 * Transposes the slot-major values [n_slots][n_vars] into var-major
 * [n_vars][n_slots], so that the values one clause reads for consecutive slots sit
 * next to each other.  This is a plain copy, no arithmetic.
 */
int oracle_transpose(int64_t n_slots, int64_t n_vars, const int8_t *slot_major, int8_t *var_major)
{
    if (n_slots < 0 || n_vars < 0)
        return -2;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n_vars; ++v)
        for (int64_t a = 0; a < n_slots; ++a)
            var_major[v * n_slots + a] = slot_major[a * n_vars + v];
    return 0;
}

/* Checks every literal against the variable range. */
static int check_clauses(int64_t n_clauses, const int64_t *offsets, const int32_t *lits, int64_t n_vars)
{
    if (n_clauses < 0 || offsets[0] < 0)
        return -2;
    for (int64_t c = 0; c < n_clauses; ++c) {
        if (offsets[c + 1] < offsets[c])
            return -2;
        for (int64_t i = offsets[c]; i < offsets[c + 1]; ++i) {
            int64_t v = lits[i] > 0 ? (int64_t)lits[i] : -(int64_t)lits[i];
            if (v == 0 || v > n_vars)
                return -1;
        }
    }
    return 0;
}

/*
 * Falsified: bit (c, a) is set iff every literal of clause c has the value F under
 * assignment a.  values_vm is var-major [n_vars][n_slots]; active is one byte per
 * slot (nonzero = the slot holds an assignment) or NULL for all slots active.
 * out has n_clauses * ceil(n_slots/64) words.
 */
int oracle_falsified(int64_t n_clauses, const int64_t *offsets, const int32_t *lits,
                     int64_t n_vars, int64_t n_slots, const int8_t *values_vm,
                     const uint8_t *active, uint64_t *out)
{
    int rc = check_clauses(n_clauses, offsets, lits, n_vars);
    if (rc != 0 || n_slots < 0)
        return rc != 0 ? rc : -2;
    const int64_t n_words = (n_slots + 63) / 64;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < n_clauses; ++c) {
        uint64_t *row = out + c * n_words;
        memset(row, 0, (size_t)n_words * sizeof(uint64_t));
        for (int64_t a = 0; a < n_slots; ++a) {
            if (active && !active[a])
                continue;
            int all_false = 1;
            for (int64_t i = offsets[c]; i < offsets[c + 1]; ++i) {
                int32_t lit = lits[i];
                int64_t v = lit > 0 ? (int64_t)lit : -(int64_t)lit;
                if (literal_value(lit, values_vm[(v - 1) * n_slots + a]) != TV_F) {
                    all_false = 0;
                    break;
                }
            }
            if (all_false)
                row[a / 64] |= (uint64_t)1 << (a % 64);
        }
    }
    return 0;
}

/*
 * Trigger (Definition 1): bit (c, a) is set iff no literal of clause c is T under
 * assignment a and at least s-1 of its s literals are F.  Same layouts as
 * oracle_falsified.
 */
int oracle_trigger(int64_t n_clauses, const int64_t *offsets, const int32_t *lits,
                   int64_t n_vars, int64_t n_slots, const int8_t *values_vm,
                   const uint8_t *active, uint64_t *out)
{
    int rc = check_clauses(n_clauses, offsets, lits, n_vars);
    if (rc != 0 || n_slots < 0)
        return rc != 0 ? rc : -2;
    const int64_t n_words = (n_slots + 63) / 64;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < n_clauses; ++c) {
        uint64_t *row = out + c * n_words;
        memset(row, 0, (size_t)n_words * sizeof(uint64_t));
        const int64_t s = offsets[c + 1] - offsets[c];
        for (int64_t a = 0; a < n_slots; ++a) {
            if (active && !active[a])
                continue;
            int64_t n_true = 0, n_false = 0, seen = 0;
            for (int64_t i = offsets[c]; i < offsets[c + 1]; ++i) {
                int32_t lit = lits[i];
                int64_t v = lit > 0 ? (int64_t)lit : -(int64_t)lit;
                int8_t val = literal_value(lit, values_vm[(v - 1) * n_slots + a]);
                seen++;
                if (val == TV_T)
                    n_true++;
                if (val == TV_F)
                    n_false++;
                /* stop once Definition 1 can no longer hold: a T literal, or two
                 * literals already seen that are not F */
                if (n_true > 0 || seen - n_false > 1)
                    break;
            }
            if (n_true == 0 && n_false >= s - 1)
                row[a / 64] |= (uint64_t)1 << (a % 64);
        }
    }
    return 0;
}

/* Number of threads the loops above use (OpenMP), for reporting. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of threads of the loops above (for timing on fewer cores);
 * returns the number now in use. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
