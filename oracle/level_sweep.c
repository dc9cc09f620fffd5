/*
 * Level-by-level evaluation oracle for leveled-DAG diagram summation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference against
 * which the GPU library is checked.  It shares no code, header, table or
 * helper with the library, and nothing on the product path may call it: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark.
 *
 * What it computes (paper Sec. II.B and the caption of Fig. combinedgraphflat):
 * the root node holds 1; every edge multiplies the value held at its source
 * node by its edge factor and adds the product into its destination node; the
 * final node then holds the sum over all root-to-final paths of the product of
 * the path's edge factors.  Edges only join consecutive levels, so the levels
 * are evaluated one after another, each level fully before the next (Sec. II.C,
 * "Windowing": a parent node is complete before its out-edges are applied).
 *
 * Edge factors, two kinds:
 *   rational (the synthetic stand-in for a Green's function of the sample's
 *   coordinates):   w_e(x) = a_e / (1 + b_e * |x - k_e|^2),  x, k_e in R^3;
 *   lookup (the paper's own form, Sec. II.B and Sec. III: a Green's function
 *   G_ab between two of the sample's vertices, times a fermion-loop sign or
 *   other constant):  w_e(s) = c_e * T_s[slot_e], T_s the sample's table.
 *
 * Arithmetic: IEEE binary64, no FMA contraction (build with -ffp-contract=off),
 * edges summed in the order the caller supplies them.  Samples are independent;
 * OpenMP hands contiguous blocks of samples to threads, and every thread runs
 * the whole sweep for its block, so each sample's arithmetic is the same for
 * any thread count.
 *
 * mode 0: the value V(x) = sum_paths prod w_e(x)
 * mode 1: A(x) = sum_paths prod |w_e(x)|   (1-norm of the path terms)
 * mode 2: Q(x) = sum_paths prod w_e(x)^2   (squared 2-norm of the path terms)
 *
 * The *_nodes entry points also return the value every node holds after the
 * sweep (the sum over root-to-node paths), for every sample.
 *
 * Self-check build (-DORACLE_LONG_DOUBLE): the same sweep with every factor,
 * product and sum carried in long double (x87 80-bit, 64-bit significand),
 * rounded to binary64 only when the final or node values are written out.  It
 * bounds the binary64 oracle's own rounding error (Sec. III, numerical
 * stability: how far a lower precision drifts from a higher one), which is
 * what the error metric of the parity tests is calibrated against.
 *
 * Parity pins: brute-force exact path sums, closed forms, transpose invariance
 * and exact power-of-two scaling (see the oracle tests).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORACLE_SRC_HASH
#define ORACLE_SRC_HASH "unknown"
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2

#define SAMPLE_BLOCK 8

/* Arithmetic type of the sweep (binary64 unless the self-check build). */
#ifdef ORACLE_LONG_DOUBLE
typedef long double real;
#define REAL_ABS fabsl
#else
typedef double real;
#define REAL_ABS fabs
#endif

const char *oracle_src_hash(void) { return ORACLE_SRC_HASH; }

/* Structural and parameter validation, written independently of the library. */
int oracle_check(int32_t L, const int64_t *widths, const int64_t *epl,
                 const int32_t *src, const int32_t *dst, const double *a,
                 const double *b, const double *k)
{
    if (L < 1 || widths[0] != 1 || widths[L] != 1)
        return ORACLE_EINVAL;
    int64_t n_nodes = 0;
    for (int32_t l = 0; l <= L; ++l) {
        if (widths[l] < 1)
            return ORACLE_EINVAL;
        n_nodes += widths[l];
    }
    if (n_nodes > INT32_MAX)
        return ORACLE_EINVAL;
    int64_t first = 0;       /* first node id of level l-1 */
    int64_t e = 0;
    for (int32_t l = 1; l <= L; ++l) {
        int64_t lo_src = first, hi_src = first + widths[l - 1];
        int64_t lo_dst = hi_src, hi_dst = hi_src + widths[l];
        if (epl[l - 1] < 0)
            return ORACLE_EINVAL;
        for (int64_t i = 0; i < epl[l - 1]; ++i, ++e) {
            if (src[e] < lo_src || src[e] >= hi_src)
                return ORACLE_EINVAL;
            if (dst[e] < lo_dst || dst[e] >= hi_dst)
                return ORACLE_EINVAL;
            if (!isfinite(a[e]) || !isfinite(b[e]) || b[e] < 0.0)
                return ORACLE_EINVAL;
            if (!isfinite(k[3 * e]) || !isfinite(k[3 * e + 1]) || !isfinite(k[3 * e + 2]))
                return ORACLE_EINVAL;
        }
        first = hi_src;
    }
    return ORACLE_OK;
}

/* Validation of a lookup graph: the same structure rules, slots inside the
   table, finite constants. */
int oracle_check_lookup(int32_t L, const int64_t *widths, const int64_t *epl,
                        const int32_t *src, const int32_t *dst, const int32_t *slot,
                        const double *coef, int32_t n_slots)
{
    if (L < 1 || widths[0] != 1 || widths[L] != 1 || n_slots < 1)
        return ORACLE_EINVAL;
    int64_t n_nodes = 0;
    for (int32_t l = 0; l <= L; ++l) {
        if (widths[l] < 1)
            return ORACLE_EINVAL;
        n_nodes += widths[l];
    }
    if (n_nodes > INT32_MAX)
        return ORACLE_EINVAL;
    int64_t first = 0;
    int64_t e = 0;
    for (int32_t l = 1; l <= L; ++l) {
        int64_t lo_src = first, hi_src = first + widths[l - 1];
        int64_t lo_dst = hi_src, hi_dst = hi_src + widths[l];
        if (epl[l - 1] < 0)
            return ORACLE_EINVAL;
        for (int64_t i = 0; i < epl[l - 1]; ++i, ++e) {
            if (src[e] < lo_src || src[e] >= hi_src)
                return ORACLE_EINVAL;
            if (dst[e] < lo_dst || dst[e] >= hi_dst)
                return ORACLE_EINVAL;
            if (slot[e] < 0 || slot[e] >= n_slots || !isfinite(coef[e]))
                return ORACLE_EINVAL;
        }
        first = hi_src;
    }
    return ORACLE_OK;
}

/* The edge factor, literally as defined. */
static real edge_factor(real a, real b, const double *k, real x0, real x1, real x2)
{
    real d0 = x0 - (real)k[0];
    real d1 = x1 - (real)k[1];
    real d2 = x2 - (real)k[2];
    real r2 = d0 * d0 + d1 * d1 + d2 * d2;
    return a / ((real)1.0 + b * r2);
}

/*
 * The sweep for either kind.  kind 0: x is float64[3][S] (coordinates), the
 * factor rational; kind 1: x is float64[n_slots][S] (each sample's table
 * T_s[slot] = x[slot * S + s]), the factor c_e * T_s[slot_e].  out: float64[S].
 * nodes (nullable): float64[n_nodes][S], every node's value.
 */
static int sweep(int32_t kind, int32_t L, const int64_t *widths, const int64_t *epl,
                 const int32_t *src, const int32_t *dst, const double *a, const double *b,
                 const double *k, const int32_t *slot, const double *coef, const double *x,
                 int64_t S, int32_t mode, int32_t nthreads, double *out, double *nodes,
                 int32_t *threads_used)
{
    if (S < 0 || mode < 0 || mode > 2)
        return ORACLE_EINVAL;
    int64_t n_nodes = 0;
    for (int32_t l = 0; l <= L; ++l)
        n_nodes += widths[l];
    int64_t *level_first = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L + 2));
    int64_t *edge_first = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L + 1));
    if (!level_first || !edge_first) {
        free(level_first);
        free(edge_first);
        return ORACLE_ENOMEM;
    }
    level_first[0] = 0;
    for (int32_t l = 0; l <= L; ++l)
        level_first[l + 1] = level_first[l] + widths[l];
    edge_first[0] = 0;
    for (int32_t l = 0; l < L; ++l)
        edge_first[l + 1] = edge_first[l] + epl[l];
    const int64_t final_node = n_nodes - 1;
    const int64_t n_blocks = (S + SAMPLE_BLOCK - 1) / SAMPLE_BLOCK;
    int failed = 0;
    int used = 1;

#ifdef _OPENMP
    /* the thread count applies to this call only (a num_threads clause, not
       omp_set_num_threads, which would persist into later calls) */
    const int nt = nthreads > 0 ? (int)nthreads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
#endif
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
        /* value[node * SAMPLE_BLOCK + j] for every node of the graph,
           allocated when this thread receives its first block */
        real *value = NULL;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t blk = 0; blk < n_blocks; ++blk) {
            if (!value)
                value = (real *)malloc(sizeof(real) * (size_t)n_nodes * SAMPLE_BLOCK);
            if (!value) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                failed = 1;
                continue;
            }
            int64_t s0 = blk * SAMPLE_BLOCK;
            int64_t nb = S - s0 < SAMPLE_BLOCK ? S - s0 : SAMPLE_BLOCK;
            /* level 0: the root holds 1 */
            for (int64_t j = 0; j < nb; ++j)
                value[0 * SAMPLE_BLOCK + j] = 1.0;
            for (int32_t l = 1; l <= L; ++l) {
                /* nodes of level l start from zero */
                for (int64_t n = level_first[l]; n < level_first[l + 1]; ++n)
                    for (int64_t j = 0; j < nb; ++j)
                        value[n * SAMPLE_BLOCK + j] = 0.0;
                /* every edge of level l: dst += factor * src, in input order */
                for (int64_t e = edge_first[l - 1]; e < edge_first[l]; ++e) {
                    for (int64_t j = 0; j < nb; ++j) {
                        int64_t s = s0 + j;
                        real w;
                        if (kind == 0)
                            w = edge_factor(a[e], b[e], &k[3 * e], x[s], x[S + s], x[2 * S + s]);
                        else
                            w = (real)coef[e] * (real)x[(int64_t)slot[e] * S + s];
                        if (mode == 1)
                            w = REAL_ABS(w);
                        else if (mode == 2)
                            w = w * w;
                        value[(int64_t)dst[e] * SAMPLE_BLOCK + j] += w * value[(int64_t)src[e] * SAMPLE_BLOCK + j];
                    }
                }
            }
            for (int64_t j = 0; j < nb; ++j)
                out[s0 + j] = (double)value[final_node * SAMPLE_BLOCK + j];
            if (nodes)
                for (int64_t n = 0; n < n_nodes; ++n)
                    for (int64_t j = 0; j < nb; ++j)
                        nodes[n * S + s0 + j] = (double)value[n * SAMPLE_BLOCK + j];
        }
        free(value);
    }
    free(level_first);
    free(edge_first);
    if (threads_used)
        *threads_used = used;
    return failed ? ORACLE_ENOMEM : ORACLE_OK;
}

/*
 * Rational factors.  x: float64[3][S] (structure of arrays), out: float64[S].
 * nthreads <= 0 leaves the OpenMP default.  *threads_used (nullable) receives
 * the number of threads that ran.
 */
int oracle_sweep(int32_t L, const int64_t *widths, const int64_t *epl,
                 const int32_t *src, const int32_t *dst, const double *a,
                 const double *b, const double *k, const double *x, int64_t S,
                 int32_t mode, int32_t nthreads, double *out, int32_t *threads_used)
{
    int rc = oracle_check(L, widths, epl, src, dst, a, b, k);
    if (rc != ORACLE_OK)
        return rc;
    return sweep(0, L, widths, epl, src, dst, a, b, k, NULL, NULL, x, S, mode, nthreads, out, NULL,
                 threads_used);
}

/* oracle_sweep that also fills nodes: float64[n_nodes][S]. */
int oracle_sweep_nodes(int32_t L, const int64_t *widths, const int64_t *epl,
                       const int32_t *src, const int32_t *dst, const double *a,
                       const double *b, const double *k, const double *x, int64_t S,
                       int32_t mode, int32_t nthreads, double *out, double *nodes)
{
    int rc = oracle_check(L, widths, epl, src, dst, a, b, k);
    if (rc != ORACLE_OK)
        return rc;
    return sweep(0, L, widths, epl, src, dst, a, b, k, NULL, NULL, x, S, mode, nthreads, out, nodes, NULL);
}

/* Lookup factors.  table: float64[n_slots][S], out: float64[S]. */
int oracle_sweep_lookup(int32_t L, const int64_t *widths, const int64_t *epl,
                        const int32_t *src, const int32_t *dst, const int32_t *slot,
                        const double *coef, int32_t n_slots, const double *table, int64_t S,
                        int32_t mode, int32_t nthreads, double *out, int32_t *threads_used)
{
    int rc = oracle_check_lookup(L, widths, epl, src, dst, slot, coef, n_slots);
    if (rc != ORACLE_OK)
        return rc;
    return sweep(1, L, widths, epl, src, dst, NULL, NULL, NULL, slot, coef, table, S, mode, nthreads, out,
                 NULL, threads_used);
}

/* oracle_sweep_lookup that also fills nodes: float64[n_nodes][S]. */
int oracle_sweep_lookup_nodes(int32_t L, const int64_t *widths, const int64_t *epl,
                              const int32_t *src, const int32_t *dst, const int32_t *slot,
                              const double *coef, int32_t n_slots, const double *table, int64_t S,
                              int32_t mode, int32_t nthreads, double *out, double *nodes)
{
    int rc = oracle_check_lookup(L, widths, epl, src, dst, slot, coef, n_slots);
    if (rc != ORACLE_OK)
        return rc;
    return sweep(1, L, widths, epl, src, dst, NULL, NULL, NULL, slot, coef, table, S, mode, nthreads, out,
                 nodes, NULL);
}
