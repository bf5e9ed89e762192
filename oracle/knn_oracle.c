/*
 * knn_oracle.c -- plain FP64 brute-force k-nearest-neighbour oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check the GPU library against the plain
 * definition.  It shares no code, header or constant with the GPU library.
 *
 * What it computes (Garcia, Debreuve, Barlaud, "Fast k Nearest Neighbor
 * Search using GPU", Section 2.1, problem definition): for a reference set
 * R = {r_1..r_m} and a query set Q = {q_1..q_n} in d dimensions, the k
 * references nearest to each query under a given distance.  Section 2.1
 * names the Euclidean and Manhattan distances and the infinity-norm
 * distance as examples; all three are implemented.
 *
 * How (the brute-force method of Section 2.1, step by step, for each query):
 *   1. compute the distance between q_i and every r_j, in double precision,
 *      in the difference form (the float inputs are converted exactly):
 *        Euclidean: v = sum_t (q_t - r_t)^2, ranked on v, reported sqrt(v)
 *        Manhattan: v = sum_t |q_t - r_t|
 *        infinity : v = max_t |q_t - r_t|
 *      The sum runs sequentially over t = 0..d-1.
 *   2. sort the m pairs (v_j, j) in lexicographic order: distance first,
 *      then reference index (readings: equal distances go to the lower
 *      index; the Euclidean sort uses v, not sqrt(v), so that rounding of
 *      the root creates no ties).
 *   3. keep the first k.
 * Step 2 is either a full qsort of all m pairs (mode 0, the literal method)
 * or a bounded max-heap of k pairs followed by a sort of those k (mode 1).
 * The comparator is a total order on (v, j), so both modes return the same
 * result; the tests assert that.
 *
 * Indices are 0-based (the paper writes r_1..r_m; reading: 0-based).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORACLE_L2 = 0, ORACLE_L1 = 1, ORACLE_LINF = 2 };

typedef struct {
    double v;
    int64_t j;
} oracle_pair;

/* lexicographic (distance, index) */
static int pair_less(const oracle_pair* a, const oracle_pair* b) {
    if (a->v < b->v) return 1;
    if (a->v > b->v) return 0;
    return a->j < b->j;
}

static int pair_cmp(const void* pa, const void* pb) {
    const oracle_pair* a = (const oracle_pair*)pa;
    const oracle_pair* b = (const oracle_pair*)pb;
    if (pair_less(a, b)) return -1;
    if (pair_less(b, a)) return 1;
    return 0;
}

/* Step 1: the ranking value of one pair, in the difference form. */
static double pair_value(const float* q, const float* r, int32_t d, int32_t metric) {
    double s = 0.0;
    for (int32_t t = 0; t < d; ++t) {
        double diff = (double)q[t] - (double)r[t];
        if (metric == ORACLE_L2) {
            s += diff * diff;
        } else if (metric == ORACLE_L1) {
            s += fabs(diff);
        } else {
            double a = fabs(diff);
            if (a > s) s = a;
        }
    }
    return s;
}

static double reported(double v, int32_t metric) { return metric == ORACLE_L2 ? sqrt(v) : v; }

/* max-heap on the (v, j) order: the root is the largest of the kept pairs */
static void heap_sift_down(oracle_pair* h, int64_t size, int64_t i) {
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, big = i;
        if (l < size && pair_less(&h[big], &h[l])) big = l;
        if (r < size && pair_less(&h[big], &h[r])) big = r;
        if (big == i) return;
        oracle_pair t = h[i];
        h[i] = h[big];
        h[big] = t;
        i = big;
    }
}

static void heap_sift_up(oracle_pair* h, int64_t i) {
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!pair_less(&h[p], &h[i])) return;
        oracle_pair t = h[i];
        h[i] = h[p];
        h[p] = t;
        i = p;
    }
}

/*
 * knn_oracle: dist[n*k] (double, ascending per query), idx[n*k] (int64).
 * Q is [n][d], R is [m][d], both row-major float32.  Returns 0, or -1 on a
 * bad argument (1 <= k <= m and d >= 1 are required), -2 if memory ran out.
 */
int knn_oracle(const float* Q, int64_t n, const float* R, int64_t m, int32_t d, int32_t k,
               int32_t metric, int32_t mode, int32_t threads, double* dist, int64_t* idx) {
    if (n < 0 || m < 1 || d < 1 || k < 1 || k > m) return -1;
    if (metric < ORACLE_L2 || metric > ORACLE_LINF) return -1;
    if (mode != 0 && mode != 1) return -1;
    int failed = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
#pragma omp parallel
    {
        int64_t cap = (mode == 0) ? m : (int64_t)k;
        oracle_pair* buf = (oracle_pair*)malloc((size_t)cap * sizeof(oracle_pair));
        if (!buf) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            if (!buf) continue;
            const float* q = Q + i * (int64_t)d;
            int64_t kept = 0;
            for (int64_t j = 0; j < m; ++j) {
                oracle_pair p;
                p.v = pair_value(q, R + j * (int64_t)d, d, metric);
                p.j = j;
                if (mode == 0) {
                    buf[kept++] = p;
                } else if (kept < k) {
                    buf[kept] = p;
                    heap_sift_up(buf, kept);
                    ++kept;
                } else if (pair_less(&p, &buf[0])) {
                    buf[0] = p;
                    heap_sift_down(buf, kept, 0);
                }
            }
            qsort(buf, (size_t)kept, sizeof(oracle_pair), pair_cmp);
            for (int32_t r = 0; r < k; ++r) {
                dist[i * k + r] = reported(buf[r].v, metric);
                idx[i * k + r] = buf[r].j;
            }
        }
        free(buf);
    }
    return failed ? -2 : 0;
}

/*
 * knn_oracle_pairs: the double-precision distance of `count` given pairs
 * (query qi[c], reference rj[c]) into out[c], reported form (sqrt for L2).
 * Used to judge a returned index that differs from the oracle's one.
 */
int knn_oracle_pairs(const float* Q, const float* R, int32_t d, int32_t metric,
                     const int64_t* qi, const int64_t* rj, int64_t count, double* out) {
    if (d < 1 || metric < ORACLE_L2 || metric > ORACLE_LINF || count < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < count; ++c)
        out[c] = reported(pair_value(Q + qi[c] * (int64_t)d, R + rj[c] * (int64_t)d, d, metric), metric);
    return 0;
}
