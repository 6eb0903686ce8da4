/*
 * stream_oracle.c -- FP64 streaming oracle for the AB-join matrix profile.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests and the benchmark's CPU legs use it.  It shares no
 * code with the HIP library, nor with the brute-force oracle in abjoin_oracle.c
 * (both are compiled into liborc.so, but neither calls the other).
 *
 * It computes the same thing as the brute-force oracle -- the matrix profile of
 * Def. 7 over the dictionary windows of Def. 8 (Alg. 2, Sec. 3.2) under the
 * z-normalised Euclidean distance of Def. 4 -- with O(1) work per pair instead
 * of O(m), so that joins of a few 1e12 pairs (a held-out series against a whole
 * database) stay within reach of a multi-core host.  The method is the classic
 * diagonal sweep of the matrix-profile literature that the paper builds on:
 *
 *   QT(i, j) = sum_k a[i+k] b[j+k] obeys, along a diagonal j - i = const,
 *   QT(i+1, j+1) = QT(i, j) - a[i] b[j] + a[i+m] b[j+m],
 *   cov(i, j) = QT(i, j) - m mu_a(i) mu_b(j),
 *   rho(i, j) = cov(i, j) / (m sigma_a(i) sigma_b(j)),
 *   d(i, j)   = sqrt(2 m (1 - rho(i, j))),
 *
 * so the nearest window of row i is the valid column with the largest
 * cov(i, j) / sigma_b(j).  Both series are shifted by their own mean first (the
 * distance does not change) and QT is recomputed exactly every kRestart steps,
 * which bounds the rounding drift of the recurrence.  Once every row's best
 * column is known, its distance is recomputed directly as
 * || z(a_i) - z(b_j) || in FP64, so a reported P carries no 1 - rho
 * cancellation; only the choice among near-equal columns can differ from the
 * brute force (by rounding of order 1e-13 in rho).
 *
 * Conventions (the same readings as the brute-force oracle; the paper is
 * silent on them): population deviation; a window is flat iff its variance is
 * <= 1e-10 x the variance of all finite samples of its series, and its
 * z-normalised form is then the zero vector (flat-flat 0, flat vs non-flat
 * sqrt(m)); reference windows holding a non-finite sample are not windows,
 * query rows holding one get P = NaN, I = -1; ties go to the smallest column;
 * a row with no window gets P = +inf, I = -1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define STR_OK 0
#define STR_EINVAL (-1)
#define STR_ENOMEM (-2)

enum { kRestart = 256, kDiagBlock = 16 };

typedef struct {
    int64_t n, W;
    double* y;     /* series minus the mean of its finite samples; non-finite -> 0 */
    double* mu;    /* window mean of y */
    double* sd;    /* window population deviation */
    uint8_t* flat; /* 1 = flat */
    uint8_t* bad;  /* 1 = holds a non-finite sample */
} series_t;

static void series_free(series_t* s)
{
    free(s->y);
    free(s->mu);
    free(s->sd);
    free(s->flat);
    free(s->bad);
    memset(s, 0, sizeof(*s));
}

/* Shifted copy, per-window mean and deviation (each window summed directly),
 * flat and non-finite flags. */
static int series_init(series_t* s, const double* x, int64_t n, int32_t m)
{
    memset(s, 0, sizeof(*s));
    s->n = n;
    s->W = n - m + 1;
    s->y = (double*)malloc(sizeof(double) * (size_t)n);
    s->mu = (double*)malloc(sizeof(double) * (size_t)s->W);
    s->sd = (double*)malloc(sizeof(double) * (size_t)s->W);
    s->flat = (uint8_t*)malloc((size_t)s->W);
    s->bad = (uint8_t*)malloc((size_t)s->W);
    if (!s->y || !s->mu || !s->sd || !s->flat || !s->bad) {
        series_free(s);
        return STR_ENOMEM;
    }
    double tot = 0.0;
    int64_t cnt = 0;
    for (int64_t t = 0; t < n; ++t)
        if (isfinite(x[t])) {
            tot += x[t];
            ++cnt;
        }
    const double shift = cnt ? tot / (double)cnt : 0.0;
    double gv = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        if (isfinite(x[t])) {
            s->y[t] = x[t] - shift;
            gv += s->y[t] * s->y[t];
        } else {
            s->y[t] = 0.0;
        }
    }
    gv = cnt ? gv / (double)cnt : 0.0;
    /* running count of non-finite samples in the window */
    int64_t nbad = 0;
    for (int64_t t = 0; t < m - 1; ++t) nbad += !isfinite(x[t]);
    for (int64_t i = 0; i < s->W; ++i) {
        nbad += !isfinite(x[i + m - 1]);
        if (i > 0) nbad -= !isfinite(x[i - 1]);
        s->bad[i] = nbad > 0;
        double sum = 0.0;
        for (int32_t k = 0; k < m; ++k) sum += s->y[i + k];
        const double mean = sum / (double)m;
        double ss = 0.0;
        for (int32_t k = 0; k < m; ++k) {
            const double e = s->y[i + k] - mean;
            ss += e * e;
        }
        const double var = ss / (double)m;
        s->mu[i] = mean;
        s->sd[i] = sqrt(var);
        s->flat[i] = !s->bad[i] && var <= 1e-10 * gv;
    }
    return STR_OK;
}

/* || z(a_i) - z(b_j) || for two non-flat, finite windows. */
static double direct_dist(const series_t* A, int64_t i, const series_t* B, int64_t j, int32_t m)
{
    const double ia = 1.0 / A->sd[i], ib = 1.0 / B->sd[j];
    double acc = 0.0;
    for (int32_t k = 0; k < m; ++k) {
        const double e = (A->y[i + k] - A->mu[i]) * ia - (B->y[j + k] - B->mu[j]) * ib;
        acc += e * e;
    }
    return sqrt(acc);
}

/*
 * Streaming AB-join.  q (nq samples) against the windows of d (nd samples) that
 * lie inside one segment of bounds[0..nseg] (Def. 8).  P, I: nq - m + 1 entries.
 */
int orc_ab_join_stream(const double* q, int64_t nq, const double* d, int64_t nd, const int64_t* bounds,
                       int32_t nseg, int32_t m, double* P, int64_t* I, int32_t nthreads)
{
    if (!q || !d || !bounds || !P || !I || m < 2 || nq < m || nd < 1 || nseg < 1) return STR_EINVAL;
    if (bounds[0] != 0 || bounds[nseg] != nd) return STR_EINVAL;
    for (int32_t s = 0; s < nseg; ++s)
        if (bounds[s + 1] <= bounds[s]) return STR_EINVAL;
    const int64_t WA = nq - m + 1;
    if (nd < m) {
        /* no reference window at all */
        series_t A;
        if (series_init(&A, q, nq, m) != STR_OK) return STR_ENOMEM;
        for (int64_t i = 0; i < WA; ++i) {
            P[i] = A.bad[i] ? NAN : INFINITY;
            I[i] = -1;
        }
        series_free(&A);
        return STR_OK;
    }
    series_t A, B;
    if (series_init(&A, q, nq, m) != STR_OK) return STR_ENOMEM;
    if (series_init(&B, d, nd, m) != STR_OK) {
        series_free(&A);
        return STR_ENOMEM;
    }
    const int64_t WB = B.W;
    /* usable[j]: inside one segment, finite, not flat (flat windows are settled
     * by the convention afterwards) */
    uint8_t* inside = (uint8_t*)calloc((size_t)WB, 1);
    double* wcol = (double*)malloc(sizeof(double) * (size_t)WB);  /* 1/sigma_b, or 0 when unusable */
    double* mua_m = (double*)malloc(sizeof(double) * (size_t)WA); /* m mu_a(i) */
    if (!inside || !wcol || !mua_m) {
        free(inside);
        free(wcol);
        free(mua_m);
        series_free(&A);
        series_free(&B);
        return STR_ENOMEM;
    }
    for (int32_t s = 0; s < nseg; ++s)
        for (int64_t j = bounds[s]; j + m <= bounds[s + 1]; ++j) inside[j] = 1;
    int64_t first_valid = -1, first_flat = -1;
    for (int64_t j = 0; j < WB; ++j) {
        const int valid = inside[j] && !B.bad[j];
        if (valid && first_valid < 0) first_valid = j;
        if (valid && B.flat[j] && first_flat < 0) first_flat = j;
        wcol[j] = (valid && !B.flat[j]) ? 1.0 / B.sd[j] : 0.0;
        inside[j] = (uint8_t)(valid && !B.flat[j]);
    }
    for (int64_t i = 0; i < WA; ++i) mua_m[i] = (double)m * A.mu[i];

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int nth = omp_get_max_threads();
#else
    (void)nthreads;
    const int nth = 1;
#endif
    /* per-thread running best score and column of every row */
    double* bs = (double*)malloc(sizeof(double) * (size_t)WA * (size_t)nth);
    int64_t* bj = (int64_t*)malloc(sizeof(int64_t) * (size_t)WA * (size_t)nth);
    if (!bs || !bj) {
        free(bs);
        free(bj);
        free(inside);
        free(wcol);
        free(mua_m);
        series_free(&A);
        series_free(&B);
        return STR_ENOMEM;
    }
    for (int64_t t = 0; t < WA * (int64_t)nth; ++t) {
        bs[t] = -INFINITY;
        bj[t] = -1;
    }
    /* diagonals c = j - i run from -(WA - 1) to WB - 1 */
    const int64_t ndiag = WA + WB - 1;
    const int64_t nblk = (ndiag + kDiagBlock - 1) / kDiagBlock;
    const double* ya = A.y;
    const double* yb = B.y;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t blk = 0; blk < nblk; ++blk) {
#ifdef _OPENMP
        const int tid = omp_get_thread_num();
#else
        const int tid = 0;
#endif
        double* mybs = bs + (size_t)tid * (size_t)WA;
        int64_t* mybj = bj + (size_t)tid * (size_t)WA;
        for (int64_t c = -(WA - 1) + blk * kDiagBlock; c < -(WA - 1) + (blk + 1) * kDiagBlock && c < WB; ++c) {
            const int64_t i0 = c < 0 ? -c : 0;
            const int64_t i1 = (WA < WB - c) ? WA : WB - c; /* exclusive */
            double qt = 0.0;
            for (int64_t i = i0; i < i1; ++i) {
                const int64_t j = i + c;
                if ((i - i0) % kRestart == 0) {
                    qt = 0.0;
                    for (int32_t k = 0; k < m; ++k) qt += ya[i + k] * yb[j + k];
                } else {
                    qt += ya[i + m - 1] * yb[j + m - 1] - ya[i - 1] * yb[j - 1];
                }
                if (!inside[j]) continue;
                const double score = (qt - mua_m[i] * B.mu[j]) * wcol[j];
                if (score > mybs[i] || (score == mybs[i] && j < mybj[i])) {
                    mybs[i] = score;
                    mybj[i] = j;
                }
            }
        }
    }
    /* merge the threads' bests, then settle each row */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < WA; ++i) {
        double s = -INFINITY;
        int64_t j = -1;
        for (int t = 0; t < nth; ++t) {
            const double v = bs[(size_t)t * (size_t)WA + (size_t)i];
            const int64_t k = bj[(size_t)t * (size_t)WA + (size_t)i];
            if (k < 0) continue;
            if (j < 0 || v > s || (v == s && k < j)) {
                s = v;
                j = k;
            }
        }
        if (A.bad[i]) {
            P[i] = NAN;
            I[i] = -1;
            continue;
        }
        if (A.flat[i]) {
            if (first_flat >= 0) {
                P[i] = 0.0;
                I[i] = first_flat;
            } else if (first_valid >= 0) {
                P[i] = sqrt((double)m);
                I[i] = first_valid;
            } else {
                P[i] = INFINITY;
                I[i] = -1;
            }
            continue;
        }
        double dist = INFINITY;
        if (j >= 0) dist = direct_dist(&A, i, &B, j, m);
        if (first_flat >= 0) {
            const double sm = sqrt((double)m);
            if (sm < dist || (sm == dist && first_flat < j)) {
                dist = sm;
                j = first_flat;
            }
        }
        P[i] = dist;
        I[i] = j;
    }
    free(bs);
    free(bj);
    free(inside);
    free(wcol);
    free(mua_m);
    series_free(&A);
    series_free(&B);
    return STR_OK;
}
