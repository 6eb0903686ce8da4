/*
 * abjoin_oracle.c -- plain, slow FP64 CPU oracle for the AB-join matrix profile.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (paper: "Error-bounded Approximate Time Series Joins Using
 * Compact Dictionary Representations of Time Series"):
 *   - Def. 2 / Def. 3: the length-m subsequences T[i : i+m] of a series,
 *     i = 0 .. n-m (0-based here; the paper counts from 1).
 *   - Def. 4: the distance between two subsequences is the z-normalised
 *     Euclidean distance (the paper cites MASS for it and gives no formula);
 *     this oracle normalises each window by its own mean and POPULATION standard
 *     deviation (divide by m), mean and deviation both taken in two passes over
 *     the window, and takes the plain Euclidean norm of the difference.
 *   - Def. 5 - Def. 7: the matrix profile P_AB[i] is the distance from window i
 *     of the query to its nearest neighbour among the reference windows; the
 *     join set pairs i with that neighbour, reported here as the index I_AB[i].
 *   - Def. 8: for a dictionary stored as a concatenation with segment offsets
 *     b_0 = 0 < b_1 < ... < b_S = n, the reference windows are those that slide
 *     inside one segment: j is a window iff b_s <= j and j + m <= b_{s+1} for
 *     some s.  Alg. 2 (JoinDictionary) is the element-wise minimum of the joins
 *     against every segment, which equals one nearest-neighbour search over
 *     exactly these windows; that is what orc_ab_join does.
 *   - Alg. 2 initialises P to +inf: a query window with no reference window
 *     gets P = +inf, I = -1.
 *
 * Readings where the paper is silent (each listed with its reason in the
 * design notes):
 *   - Constant ("flat") windows: a window is flat iff its population variance
 *     is <= 1e-10 times the population variance of all finite samples of the
 *     series it comes from.  A flat window's z-normalised form is the zero
 *     vector, so flat-flat = 0 and flat-vs-non-flat = sqrt(m) exactly.
 *   - Windows holding a non-finite sample: on the reference side they are not
 *     windows; on the query side the row gets P = NaN, I = -1.
 *   - Ties: the smallest reference index wins (strict '<' in index order).
 *   - No exclusion zone in the AB-join.  The self-join used by the learning
 *     phase (Alg. 1's P_B) excludes |i - j| <= floor(m/2).
 *
 * All arithmetic is IEEE double; the build uses -O2 without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* Population variance of the finite samples of x (two passes). 0 if none. */
static double series_var(const double* x, int64_t n)
{
    double s = 0.0;
    int64_t c = 0;
    for (int64_t t = 0; t < n; ++t)
        if (isfinite(x[t])) { s += x[t]; ++c; }
    if (c == 0) return 0.0;
    const double mu = s / (double)c;
    double v = 0.0;
    for (int64_t t = 0; t < n; ++t)
        if (isfinite(x[t])) { const double e = x[t] - mu; v += e * e; }
    return v / (double)c;
}

/*
 * Per-window mean, population standard deviation, flat flag and non-finite
 * flag for the n-m+1 windows of x.  Two passes per window.
 */
int orc_window_stats(const double* x, int64_t n, int32_t m,
                     double* mu, double* sd, uint8_t* flat, uint8_t* bad)
{
    if (!x || m < 2 || n < m) return ORC_EINVAL;
    const double gvar = series_var(x, n);
    const int64_t W = n - m + 1;
    for (int64_t i = 0; i < W; ++i) {
        int finite = 1;
        double s = 0.0;
        for (int32_t k = 0; k < m; ++k) {
            if (!isfinite(x[i + k])) { finite = 0; break; }
            s += x[i + k];
        }
        if (!finite) {
            if (mu) mu[i] = NAN;
            if (sd) sd[i] = NAN;
            if (flat) flat[i] = 0;
            if (bad) bad[i] = 1;
            continue;
        }
        const double mean = s / (double)m;
        double v = 0.0;
        for (int32_t k = 0; k < m; ++k) {
            const double e = x[i + k] - mean;
            v += e * e;
        }
        v /= (double)m;
        if (mu) mu[i] = mean;
        if (sd) sd[i] = sqrt(v);
        if (flat) flat[i] = (uint8_t)(v <= 1e-10 * gvar);
        if (bad) bad[i] = 0;
    }
    return ORC_OK;
}

/* Def. 8: valid[j] = 1 iff window j lies inside one segment of the dictionary. */
int orc_valid_windows(const int64_t* bounds, int32_t nseg, int64_t n, int32_t m, uint8_t* valid)
{
    if (!bounds || nseg < 1 || m < 2 || n < m || !valid) return ORC_EINVAL;
    if (bounds[0] != 0 || bounds[nseg] != n) return ORC_EINVAL;
    for (int32_t s = 0; s < nseg; ++s)
        if (bounds[s + 1] <= bounds[s]) return ORC_EINVAL;
    const int64_t W = n - m + 1;
    memset(valid, 0, (size_t)W);
    for (int32_t s = 0; s < nseg; ++s)
        for (int64_t j = bounds[s]; j + m <= bounds[s + 1]; ++j)
            valid[j] = 1;
    return ORC_OK;
}

/* z-normalised windows, row-major W x m; flat windows become zero vectors. */
static double* znorm_all(const double* x, int64_t n, int32_t m,
                         uint8_t** flat_out, uint8_t** bad_out)
{
    const int64_t W = n - m + 1;
    double* mu = (double*)malloc(sizeof(double) * (size_t)W);
    double* sd = (double*)malloc(sizeof(double) * (size_t)W);
    uint8_t* flat = (uint8_t*)malloc((size_t)W);
    uint8_t* bad = (uint8_t*)malloc((size_t)W);
    double* z = (double*)malloc(sizeof(double) * (size_t)W * (size_t)m);
    if (!mu || !sd || !flat || !bad || !z) {
        free(mu); free(sd); free(flat); free(bad); free(z);
        return NULL;
    }
    orc_window_stats(x, n, m, mu, sd, flat, bad);
    for (int64_t i = 0; i < W; ++i) {
        double* zi = z + (size_t)i * (size_t)m;
        if (bad[i] || flat[i]) {
            for (int32_t k = 0; k < m; ++k) zi[k] = 0.0;
        } else {
            for (int32_t k = 0; k < m; ++k) zi[k] = (x[i + k] - mu[i]) / sd[i];
        }
    }
    free(mu);
    free(sd);
    *flat_out = flat;
    *bad_out = bad;
    return z;
}

/* Distance between two z-normalised windows under the flat convention. */
static double zdist(const double* za, int fa, const double* zb, int fb, int32_t m)
{
    if (fa && fb) return 0.0;
    if (fa || fb) return sqrt((double)m);
    double acc = 0.0;
    for (int32_t k = 0; k < m; ++k) {
        const double e = za[k] - zb[k];
        acc += e * e;
    }
    return sqrt(acc);
}

/*
 * AB-join of query q against the windows of dictionary d that lie inside one
 * segment (Alg. 2 over the windows of Def. 8), by brute force.
 *
 * rows: optional list of query windows to evaluate (NULL = all n_q-m+1, in
 * order); results are written compactly, entry r for rows[r].
 * P: distance to the nearest neighbour; I: its 0-based window index in d;
 * P2 (optional): smallest distance over all other reference windows.
 * nthreads <= 0 lets OpenMP choose.
 */
int orc_ab_join(const double* q, int64_t nq, const double* d, int64_t nd,
                const int64_t* bounds, int32_t nseg, int32_t m,
                const int64_t* rows, int64_t nrows,
                double* P, int64_t* I, double* P2, int32_t nthreads)
{
    if (!q || !d || !bounds || !P || !I || m < 2 || nq < m || nd < 1) return ORC_EINVAL;
    const int64_t WA = nq - m + 1;
    const int64_t WB = nd >= m ? nd - m + 1 : 0;
    if (!rows) nrows = WA;
    for (int64_t r = 0; rows && r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= WA) return ORC_EINVAL;
    if (bounds[0] != 0 || bounds[nseg] != nd) return ORC_EINVAL;
    for (int32_t s = 0; s < nseg; ++s)
        if (bounds[s + 1] <= bounds[s]) return ORC_EINVAL;

    uint8_t *fa = NULL, *ba = NULL, *fb = NULL, *bb = NULL, *valid = NULL;
    double* za = znorm_all(q, nq, m, &fa, &ba);
    double* zb = WB ? znorm_all(d, nd, m, &fb, &bb) : NULL;
    if (WB) {
        valid = (uint8_t*)malloc((size_t)WB);
        if (valid) orc_valid_windows(bounds, nseg, nd, m, valid);
    }
    if (!za || (WB && (!zb || !valid))) {
        free(za); free(fa); free(ba); free(zb); free(fb); free(bb); free(valid);
        return ORC_ENOMEM;
    }
    /* A reference window with a non-finite sample is not a window. */
    for (int64_t j = 0; j < WB; ++j)
        if (bb[j]) valid[j] = 0;

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows ? rows[r] : r;
        if (ba[i]) {
            P[r] = NAN;
            I[r] = -1;
            if (P2) P2[r] = NAN;
            continue;
        }
        const double* zi = za + (size_t)i * (size_t)m;
        double best = INFINITY, second = INFINITY;
        int64_t arg = -1;
        for (int64_t j = 0; j < WB; ++j) {
            if (!valid[j]) continue;
            const double dist = zdist(zi, fa[i], zb + (size_t)j * (size_t)m, fb[j], m);
            if (dist < best) {
                second = best;
                best = dist;
                arg = j;
            } else if (dist < second) {
                second = dist;
            }
        }
        P[r] = best;
        I[r] = arg;
        if (P2) P2[r] = second;
    }
    free(za); free(fa); free(ba); free(zb); free(fb); free(bb); free(valid);
    return ORC_OK;
}

/*
 * Distances for an explicit list of (query window, reference window) pairs,
 * with no segment mask: out[p] = dist(q[ii[p] : ii[p]+m], d[jj[p] : jj[p]+m]).
 * NaN if either window holds a non-finite sample.
 */
int orc_pair_dists(const double* q, int64_t nq, const double* d, int64_t nd, int32_t m,
                   const int64_t* ii, const int64_t* jj, int64_t npairs, double* out)
{
    if (!q || !d || !ii || !jj || !out || m < 2 || nq < m || nd < m) return ORC_EINVAL;
    const int64_t WA = nq - m + 1, WB = nd - m + 1;
    for (int64_t p = 0; p < npairs; ++p)
        if (ii[p] < 0 || ii[p] >= WA || jj[p] < 0 || jj[p] >= WB) return ORC_EINVAL;
    const double gva = series_var(q, nq), gvb = series_var(d, nd);
    double* za = (double*)malloc(sizeof(double) * (size_t)m);
    double* zb = (double*)malloc(sizeof(double) * (size_t)m);
    if (!za || !zb) { free(za); free(zb); return ORC_ENOMEM; }
    for (int64_t p = 0; p < npairs; ++p) {
        const double* wins[2] = {q + ii[p], d + jj[p]};
        const double gv[2] = {gva, gvb};
        double* zs[2] = {za, zb};
        int flat[2] = {0, 0}, bad = 0;
        for (int w = 0; w < 2 && !bad; ++w) {
            const double* x = wins[w];
            double s = 0.0;
            for (int32_t k = 0; k < m; ++k) {
                if (!isfinite(x[k])) { bad = 1; break; }
                s += x[k];
            }
            if (bad) break;
            const double mean = s / (double)m;
            double v = 0.0;
            for (int32_t k = 0; k < m; ++k) { const double e = x[k] - mean; v += e * e; }
            v /= (double)m;
            flat[w] = v <= 1e-10 * gv[w];
            const double sdv = sqrt(v);
            for (int32_t k = 0; k < m; ++k) zs[w][k] = flat[w] ? 0.0 : (x[k] - mean) / sdv;
        }
        out[p] = bad ? NAN : zdist(za, flat[0], zb, flat[1], m);
    }
    free(za);
    free(zb);
    return ORC_OK;
}

/* Full distance matrix D[i * WB + j] between every window of q and of d (no mask). */
int orc_dist_matrix(const double* q, int64_t nq, const double* d, int64_t nd, int32_t m, double* D)
{
    if (!q || !d || !D || m < 2 || nq < m || nd < m) return ORC_EINVAL;
    const int64_t WA = nq - m + 1, WB = nd - m + 1;
    uint8_t *fa = NULL, *ba = NULL, *fb = NULL, *bb = NULL;
    double* za = znorm_all(q, nq, m, &fa, &ba);
    double* zb = znorm_all(d, nd, m, &fb, &bb);
    if (!za || !zb) { free(za); free(fa); free(ba); free(zb); free(fb); free(bb); return ORC_ENOMEM; }
    for (int64_t i = 0; i < WA; ++i)
        for (int64_t j = 0; j < WB; ++j)
            D[(size_t)i * (size_t)WB + (size_t)j] =
                (ba[i] || bb[j]) ? NAN
                                 : zdist(za + (size_t)i * (size_t)m, fa[i], zb + (size_t)j * (size_t)m, fb[j], m);
    free(za); free(fa); free(ba); free(zb); free(fb); free(bb);
    return ORC_OK;
}

/*
 * Self-join matrix profile (the intra-similarity join that gives Alg. 1's P_B): for
 * every window i of x, the nearest other window j with |i - j| > excl.
 */
int orc_self_join(const double* x, int64_t n, int32_t m, int64_t excl,
                  double* P, int64_t* I, int32_t nthreads)
{
    if (!x || !P || !I || m < 2 || n < m || excl < 0) return ORC_EINVAL;
    const int64_t W = n - m + 1;
    uint8_t *f = NULL, *b = NULL;
    double* z = znorm_all(x, n, m, &f, &b);
    if (!z) return ORC_ENOMEM;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < W; ++i) {
        double best = INFINITY;
        int64_t arg = -1;
        if (!b[i]) {
            for (int64_t j = 0; j < W; ++j) {
                if (b[j] || llabs(i - j) <= excl) continue;
                const double dist = zdist(z + (size_t)i * (size_t)m, f[i], z + (size_t)j * (size_t)m, f[j], m);
                if (dist < best) { best = dist; arg = j; }
            }
        } else {
            best = NAN;
        }
        P[i] = best;
        I[i] = arg;
    }
    free(z); free(f); free(b);
    return ORC_OK;
}

/*
 * Distance profile (Def. 4): the distance between the length-m query w and
 * every window of x.  The flat test for w uses the variance of x's samples,
 * since w is one of x's subsequences in Alg. 1.
 */
int orc_dist_profile(const double* x, int64_t n, int32_t m, const double* w, double* S)
{
    if (!x || !w || !S || m < 2 || n < m) return ORC_EINVAL;
    const int64_t W = n - m + 1;
    const double gv = series_var(x, n);
    double* zw = (double*)malloc(sizeof(double) * (size_t)m);
    if (!zw) return ORC_ENOMEM;
    double s = 0.0;
    int badw = 0;
    for (int32_t k = 0; k < m; ++k) { if (!isfinite(w[k])) badw = 1; s += w[k]; }
    const double mean = s / (double)m;
    double v = 0.0;
    for (int32_t k = 0; k < m; ++k) { const double e = w[k] - mean; v += e * e; }
    v /= (double)m;
    const int fw = v <= 1e-10 * gv;
    for (int32_t k = 0; k < m; ++k) zw[k] = fw ? 0.0 : (w[k] - mean) / sqrt(v);
    uint8_t *f = NULL, *b = NULL;
    double* z = znorm_all(x, n, m, &f, &b);
    if (!z) { free(zw); return ORC_ENOMEM; }
    for (int64_t j = 0; j < W; ++j)
        S[j] = (badw || b[j]) ? NAN : zdist(zw, fw, z + (size_t)j * (size_t)m, f[j], m);
    free(z); free(f); free(b); free(zw);
    return ORC_OK;
}
