// Per-window statistics on the GPU: the O(n) step before the pair loop.
//
// The z-normalised distance (Def. 4) needs each window's mean and population
// deviation.  They come from prefix sums of the series kept as double-double
// pairs (error-free TwoSum accumulation, squares split exactly with an FMA):
// on a long random walk the plain running sum of squares reaches ~1e12 and a
// window difference would otherwise lose ~1e-4 absolute, which is enough to
// misjudge short, nearly constant windows; with ~106 bits the window variance
// m var = sum x^2 - (sum x)^2 / m keeps full FP64 precision without centring
// the series first.  Four launches: block sums, top scan (also the series
// variance for the flat test), local scan, per-window pass.  The same pass produces the
// per-window terms of the diagonal covariance recurrence used by the FP32 join:
//   df(i) = (x[i+m] - x[i]) / 2,
//   dg(i) = (x[i+m] - mu(i+1)) + (x[i] - mu(i)),
// with which cov(i+1, j+1) = cov(i, j) + df_a(i) dg_b(j) + df_b(j) dg_a(i),
// where cov(i, j) = sum_k (a[i+k] - mu_a(i)) (b[j+k] - mu_b(j)).
#include <math.h>
#include <string.h>

#include "abj_internal.hpp"

// The double-double sums below are error-free transformations: a multiply
// must never be fused into the add that follows it, or the TwoSum error terms
// stop matching the sums they correct.  Explicit fma() calls are unaffected.
#pragma clang fp contract(off)

namespace abj {

namespace {

// One wave per workgroup: the block scans below then wait at barriers of one
// wave only (4 waves per workgroup took 4 us longer on a 131,072 + 32,000
// sample pair of series).
constexpr int kThreads = 64;
constexpr int kPerThread = 8;
constexpr int kBlockElems = kThreads * kPerThread;  // 512 samples per scan block

__device__ inline bool finite_d(double v) { return isfinite(v); }

// Double-double value hi + lo with |lo| <= ulp(hi) / 2.
struct dd {
    double hi, lo;
};

// Knuth's TwoSum: a + b = s + e exactly.
__device__ inline dd two_sum(double a, double b)
{
    const double s = a + b;
    const double bp = s - a;
    const double e = (a - (s - bp)) + (b - bp);
    return {s, e};
}

__device__ inline dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return two_sum(s.hi, s.lo);
}

// Exact square of d as a double-double (FMA gives the rounding error).
__device__ inline dd dd_sqr(double d)
{
    const double p = d * d;
    return {p, fma(d, d, -p)};
}

// b - a as a double-double.
__device__ inline dd dd_sub(dd b, dd a) { return dd_add(b, {-a.hi, -a.lo}); }

// a * a as a double-double.
__device__ inline dd dd_square(dd a)
{
    const double p = a.hi * a.hi;
    const double e = fma(a.hi, a.hi, -p) + 2.0 * a.hi * a.lo;
    return two_sum(p, e);
}

// a / b for a double divisor, as a double-double.
__device__ inline dd dd_div(dd a, double b)
{
    const double q1 = a.hi / b;
    const double p = q1 * b;
    const double pe = fma(q1, b, -p);
    const dd r = dd_sub(a, {p, pe});
    const double q2 = (r.hi + r.lo) / b;
    return two_sum(q1, q2);
}

// Block-wide exclusive scans (Hillis-Steele in LDS).
__device__ inline dd block_excl_scan_dd(dd v, double* shh, double* shl, dd* total)
{
    const int t = threadIdx.x;
    shh[t] = v.hi;
    shl[t] = v.lo;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        dd add = {0.0, 0.0};
        if (t >= off) add = {shh[t - off], shl[t - off]};
        __syncthreads();
        const dd cur = dd_add({shh[t], shl[t]}, add);
        shh[t] = cur.hi;
        shl[t] = cur.lo;
        __syncthreads();
    }
    const dd incl = {shh[t], shl[t]};
    if (total) *total = {shh[kThreads - 1], shl[kThreads - 1]};
    __syncthreads();
    return dd_add(incl, {-v.hi, -v.lo});
}

__device__ inline long long block_excl_scan_i(long long v, long long* sh, long long* total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        long long add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    long long incl = sh[t];
    if (total) *total = sh[kThreads - 1];
    __syncthreads();
    return incl - v;
}

// Pass 1: the working copy xc (non-finite -> 0, zero tail of kSeriesPad
// samples), its 16-row copy xt (16 nb16 samples; the grid covers them, as
// 16 divides kBlockElems) and per-block sums of xc, xc^2 (double-double) and
// the non-finite count.
__device__ void block_sums_body(const double* __restrict__ x, int64_t n, double* __restrict__ xc,
                                double* __restrict__ xt, int64_t nb16, dd* __restrict__ b1, dd* __restrict__ b2,
                                long long* __restrict__ bnf, int64_t blk)
{
    __shared__ double shh[kThreads], shl[kThreads];
    __shared__ long long shc[kThreads];
    const int64_t base = blk * kBlockElems + (int64_t)threadIdx.x * kPerThread;
    dd s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
    long long nf = 0;
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        const int64_t t = base + e;
        double d = 0.0;
        if (t < n) {
            double v = x[t];
            if (finite_d(v)) {
                d = v;
            } else {
                ++nf;
            }
            xc[t] = d;
            s1 = dd_add(s1, {d, 0.0});
            s2 = dd_add(s2, dd_sqr(d));
        } else if (t < n + kSeriesPad) {
            xc[t] = 0.0;
        }
        if (t < 16 * nb16) xt[(t & 15) * nb16 + (t >> 4)] = d;
    }
    dd t1, t2;
    long long tn;
    block_excl_scan_dd(s1, shh, shl, &t1);
    block_excl_scan_dd(s2, shh, shl, &t2);
    block_excl_scan_i(nf, shc, &tn);
    if (threadIdx.x == 0) {
        b1[blk] = t1;
        b2[blk] = t2;
        bnf[blk] = tn;
    }
}

// Pass 2: exclusive scan of the block sums (one workgroup); the series'
// finite count -> scal[2], variance about its mean -> scal[1] (scal[0] = 0:
// the working copy is not shifted); first[] reset for the per-window pass.
__device__ void scan_top_body(dd* __restrict__ b1, dd* __restrict__ b2, long long* __restrict__ bnf, int64_t nb,
                              int64_t n, double* __restrict__ scal, unsigned long long* __restrict__ first)
{
    __shared__ double shh[kThreads], shl[kThreads];
    __shared__ long long shc[kThreads];
    const int64_t per = (nb + kThreads - 1) / kThreads;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    dd s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
    long long nf = 0;
    for (int64_t b = lo; b < hi; ++b) {
        s1 = dd_add(s1, b1[b]);
        s2 = dd_add(s2, b2[b]);
        nf += bnf[b];
    }
    dd tot1, tot2;
    long long totn;
    dd o1 = block_excl_scan_dd(s1, shh, shl, &tot1);
    dd o2 = block_excl_scan_dd(s2, shh, shl, &tot2);
    long long on = block_excl_scan_i(nf, shc, &totn);
    for (int64_t b = lo; b < hi; ++b) {
        const dd v1 = b1[b], v2 = b2[b];
        const long long vn = bnf[b];
        b1[b] = o1;
        b2[b] = o2;
        bnf[b] = on;
        o1 = dd_add(o1, v1);
        o2 = dd_add(o2, v2);
        on += vn;
    }
    if (threadIdx.x == 0) {
        const double cnt = (double)(n - totn);
        double var = 0.0;
        if (cnt > 0) {
            // n var = sum x^2 - (sum x)^2 / n over the finite samples
            const dd v = dd_sub(tot2, dd_div(dd_square(tot1), cnt));
            var = (v.hi + v.lo) / cnt;
            if (var < 0) var = 0.0;
        }
        scal[0] = 0.0;
        scal[1] = var;
        scal[2] = cnt;
        first[0] = ~0ull;
        first[1] = ~0ull;
    }
}

// Pass 3: inclusive prefix arrays S1[t+1], S2[t+1], NF[t+1] (S[0] = 0).
__device__ void scan_local_body(const double* __restrict__ xc, int64_t n, const dd* __restrict__ b1,
                                const dd* __restrict__ b2, const long long* __restrict__ bnf, dd* __restrict__ S1,
                                dd* __restrict__ S2, int* __restrict__ NF, const double* __restrict__ x, int64_t blk)
{
    __shared__ double shh[kThreads], shl[kThreads];
    __shared__ long long shc[kThreads];
    const int64_t base = blk * kBlockElems + (int64_t)threadIdx.x * kPerThread;
    dd v1[kPerThread], v2[kPerThread];
    int vn[kPerThread];
    dd s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
    long long nf = 0;
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        const int64_t t = base + e;
        double d = 0.0;
        int bad = 0;
        if (t < n) {
            d = xc[t];
            bad = !finite_d(x[t]);
        }
        s1 = dd_add(s1, {d, 0.0});
        s2 = dd_add(s2, dd_sqr(d));
        nf += bad;
        v1[e] = s1;
        v2[e] = s2;
        vn[e] = (int)nf;
    }
    const dd o1 = dd_add(block_excl_scan_dd(s1, shh, shl, nullptr), b1[blk]);
    const dd o2 = dd_add(block_excl_scan_dd(s2, shh, shl, nullptr), b2[blk]);
    const long long on = block_excl_scan_i(nf, shc, nullptr) + bnf[blk];
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        const int64_t t = base + e;
        if (t < n) {
            S1[t + 1] = dd_add(o1, v1[e]);
            S2[t + 1] = dd_add(o2, v2[e]);
            NF[t + 1] = (int)(on + vn[e]);
        }
    }
    if (blk == 0 && threadIdx.x == 0) {
        S1[0] = {0.0, 0.0};
        S2[0] = {0.0, 0.0};
        NF[0] = 0;
    }
}

// Pass 4: per-window statistics, flags, recurrence terms and column records.
__device__ void window_stats_body(const double* __restrict__ xc, const dd* __restrict__ S1,
                                  const dd* __restrict__ S2, const int* __restrict__ NF,
                                  const double* __restrict__ scal, int64_t W, int m,
                                  const int64_t* __restrict__ bounds, int n_seg, double* __restrict__ mu,
                                  double* __restrict__ sig, float2* __restrict__ dfdg, float4* __restrict__ col,
                                  uint8_t* __restrict__ flags, unsigned long long* __restrict__ first,
                                  unsigned long long* __restrict__ clear, int64_t i)
{
    if (i >= W) return;
    if (clear) clear[i] = 0ull;  // the join's key for this row
    const double inv_m = 1.0 / (double)m;
    const double gvar = scal[1];
    // window sums of xc and xc^2, then m var = sum xc^2 - (sum xc)^2 / m, all in
    // double-double so the cancellation of the two large terms stays exact
    const dd s1 = dd_sub(S1[i + m], S1[i]);
    const dd s2 = dd_sub(S2[i + m], S2[i]);
    const int nf = NF[i + m] - NF[i];
    const dd mdd = dd_div(s1, (double)m);
    const double mean = mdd.hi + mdd.lo;
    const dd vm = dd_sub(s2, dd_div(dd_square(s1), (double)m));
    double var = (vm.hi + vm.lo) * inv_m;
    if (var < 0) var = 0.0;
    const double sd = sqrt(var);
    uint8_t f = 0;
    if (nf > 0) f |= kFlagBad;
    else if (var <= kFlatRel * gvar) f |= kFlagFlat;
    if (bounds) {
        // segment s with bounds[s] <= i < bounds[s+1]; the window is valid iff i + m <= bounds[s+1]
        int lo = 0, hi = n_seg;  // invariant: bounds[lo] <= i < bounds[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (bounds[mid] <= i) lo = mid;
            else hi = mid;
        }
        if (i + m > bounds[lo + 1]) f |= kFlagInvalid;
    }
    mu[i] = mean;
    sig[i] = sd;
    flags[i] = f;
    float df = 0.f, dg = 0.f;
    if (i + 1 < W) {
        const dd mn = dd_div(dd_sub(S1[i + 1 + m], S1[i + 1]), (double)m);
        const double mean_next = mn.hi + mn.lo;
        const double xa = xc[i], xb = xc[i + m];
        df = (float)(0.5 * (xb - xa));
        dg = (float)((xb - mean_next) + (xa - mean));
    }
    dfdg[i] = make_float2(df, dg);
    const bool usable = f == 0;
    // weight NaN: every score of the window is NaN, which the FP32 engine's
    // maxima drop, so the window never wins a row
    col[i] = make_float4(df, dg, usable ? (float)(1.0 / sd) : __builtin_nanf(""), 0.f);
    if (first) {
        // one atomic per wave: windows ascend with the lane, so the lowest
        // lane of each ballot holds the wave's first valid / flat window
        const bool valid = !(f & (kFlagBad | kFlagInvalid));
        const unsigned long long bv = __ballot(valid), bf = __ballot(valid && (f & kFlagFlat));
        const int lane = (int)__lane_id();
        if (bv && lane == __ffsll((long long)bv) - 1) atomicMin(&first[1], (unsigned long long)i);
        if (bf && lane == __ffsll((long long)bf) - 1) atomicMin(&first[0], (unsigned long long)i);
    }
}

// One series per launch.
__global__ __launch_bounds__(kThreads) void k_block_sums(const double* __restrict__ x, int64_t n,
                                                         double* __restrict__ xc, double* __restrict__ xt,
                                                         int64_t nb16, dd* __restrict__ b1, dd* __restrict__ b2,
                                                         long long* __restrict__ bnf)
{
    block_sums_body(x, n, xc, xt, nb16, b1, b2, bnf, blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_scan_top(dd* __restrict__ b1, dd* __restrict__ b2,
                                                       long long* __restrict__ bnf, int64_t nb, int64_t n,
                                                       double* __restrict__ scal,
                                                       unsigned long long* __restrict__ first)
{
    scan_top_body(b1, b2, bnf, nb, n, scal, first);
}

__global__ __launch_bounds__(kThreads) void k_scan_local(const double* __restrict__ xc, int64_t n,
                                                         const dd* __restrict__ b1, const dd* __restrict__ b2,
                                                         const long long* __restrict__ bnf, dd* __restrict__ S1,
                                                         dd* __restrict__ S2, int* __restrict__ NF,
                                                         const double* __restrict__ x)
{
    scan_local_body(xc, n, b1, b2, bnf, S1, S2, NF, x, blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_window_stats(
    const double* __restrict__ xc, const dd* __restrict__ S1, const dd* __restrict__ S2,
    const int* __restrict__ NF, const double* __restrict__ scal, int64_t W, int m,
    const int64_t* __restrict__ bounds, int n_seg, double* __restrict__ mu, double* __restrict__ sig,
    float2* __restrict__ dfdg, float4* __restrict__ col, uint8_t* __restrict__ flags,
    unsigned long long* __restrict__ first)
{
    window_stats_body(xc, S1, S2, NF, scal, W, m, bounds, n_seg, mu, sig, dfdg, col, flags, first, nullptr,
                      (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

// Many series per launch (a serving batch): each workgroup finds its series
// in the job table by its block number.
struct StatsJobDev {
    const double* x;
    double* xc;
    double* xt;
    int64_t nb16;
    int64_t n, W;
    int32_t m, pad0;
    dd *b1, *b2;
    long long* bnf;
    dd *S1, *S2;
    int* NF;
    double *mu, *sig;
    float2* dfdg;
    float4* col;
    uint8_t* flags;
    double* scal;
    unsigned long long* first;
    unsigned long long* clear;  // keys of the join to clear (W entries)
    const int64_t* bounds;      // segment bounds of a reference series, or NULL
    int64_t n_seg;
    int64_t blk_sum, blk_loc, blk_win;  // first block of this series in each launch's grid
};

// Last job whose first block (field F) is <= b.
// (The result is made wave-uniform explicitly, so that the job's fields are
// scalar loads.)
template <int64_t StatsJobDev::*F>
__device__ inline int find_job(const StatsJobDev* __restrict__ jobs, int njobs, int64_t b)
{
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].*F <= b) lo = mid;
        else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

__global__ __launch_bounds__(kThreads) void k_block_sums_many(const StatsJobDev* __restrict__ jobs, int njobs)
{
    const int jx = find_job<&StatsJobDev::blk_sum>(jobs, njobs, blockIdx.x);
    const StatsJobDev& J = jobs[jx];
    block_sums_body(J.x, J.n, J.xc, J.xt, J.nb16, J.b1, J.b2, J.bnf, (int64_t)blockIdx.x - J.blk_sum);
}

__global__ __launch_bounds__(kThreads) void k_scan_top_many(const StatsJobDev* __restrict__ jobs)
{
    const StatsJobDev& J = jobs[blockIdx.x];
    scan_top_body(J.b1, J.b2, J.bnf, (J.n + kBlockElems - 1) / kBlockElems, J.n, J.scal, J.first);
}

__global__ __launch_bounds__(kThreads) void k_scan_local_many(const StatsJobDev* __restrict__ jobs, int njobs)
{
    const int jx = find_job<&StatsJobDev::blk_loc>(jobs, njobs, blockIdx.x);
    const StatsJobDev& J = jobs[jx];
    scan_local_body(J.xc, J.n, J.b1, J.b2, J.bnf, J.S1, J.S2, J.NF, J.x, (int64_t)blockIdx.x - J.blk_loc);
}

__global__ __launch_bounds__(kThreads) void k_window_stats_many(const StatsJobDev* __restrict__ jobs, int njobs)
{
    const int jx = find_job<&StatsJobDev::blk_win>(jobs, njobs, blockIdx.x);
    const StatsJobDev& J = jobs[jx];
    window_stats_body(J.xc, J.S1, J.S2, J.NF, J.scal, J.W, J.m, J.bounds, (int)J.n_seg, J.mu, J.sig, J.dfdg, J.col,
                      J.flags, J.bounds ? J.first : nullptr, J.clear,
                      ((int64_t)blockIdx.x - J.blk_win) * kThreads + threadIdx.x);
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void k_public_stats(const double* __restrict__ mu_c, const double* __restrict__ sig_in,
                               const uint8_t* __restrict__ fl_in, const double* __restrict__ scal, int64_t W,
                               double* __restrict__ mu, double* __restrict__ sig, uint8_t* __restrict__ fl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= W) return;
    const bool bad = fl_in[i] & kFlagBad;
    mu[i] = bad ? NAN : mu_c[i] + scal[0];
    sig[i] = bad ? NAN : sig_in[i];
    fl[i] = fl_in[i] & (kFlagFlat | kFlagBad);
}

inline int64_t nblocks_of(int64_t n) { return (n + kBlockElems - 1) / kBlockElems; }

}  // namespace

int fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t stream)
{
    if (n <= 0) return ABJ_OK;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)g), dim3(256), 0, stream, p, n, v);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

size_t stats_scratch_bytes(int64_t n, int64_t W)
{
    const int64_t nb = nblocks_of(n + kSeriesPad);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t b = 0;
    b += al(sizeof(double) * (size_t)(n + kSeriesPad));  // xc
    b += al(sizeof(double) * 16 * (size_t)((n + kSeriesPad + 15) / 16));  // xt
    b += al(sizeof(double) * (size_t)W) * 2;             // mu, sig
    b += al(sizeof(float2) * (size_t)W);                 // dfdg
    b += al(sizeof(float4) * (size_t)W);                 // col
    b += al((size_t)W);                                  // flags
    b += al(sizeof(double) * 4);                         // scal
    b += al(sizeof(unsigned long long) * 2);             // first
    // transient: block sums, prefix arrays
    b += al(sizeof(dd) * (size_t)nb) * 2 + al(sizeof(long long) * (size_t)nb);
    b += al(sizeof(dd) * (size_t)(n + 1)) * 2 + al(sizeof(int) * (size_t)(n + 1));
    return b;
}

void stats_carve(Arena& a, int64_t n, int32_t m, SeriesDev* s)
{
    s->n = n;
    s->m = m;
    s->W = n >= m ? n - m + 1 : 0;
    s->xc = a.take<double>((size_t)(n + kSeriesPad));
    s->nb16 = (n + kSeriesPad + 15) / 16;
    s->xt = a.take<double>(16 * (size_t)s->nb16);
    s->mu = a.take<double>((size_t)s->W);
    s->sig = a.take<double>((size_t)s->W);
    s->dfdg = a.take<float2>((size_t)s->W);
    s->col = a.take<float4>((size_t)s->W);
    s->flags = a.take<uint8_t>((size_t)s->W);
    s->scal = a.take<double>(4);
    s->first = a.take<unsigned long long>(2);
}

int stats_compute(const double* x, SeriesDev* s, const int64_t* seg_bounds_dev, int32_t n_seg, Arena& a,
                  hipStream_t stream)
{
    const int64_t n = s->n;
    const int64_t nb = nblocks_of(n);              // blocks holding samples
    const int64_t nbp = nblocks_of(n + kSeriesPad);  // ... and the zero tail
    dd* b1 = a.take<dd>((size_t)nbp);
    dd* b2 = a.take<dd>((size_t)nbp);
    long long* bnf = a.take<long long>((size_t)nbp);
    dd* S1 = a.take<dd>((size_t)(n + 1));
    dd* S2 = a.take<dd>((size_t)(n + 1));
    int* NF = a.take<int>((size_t)(n + 1));

    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nbp), dim3(kThreads), 0, stream, x, n, s->xc, s->xt, s->nb16,
                       b1, b2, bnf);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, stream, b1, b2, bnf, nb, n, s->scal, s->first);
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kThreads), 0, stream, s->xc, n, b1, b2, bnf, S1, S2,
                       NF, x);
    if (s->W > 0) {
        const int64_t g = (s->W + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_window_stats, dim3((unsigned)g), dim3(kThreads), 0, stream, s->xc, S1, S2, NF, s->scal,
                           s->W, (int)s->m, seg_bounds_dev, (int)n_seg, s->mu, s->sig, s->dfdg, s->col, s->flags,
                           seg_bounds_dev ? s->first : nullptr);
    }
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

size_t stats_job_bytes() { return sizeof(StatsJobDev); }

void stats_carve_job(Arena& a, const double* x_dev, int64_t n, int32_t m, SeriesDev* s, unsigned long long* clear,
                     void* job_host, int64_t* blk_sum, int64_t* blk_loc, int64_t* blk_win, const int64_t* bounds_dev,
                     int32_t n_seg)
{
    stats_carve(a, n, m, s);
    StatsJobDev J = {};
    const int64_t nb = nblocks_of(n), nbp = nblocks_of(n + kSeriesPad);
    J.x = x_dev;
    J.xc = s->xc;
    J.xt = s->xt;
    J.nb16 = s->nb16;
    J.n = n;
    J.W = s->W;
    J.m = m;
    J.b1 = a.take<dd>((size_t)nbp);
    J.b2 = a.take<dd>((size_t)nbp);
    J.bnf = a.take<long long>((size_t)nbp);
    J.S1 = a.take<dd>((size_t)(n + 1));
    J.S2 = a.take<dd>((size_t)(n + 1));
    J.NF = a.take<int>((size_t)(n + 1));
    J.mu = s->mu;
    J.sig = s->sig;
    J.dfdg = s->dfdg;
    J.col = s->col;
    J.flags = s->flags;
    J.scal = s->scal;
    J.first = s->first;
    J.clear = clear;
    J.bounds = bounds_dev;
    J.n_seg = bounds_dev ? n_seg : 0;
    J.blk_sum = *blk_sum;
    J.blk_loc = *blk_loc;
    J.blk_win = *blk_win;
    *blk_sum += nbp;
    *blk_loc += nb;
    *blk_win += (s->W + kThreads - 1) / kThreads;
    memcpy(job_host, &J, sizeof(J));
}

int stats_launch_many(const void* jobs_dev, int njobs, int64_t blk_sum, int64_t blk_loc, int64_t blk_win,
                      hipStream_t stream)
{
    if (njobs <= 0) return ABJ_OK;
    const StatsJobDev* J = static_cast<const StatsJobDev*>(jobs_dev);
    hipLaunchKernelGGL(k_block_sums_many, dim3((unsigned)blk_sum), dim3(kThreads), 0, stream, J, njobs);
    hipLaunchKernelGGL(k_scan_top_many, dim3((unsigned)njobs), dim3(kThreads), 0, stream, J);
    hipLaunchKernelGGL(k_scan_local_many, dim3((unsigned)blk_loc), dim3(kThreads), 0, stream, J, njobs);
    if (blk_win > 0)
        hipLaunchKernelGGL(k_window_stats_many, dim3((unsigned)blk_win), dim3(kThreads), 0, stream, J, njobs);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

int stats_export(const SeriesDev& s, double* mu, double* sig, uint8_t* flags, hipStream_t stream)
{
    if (s.W <= 0) return ABJ_OK;
    const int64_t g = (s.W + 255) / 256;
    hipLaunchKernelGGL(k_public_stats, dim3((unsigned)g), dim3(256), 0, stream, s.mu, s.sig, s.flags, s.scal, s.W,
                       mu, sig, flags);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

}  // namespace abj
