// Self-join and the learning phase (Sec. 3.1, Alg. 1).
//
// The self-join reuses the FP32 diagonal engine with a trivial-match zone:
// only tiles that meet the band |j - i| <= excl take the masked sweep.  The
// greedy loop keeps P_B, the running minimum S of the distance profiles of the
// chosen windows, and the exclusion mask in HBM; each step is one fused kernel
// (profile of the previous choice, S update, P' = P_B - S, block minimum) and
// one tie-break kernel, and the host reads back one index.  The e_max stop
// condition (Def. 10) runs the FP32 AB-join of T_B against the current
// dictionary.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "abj_internal.hpp"

namespace abj {

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr unsigned long long kNone = ~0ull;

// Total order of non-NaN doubles as unsigned integers.
__device__ inline unsigned long long ord_key(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ inline unsigned long long wave_min_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}

// Block minimum folded into *out with one atomic per wave.
__device__ inline void fold_min(unsigned long long v, unsigned long long* out)
{
    v = wave_min_u64(v);
    if ((threadIdx.x % kWave) == 0 && v != kNone) atomicMin(out, v);
}

// One greedy step for every window i.  When the previous step chose window
// c (c >= 0):
//   S'(i) = distance of window i to window c (Def. 4, flat conventions)
//   S(i)  = S'(i) on the first update, else min(S(i), S'(i)) (NaN propagates)
//   windows with |i - c| <= excl are excluded from then on.
// Then P'(i) = P_B(i) - S(i) (+inf when excluded or P_B(i) is not finite) is
// stored and its minimum folded into *minkey.
__global__ __launch_bounds__(kBlock) void k_step(const double* __restrict__ xc, const double* __restrict__ mu,
                                                 const double* __restrict__ sig, const uint8_t* __restrict__ flags,
                                                 int64_t W, int m, int64_t c, int first, int64_t excl,
                                                 const double* __restrict__ PB, double* __restrict__ S,
                                                 uint8_t* __restrict__ blocked, double* __restrict__ Pp,
                                                 unsigned long long* __restrict__ minkey)
{
    extern __shared__ double lds[];
    const int64_t i0 = (int64_t)blockIdx.x * kBlock;
    const int64_t i = i0 + threadIdx.x;
    if (c >= 0) {
        double* zw = lds;      // m: window c z-normalised (zero when flat)
        double* xs = lds + m;  // kBlock + m - 1 centred samples from i0 (the copy has a zero tail)
        const bool wflat = flags[c] & kFlagFlat;
        const double mc = mu[c], ic = wflat ? 0.0 : 1.0 / sig[c];
        for (int k = threadIdx.x; k < m; k += kBlock) zw[k] = (xc[c + k] - mc) * ic;
        for (int k = threadIdx.x; k < kBlock + m - 1; k += kBlock) xs[k] = xc[i0 + k];
        __syncthreads();
        if (i < W) {
            const uint8_t f = flags[i];
            double d;
            if (f & kFlagBad) {
                d = NAN;
            } else if ((f & kFlagFlat) || wflat) {
                d = ((f & kFlagFlat) && wflat) ? 0.0 : sqrt((double)m);
            } else {
                const double mi = mu[i], ii = 1.0 / sig[i];
                double acc = 0.0;
                for (int k = 0; k < m; ++k) {
                    const double e = zw[k] - (xs[threadIdx.x + k] - mi) * ii;
                    acc = fma(e, e, acc);
                }
                d = sqrt(acc);
            }
            const double s = S[i];
            S[i] = (first || isnan(s) || isnan(d)) ? (first ? d : NAN) : fmin(s, d);
            if (i - c <= excl && c - i <= excl) blocked[i] = 1;
        }
    }
    unsigned long long key = kNone;
    if (i < W) {
        const double pb = PB[i];
        double p = INFINITY;
        if (!blocked[i] && isfinite(pb)) p = pb - S[i];
        Pp[i] = p;
        if (isfinite(p)) key = ord_key(p);
    }
    fold_min(key, minkey);
}

// Smallest index whose P' has the minimum key.
__global__ __launch_bounds__(kBlock) void k_pick(const double* __restrict__ Pp, int64_t W,
                                                 const unsigned long long* __restrict__ minkey,
                                                 unsigned long long* __restrict__ minidx)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const unsigned long long want = *minkey;
    unsigned long long idx = kNone;
    if (want != kNone && i < W) {
        const double p = Pp[i];
        if (isfinite(p) && ord_key(p) == want) idx = (unsigned long long)i;
    }
    fold_min(idx, minidx);
}

// max over P (NaN if any entry is NaN): out[0] = max bits (distances are >= 0,
// so their bit patterns order as unsigned), out[1] = NaN seen.
__global__ __launch_bounds__(kBlock) void k_max_nan(const double* __restrict__ P, int64_t W,
                                                    unsigned long long* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long v = 0, nan = 0;
    if (i < W) {
        const double p = P[i];
        if (isnan(p))
            nan = 1;
        else
            v = (unsigned long long)__double_as_longlong(p);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
        nan |= __shfl_xor(nan, off, kWave);
    }
    if ((threadIdx.x % kWave) == 0) {
        if (v) atomicMax(&out[0], v);
        if (nan) atomicOr(&out[1], nan);
    }
}

// dict[k] = T[start of its segment + offset]: the concatenation of the
// segments [starts[s], starts[s] + bounds[s+1] - bounds[s]).
__global__ __launch_bounds__(kBlock) void k_gather(const double* __restrict__ T, const int64_t* __restrict__ starts,
                                                   const int64_t* __restrict__ bounds, int nseg, int64_t nd,
                                                   double* __restrict__ dict)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nd) return;
    int lo = 0, hi = nseg - 1;  // last s with bounds[s] <= k
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (bounds[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    dict[k] = T[starts[lo] + (k - bounds[lo])];
}

unsigned grid_of(int64_t W) { return (unsigned)((W + kBlock - 1) / kBlock); }

struct Seg {
    int64_t a, b;
};

// Element of chosen window j: ceil(k m) samples (at least m, at most n)
// centred on the window and clipped to the series.
Seg element_of(int64_t j, int64_t n, int32_t m, double k)
{
    const int64_t L = std::min<int64_t>(n, std::max<int64_t>(m, (int64_t)ceil(k * (double)m)));
    int64_t c0 = j - (L - m) / 2;
    c0 = std::min(std::max<int64_t>(c0, 0), n - L);
    return {c0, c0 + L};
}

// Elements that overlap or touch merge; result sorted by start.
std::vector<Seg> merge_elements(std::vector<Seg> e)
{
    std::sort(e.begin(), e.end(), [](const Seg& x, const Seg& y) { return x.a < y.a || (x.a == y.a && x.b < y.b); });
    std::vector<Seg> out;
    for (const Seg& s : e) {
        if (!out.empty() && s.a <= out.back().b)
            out.back().b = std::max(out.back().b, s.b);
        else
            out.push_back(s);
    }
    return out;
}

// Self-join of the statistics T (computed with the one-segment bounds) into
// keys -> P / I / P64.
int self_join_launch(const SeriesDev& T, int64_t excl, unsigned long long* keys, Fp32Slot* dslot,
                     unsigned long long* counter, float* P, int64_t* I, double* P64, hipStream_t stream,
                     bool pearson = false)
{
    ABJ_TRY(fill_u64(keys, T.W, 0ull, stream));
    Fp32Slot sl;
    fp32_slot(T, T, keys, 0, &sl);
    sl.excl = excl;
    ABJ_HIP(hipMemcpyAsync(dslot, &sl, sizeof(sl), hipMemcpyHostToDevice, stream));
    ABJ_TRY(join_fp32_batch(dslot, 1, fp32_slot_tiles(sl), T.m, T.chunk_w, sl.pairs, counter, stream, true));
    return finalize_launch(T, T, keys, P, I, stream, P64, excl, pearson);
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

int check_self_args(const double* x, int64_t n, int32_t m, const abj_opts* opts)
{
    abj_opts o;
    ABJ_TRY(check_opts(opts, &o));
    if (o.tier != ABJ_TIER_FP32) return set_error(ABJ_EINVAL, "the self-join runs the FP32 tier only");
    if (m < 2 || m > kMaxM) return set_error(ABJ_EINVAL, "m must be in [2, %d] (got %d)", kMaxM, m);
    if (n < m || n > kMaxN) return set_error(ABJ_EINVAL, "n must be in [m, 2^31-1] (got %lld)", (long long)n);
    return check_dev_buf(x, sizeof(double) * (size_t)n, "series");
}

// Statistics of one series as a one-segment reference (so that flat-window
// lookups work for the self-join), carved from `ar`.
int series_stats(const double* x, int64_t n, int32_t m, Arena& ar, SeriesDev* T, hipStream_t stream)
{
    stats_carve(ar, n, m, T);
    // the chunk width of a join of the series with itself (fp32_wide_chunks)
    const int64_t W = n - m + 1;
    const bool wide = fp32_wide_chunks(W, (int64_t)fp32_chunk_list(nullptr, 0, n, m).size() / 2);
    ABJ_TRY(fp32_chunks_upload(nullptr, 0, n, m, ar, T, stream, nullptr, wide ? 0 : kFp32NarrowChunk));
    T->nvalid = T->W;
    int64_t* db = ar.take<int64_t>(2);
    const int64_t hb[2] = {0, n};
    ABJ_HIP(hipMemcpyAsync(db, hb, sizeof(hb), hipMemcpyHostToDevice, stream));
    return stats_compute(x, T, db, 1, ar, stream);
}

size_t series_stats_bytes(int64_t n, int64_t W)
{
    return stats_scratch_bytes(n, W) + al256(2 * sizeof(int64_t)) + fp32_chunk_bytes(0, n, kFp32NarrowChunk);
}

// State of one dict_build call.
struct Learner {
    hipStream_t stream;
    const double* T;  // device training series
    int64_t n, W;
    int32_t m;
    SeriesDev ts;            // statistics of T_B
    unsigned long long* keys;
    Fp32Slot* slot;
    unsigned long long* counter;
    float* P;                // FP32 profile scratch (self-join, then e_max joins)
    int64_t* I;
    double* P64;             // scratch FP64 profile of the e_max joins
    double* PB;              // P_B
    double* S;
    double* Pp;
    uint8_t* blocked;
    unsigned long long* red; // [0] min key, [1] min index, [2] max bits, [3] NaN seen
    double* dict;            // n: dictionary samples
    int64_t* dstarts;        // segment starts in T and bounds in the dictionary
    int64_t* dbounds;
    int64_t max_dseg;
    void* dict_ws;           // workspace of the dictionary statistics
    size_t dict_ws_bytes;
    unsigned long long* host;  // pinned: 4 words read back per step
    int64_t* host_seg;         // pinned: 2 * max_dseg + 1 words
};

// Def. 10: max over the windows of T_B of the AB-join distance to the
// dictionary made of `segs`; +inf for an empty dictionary.
int e_max_of(Learner& L, const std::vector<Seg>& segs, double* out)
{
    int64_t nd = 0;
    for (const Seg& s : segs) nd += s.b - s.a;
    if (nd < L.m) {
        *out = INFINITY;
        return ABJ_OK;
    }
    const int nseg = (int)segs.size();
    if (nseg > L.max_dseg) return set_error(ABJ_EINVAL, "internal: %d dictionary segments exceed %lld", nseg,
                                            (long long)L.max_dseg);
    // bounds (nseg + 1) then starts (nseg) through one pinned staging copy
    int64_t* hb = L.host_seg;
    hb[0] = 0;
    for (int s = 0; s < nseg; ++s) {
        hb[s + 1] = hb[s] + (segs[s].b - segs[s].a);
        hb[nseg + 1 + s] = segs[s].a;
    }
    ABJ_HIP(hipMemcpyAsync(L.dbounds, hb, sizeof(int64_t) * (size_t)(2 * nseg + 1), hipMemcpyHostToDevice,
                           L.stream));
    const int64_t* dstarts = L.dbounds + nseg + 1;
    hipLaunchKernelGGL(k_gather, dim3(grid_of(nd)), dim3(kBlock), 0, L.stream, L.T, dstarts, L.dbounds, nseg, nd,
                       L.dict);
    ABJ_HIP(hipGetLastError());
    Arena ar(L.dict_ws, L.dict_ws_bytes);
    SeriesDev B;
    stats_carve(ar, nd, L.m, &B);
    ABJ_TRY(fp32_chunks_upload(hb, nseg, nd, L.m, ar, &B, L.stream));
    for (const Seg& s : segs)
        if (s.b - s.a >= L.m) B.nvalid += s.b - s.a - L.m + 1;
    ABJ_TRY(stats_compute(L.dict, &B, L.dbounds, nseg, ar, L.stream));
    ABJ_TRY(fill_u64(L.keys, L.W, 0ull, L.stream));
    Fp32Slot sl;
    fp32_slot(L.ts, B, L.keys, 0, &sl);
    ABJ_HIP(hipMemcpyAsync(L.slot, &sl, sizeof(sl), hipMemcpyHostToDevice, L.stream));
    ABJ_TRY(join_fp32_batch(L.slot, 1, fp32_slot_tiles(sl), L.m, B.chunk_w, sl.pairs, L.counter, L.stream));
    ABJ_TRY(finalize_launch(L.ts, B, L.keys, L.P, L.I, L.stream, L.P64));
    ABJ_TRY(fill_u64(L.red + 2, 2, 0ull, L.stream));
    hipLaunchKernelGGL(k_max_nan, dim3(grid_of(L.W)), dim3(kBlock), 0, L.stream, L.P64, L.W, L.red + 2);
    ABJ_HIP(hipGetLastError());
    ABJ_HIP(hipMemcpyAsync(L.host + 2, L.red + 2, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           L.stream));
    ABJ_HIP(hipStreamSynchronize(L.stream));
    if (L.host[3])
        *out = NAN;
    else {
        const unsigned long long bits = L.host[2];
        double v;
        memcpy(&v, &bits, sizeof(v));
        *out = v;
    }
    return ABJ_OK;
}

struct PinnedHost {
    void* p = nullptr;
    ~PinnedHost()
    {
        if (p) (void)hipHostFree(p);
    }
};

}  // namespace

}  // namespace abj

using namespace abj;

extern "C" int self_join(const double* x, int64_t n, int32_t m, int64_t excl, float* P, int64_t* I, double* P64,
                         const abj_opts* opts, void* hip_stream)
{
    ABJ_TRY(check_self_args(x, n, m, opts));
    const int64_t W = n - m + 1;
    if (excl < 0) excl = m / 2;
    if (excl >= W) return set_error(ABJ_EINVAL, "excl must be < n-m+1 (got %lld)", (long long)excl);
    ABJ_TRY(check_dev_buf(P, sizeof(float) * (size_t)W, "P"));
    ABJ_TRY(check_dev_buf(I, sizeof(int64_t) * (size_t)W, "I"));
    if (P64) ABJ_TRY(check_dev_buf(P64, sizeof(double) * (size_t)W, "P64"));
    ABJ_TRY(ensure_device());
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Arena ar(stream);
    ar.reserve(series_stats_bytes(n, W));
    ar.reserve(sizeof(unsigned long long) * (size_t)W);
    ar.reserve(sizeof(Fp32Slot));
    ar.reserve(kTileCounterBytes);
    ABJ_TRY(ar.commit());
    SeriesDev T;
    ABJ_TRY(series_stats(x, n, m, ar, &T, stream));
    unsigned long long* keys = ar.take<unsigned long long>((size_t)W);
    Fp32Slot* dslot = ar.take<Fp32Slot>(1);
    unsigned long long* counter = ar.take<unsigned long long>(kTileCounterBytes / 8);
    const bool pearson = opts && (opts->flags & ABJ_FLAG_PEARSON);
    return self_join_launch(T, excl, keys, dslot, counter, P, I, P64, stream, pearson);
}

extern "C" int dict_build(const double* series, int64_t n, int32_t m, const abj_learn_opts* opts,
                          int64_t* segments, int32_t max_segments, int32_t* n_segments, int64_t* chosen,
                          int32_t max_chosen, int32_t* n_chosen, double* dict_out, int64_t* n_dict, double* e_max,
                          double* p_self, void* hip_stream)
{
    // ---- validation ----
    // sizing call: no segments, chosen or dict_out buffer; nothing runs
    const bool sizing = !segments && !chosen && !dict_out;
    if (sizing) {
        if (m < 2 || m > kMaxM) return set_error(ABJ_EINVAL, "m must be in [2, %d] (got %d)", kMaxM, m);
        if (n < m || n > kMaxN) return set_error(ABJ_EINVAL, "n must be in [m, 2^31-1] (got %lld)", (long long)n);
    } else {
        ABJ_TRY(check_self_args(series, n, m, nullptr));
    }
    if (!opts) return set_error(ABJ_EINVAL, "opts is NULL");
    const abj_learn_opts o = *opts;
    if (!(o.context > 0.0) || !isfinite(o.context)) return set_error(ABJ_EINVAL, "context must be finite and > 0");
    if (o.stop == ABJ_STOP_SPACE_SAVING) {
        if (!(o.stop_value >= 0.0 && o.stop_value <= 1.0))
            return set_error(ABJ_EINVAL, "space saving must be in [0, 1]");
    } else if (o.stop == ABJ_STOP_EMAX) {
        if (!(o.stop_value >= 0.0) || !isfinite(o.stop_value))
            return set_error(ABJ_EINVAL, "e_max target must be finite and >= 0");
    } else {
        return set_error(ABJ_EINVAL, "unknown stop condition %d", o.stop);
    }
    if (o.max_iters < 0) return set_error(ABJ_EINVAL, "max_iters must be >= 0");
    if (sizing) {
        // upper bounds that hold for every run: chosen windows are more than
        // m/2 (rounded down) apart, merged segments hold at least
        // ceil(context m) samples (at least m, at most n) and do not touch
        const int64_t W = n - m + 1;
        const int64_t Lmin = std::max<int64_t>(m, std::min<int64_t>(n, (int64_t)ceil(o.context * (double)m)));
        int64_t most_chosen = (W + m / 2) / (m / 2 + 1);
        if (o.max_iters > 0) most_chosen = std::min<int64_t>(most_chosen, o.max_iters);
        const int64_t most_segs = std::min<int64_t>(n / (Lmin + 1) + 1, most_chosen);
        if (!n_segments && !n_chosen && !n_dict)
            return set_error(ABJ_EINVAL, "a sizing call needs n_segments, n_chosen or n_dict");
        if (n_segments) *n_segments = (int32_t)std::min<int64_t>(most_segs, INT32_MAX);
        if (n_chosen) *n_chosen = (int32_t)std::min<int64_t>(most_chosen, INT32_MAX);
        if (n_dict) *n_dict = n;
        return ABJ_OK;
    }
    if (!segments || !n_segments || max_segments < 0)
        return set_error(ABJ_EINVAL, "segments / n_segments are required");
    if (chosen && max_chosen < 0) return set_error(ABJ_EINVAL, "max_chosen must be >= 0");
    if (dict_out && !n_dict) return set_error(ABJ_EINVAL, "n_dict is required with dict_out");
    const int64_t W = n - m + 1;
    if (dict_out) ABJ_TRY(check_dev_buf(dict_out, sizeof(double) * (size_t)n, "dict_out"));
    if (p_self) ABJ_TRY(check_dev_buf(p_self, sizeof(double) * (size_t)W, "p_self"));
    ABJ_TRY(ensure_device());

    // ---- workspace ----
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Learner L;
    L.stream = stream;
    L.T = series;
    L.n = n;
    L.W = W;
    L.m = m;
    const int64_t Lmin = std::max<int64_t>(m, std::min<int64_t>(n, (int64_t)ceil(o.context * (double)m)));
    L.max_dseg = n / (Lmin + 1) + 1;  // merged segments are disjoint and do not touch
    const int32_t most_seg = (int32_t)std::min<int64_t>(L.max_dseg, INT32_MAX);
    L.dict_ws_bytes = stats_scratch_bytes(n, W) + fp32_chunk_bytes(most_seg, n) + 256;
    Arena ar(stream);
    ar.reserve(series_stats_bytes(n, W));
    ar.reserve(sizeof(unsigned long long) * (size_t)W);  // keys
    ar.reserve(sizeof(Fp32Slot));
    ar.reserve(kTileCounterBytes);                        // tile counters
    ar.reserve(sizeof(float) * (size_t)W);                // P
    ar.reserve(sizeof(int64_t) * (size_t)W);              // I
    ar.reserve(sizeof(double) * (size_t)W);               // P64
    ar.reserve(sizeof(double) * (size_t)W);               // P_B
    ar.reserve(sizeof(double) * (size_t)W);               // S
    ar.reserve(sizeof(double) * (size_t)W);               // P'
    ar.reserve((size_t)W);                                // blocked
    ar.reserve(4 * sizeof(unsigned long long));           // reductions
    ar.reserve(sizeof(double) * (size_t)n);               // dictionary
    ar.reserve(sizeof(int64_t) * (size_t)(2 * L.max_dseg + 1));
    ar.reserve(L.dict_ws_bytes);
    ABJ_TRY(ar.commit());
    PinnedHost pin;
    {
        hipError_t e = hipHostMalloc(&pin.p, sizeof(int64_t) * (size_t)(2 * L.max_dseg + 1 + 4), 0);
        if (e != hipSuccess) {
            pin.p = nullptr;
            (void)hipGetLastError();
            return set_error(ABJ_ENOMEM, "pinned staging: %s", hipGetErrorString(e));
        }
    }
    L.host = static_cast<unsigned long long*>(pin.p);
    L.host_seg = reinterpret_cast<int64_t*>(L.host + 4);
    ABJ_TRY(series_stats(series, n, m, ar, &L.ts, stream));
    L.keys = ar.take<unsigned long long>((size_t)W);
    L.slot = ar.take<Fp32Slot>(1);
    L.counter = ar.take<unsigned long long>(kTileCounterBytes / 8);
    L.P = ar.take<float>((size_t)W);
    L.I = ar.take<int64_t>((size_t)W);
    L.P64 = ar.take<double>((size_t)W);
    L.PB = ar.take<double>((size_t)W);
    L.S = ar.take<double>((size_t)W);
    L.Pp = ar.take<double>((size_t)W);
    L.blocked = ar.take<uint8_t>((size_t)W);
    L.red = ar.take<unsigned long long>(4);
    L.dict = ar.take<double>((size_t)n);
    L.dbounds = ar.take<int64_t>((size_t)(2 * L.max_dseg + 1));
    L.dict_ws = ar.take<char>(L.dict_ws_bytes);

    // ---- P_B: self-join of T_B with the m/2 zone (Alg. 1) ----
    const int64_t excl = m / 2;
    ABJ_TRY(self_join_launch(L.ts, excl, L.keys, L.slot, L.counter, L.P, L.I, L.PB, stream));
    ABJ_HIP(hipMemsetAsync(L.S, 0, sizeof(double) * (size_t)W, stream));
    ABJ_HIP(hipMemsetAsync(L.blocked, 0, (size_t)W, stream));

    // ---- greedy loop ----
    const int64_t cap = o.max_iters > 0 ? std::min<int64_t>(o.max_iters, W) : W;
    std::vector<int64_t> picks;
    std::vector<Seg> elements, segs;
    int64_t prev = -1;
    const size_t lds = sizeof(double) * (size_t)(kBlock + 2 * m - 1);
    for (int64_t it = 0; it < cap; ++it) {
        ABJ_TRY(fill_u64(L.red, 2, kNone, stream));
        hipLaunchKernelGGL(k_step, dim3(grid_of(W)), dim3(kBlock), prev >= 0 ? lds : 0, stream, L.ts.xc, L.ts.mu,
                           L.ts.sig, L.ts.flags, W, m, prev, it == 1 ? 1 : 0, excl, L.PB, L.S, L.blocked, L.Pp,
                           L.red);
        ABJ_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_pick, dim3(grid_of(W)), dim3(kBlock), 0, stream, L.Pp, W, L.red, L.red + 1);
        ABJ_HIP(hipGetLastError());
        ABJ_HIP(hipMemcpyAsync(L.host, L.red, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
        ABJ_HIP(hipStreamSynchronize(stream));
        if (L.host[1] == kNone) break;  // every P' is +inf
        const int64_t j = (int64_t)L.host[1];
        picks.push_back(j);
        elements.push_back(element_of(j, n, m, o.context));
        segs = merge_elements(elements);
        int64_t size = 0;
        for (const Seg& s : segs) size += s.b - s.a;
        if (o.stop == ABJ_STOP_SPACE_SAVING && (double)size >= (1.0 - o.stop_value) * (double)n) break;
        if (o.stop == ABJ_STOP_EMAX) {
            double e = 0.0;
            ABJ_TRY(e_max_of(L, segs, &e));
            if (e <= o.stop_value) break;
        }
        prev = j;
    }

    // ---- outputs ----
    if ((int64_t)segs.size() > max_segments)
        return set_error(ABJ_EINVAL, "%zu segments exceed max_segments = %d", segs.size(), max_segments);
    if (chosen && (int64_t)picks.size() > max_chosen)
        return set_error(ABJ_EINVAL, "%zu choices exceed max_chosen = %d", picks.size(), max_chosen);
    double em = INFINITY;
    if (e_max || dict_out) ABJ_TRY(e_max_of(L, segs, &em));  // also leaves the dictionary in L.dict
    int64_t nd = 0;
    for (size_t s = 0; s < segs.size(); ++s) {
        segments[2 * s] = segs[s].a;
        segments[2 * s + 1] = segs[s].b;
        nd += segs[s].b - segs[s].a;
    }
    *n_segments = (int32_t)segs.size();
    if (chosen) std::copy(picks.begin(), picks.end(), chosen);
    if (n_chosen) *n_chosen = (int32_t)picks.size();
    if (e_max) *e_max = em;
    if (dict_out) {
        *n_dict = nd;
        if (nd > 0) {
            if (nd < m) {
                // e_max_of skips dictionaries shorter than m; gather them here
                int64_t off = 0;
                for (const Seg& s : segs) {
                    ABJ_HIP(hipMemcpyAsync(dict_out + off, series + s.a, sizeof(double) * (size_t)(s.b - s.a),
                                           hipMemcpyDeviceToDevice, stream));
                    off += s.b - s.a;
                }
            } else {
                ABJ_HIP(hipMemcpyAsync(dict_out, L.dict, sizeof(double) * (size_t)nd, hipMemcpyDeviceToDevice,
                                       stream));
            }
        }
    }
    if (p_self) ABJ_HIP(hipMemcpyAsync(p_self, L.PB, sizeof(double) * (size_t)W, hipMemcpyDeviceToDevice, stream));
    ABJ_HIP(hipStreamSynchronize(stream));
    return ABJ_OK;
}
