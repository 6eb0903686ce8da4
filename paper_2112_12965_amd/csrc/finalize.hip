// Row epilogue of the FP32 join: unpack each row's winning group of 16
// columns, pick the column with the largest correlation among them from FP32
// dot products of the centred windows (one wave per 4 rows, 16 lanes per row,
// one lane per candidate column), recompute the winner's distance in FP64
// from the windows themselves (the norm of the difference of the
// z-normalised windows, so there is no 1 - rho cancellation), and apply the
// flat / non-finite conventions.
//
// The samples are staged in LDS as doubles: one span for the wave's four
// overlapping row windows, one span per row for its group's 16 columns.  The
// FP32 dots convert as they read, and a window of up to 256 samples then
// takes its FP64 distance from the same stage, so a wave makes two memory
// round trips: the keys with the row windows, then the groups' spans.  The
// exchanges within a row run on the DPP path rather than through LDS.  For
// windows shorter than kFp32SmallM the key names the best column itself (the
// tile kernel compared FP64 correlations), and only its distance is computed.
#include <math.h>
#include <string.h>

#include "abj_internal.hpp"

namespace abj {

namespace {

constexpr unsigned long long kNone = ~0ull;

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 1;

// Pearson correlation of a distance, rho = 1 - d^2 / (2m); no window (+inf)
// becomes -inf, NaN stays NaN.
__device__ inline double pearson_of(double d, int m)
{
    if (isnan(d)) return d;
    if (isinf(d)) return -INFINITY;
    return 1.0 - d * d / (2.0 * (double)m);
}

constexpr int kGroup = 16;                    // columns per candidate group of the FP32 engine
constexpr int kRowsPerWave = kWave / kGroup;  // 16 lanes per row
constexpr int kKC = 256;                      // window samples staged per pass
constexpr int kSlice = kKC / kGroup;          // samples per lane and pass
static_assert(kSlice == 16, "lane c's slice is samples 16 c .. 16 c + 15");
constexpr int kALen = kKC + kRowsPerWave - 1;  // query samples of the wave's four windows per pass
constexpr int kBLen = kKC + kGroup - 1;        // reference samples of one row's group per pass
// LDS index of a staged double: one pad per 16 keeps the lanes' slices (16
// samples apart) on distinct banks; pad(16 q + v) = 17 q + pad(v).
__host__ __device__ constexpr int pad(int t) { return t + (t >> 4); }
constexpr int kASpan = pad(kALen - 1) + 1;            // 275 doubles
constexpr int kBSpan = pad(kBLen - 1) + 1;            // 287 doubles per row
constexpr int kStage = kASpan + kRowsPerWave * kBSpan;  // doubles per wave (11.4 KB)
constexpr int kAL = (kALen + kWave - 1) / kWave;      // span samples per lane in a pass
constexpr int kBL = (kBLen + kWave - 1) / kWave;

// Lane l's value of v, wave-uniform.
__device__ __forceinline__ int64_t lane_i64(int64_t v, int l)
{
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)((unsigned long long)v >> 32), l);
    return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// First reference window at or after `from` that is valid and, when
// `want_flat`, flat; kNone if there is none.  Wave-wide scan, 64 columns a step.
__device__ inline unsigned long long wave_find(const uint8_t* __restrict__ bflags, int64_t WB, int64_t from,
                                               bool want_flat, int lane)
{
    for (int64_t base = from; base < WB; base += kWave) {
        const int64_t j = base + lane;
        bool ok = false;
        if (j < WB) {
            const uint8_t f = bflags[j];
            ok = !(f & (kFlagBad | kFlagInvalid)) && (!want_flat || (f & kFlagFlat));
        }
        const unsigned long long hit = __ballot(ok);
        if (hit) return (unsigned long long)(base + __ffsll((long long)hit) - 1);
    }
    return kNone;
}

// The first window of the list that lies outside the zone |j - i| <= excl:
// `first` if it does, else the first after the zone.
__device__ inline unsigned long long outside_zone(unsigned long long first, const uint8_t* __restrict__ bflags,
                                                  int64_t WB, int64_t i, int64_t excl, bool want_flat, int lane)
{
    if (first == kNone || excl < 0) return first;
    const int64_t f = (int64_t)first;
    if (f < i - excl || f > i + excl) return first;
    return wave_find(bflags, WB, i + excl + 1, want_flat, lane);
}

// Exchanges within a row of 16 lanes on the DPP path (no LDS round trip):
// quad_perm xor 1 and xor 2, half-row mirror (lane c with 7 - c of its half:
// xor 7) and row rotate by 8 (xor 8).  Each pairs lanes that differ in bit
// 0, 1, 2 and 3 of c respectively, so four steps reach all 16 lanes.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRor8 = 0x128;
template <int kCtrl>
__device__ __forceinline__ unsigned dpp_u32(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xf, 0xf, true);
}
template <int kCtrl>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __uint_as_float(dpp_u32<kCtrl>(__float_as_uint(v)));
}
template <int kCtrl>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v)
{
    return ((unsigned long long)dpp_u32<kCtrl>((unsigned)(v >> 32)) << 32) | dpp_u32<kCtrl>((unsigned)v);
}
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v)
{
    return __longlong_as_double((long long)dpp_u64<kCtrl>((unsigned long long)__double_as_longlong(v)));
}
// The largest key and the sum over the row's 16 lanes, in every lane.
__device__ __forceinline__ unsigned long long row_max_u64(unsigned long long v)
{
    unsigned long long o = dpp_u64<kDppXor1>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppXor2>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppHalfMirror>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppRor8>(v);
    return o > v ? o : v;
}
__device__ __forceinline__ double row_sum_f64(double v)
{
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    return v + dpp_f64<kDppRor8>(v);
}
// One argmax step: take the partner's (score, column) if it is better (ties
// -> the smaller column).
template <int kCtrl>
__device__ __forceinline__ void argmax_step(float& score, int& cb)
{
    const float os = dpp_f32<kCtrl>(score);
    const int oc = (int)dpp_u32<kCtrl>((unsigned)cb);
    if (os > score || (os == score && oc < cb)) {
        score = os;
        cb = oc;
    }
}

__device__ __forceinline__ void finalize_body(
    const double* __restrict__ axc, const double* __restrict__ amu, const double* __restrict__ asig,
    const uint8_t* __restrict__ aflags, int64_t WA, const double* __restrict__ bxc, const double* __restrict__ bmu,
    const double* __restrict__ bsig, const unsigned long long* __restrict__ bfirst,
    const uint8_t* __restrict__ bflags, int64_t WB, int m, int64_t excl, int pearson,
    const unsigned long long* __restrict__ keys, float* __restrict__ P, int64_t* __restrict__ I,
    double* __restrict__ P64, int64_t blk, const unsigned long long* __restrict__ part = nullptr, int nparts = 0)
{
    __shared__ double stage_all[kWavesPerBlock][kStage];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t row0 = (blk * kWavesPerBlock + wave) * kRowsPerWave;
    double* __restrict__ sa = stage_all[wave];            // samples row0 + kc + t, t < kALen
    double* __restrict__ sb = stage_all[wave] + kASpan;   // per row: samples jb + kc + t, t < kBLen

    // ---- lanes 16 r .. 16 r + 15 serve row row0 + r; lane c scores column
    // jb + c of the row's winning group ----
    const int r = lane / kGroup, c = lane % kGroup;
    const int64_t i = row0 + r;
    const int64_t ic = i < WA ? i : WA - 1;  // rows past the end read a valid row and are masked

    // the wave's query span of pass kc (lane l takes samples l, l + 64, ...;
    // rows past the end read the zero tail of the padded copy)
    auto load_rows = [&](int kc, double (&la)[kAL]) {
#pragma unroll
        for (int x = 0; x < kAL; ++x) {
            const int t = lane + x * kWave;
            la[x] = axc[row0 + kc + (t < kALen ? t : kALen - 1)];
        }
    };
    auto store_rows = [&](const double (&la)[kAL]) {
#pragma unroll
        for (int x = 0; x < kAL; ++x)
            if (lane + x * kWave < kALen) sa[pad(lane) + pad(x * kWave)] = la[x];
    };
    // the groups' spans of pass kc (rows without a group read a valid address;
    // their stage is never read)
    auto load_spans = [&](int kc, const int64_t (&jrows)[kRowsPerWave], double (&lb)[kRowsPerWave][kBL]) {
#pragma unroll
        for (int rr = 0; rr < kRowsPerWave; ++rr) {
            const double* __restrict__ br_ = bxc + (jrows[rr] >= 0 ? jrows[rr] : 0) + kc;  // < n + 15: padded
#pragma unroll
            for (int x = 0; x < kBL; ++x) {
                const int t = lane + x * kWave;
                lb[rr][x] = br_[t < kBLen ? t : kBLen - 1];
            }
        }
    };
    auto store_spans = [&](const double (&lb)[kRowsPerWave][kBL]) {
#pragma unroll
        for (int rr = 0; rr < kRowsPerWave; ++rr)
#pragma unroll
            for (int x = 0; x < kBL; ++x)
                if (lane + x * kWave < kBLen) sb[rr * kBSpan + pad(lane) + pad(x * kWave)] = lb[rr][x];
    };
    // Row r's samples 16 c + u (u < 16) sit in the query span at r + 16 c + u,
    // index 17 c + r + u, plus one once r + u reaches 16.
    const double* __restrict__ qa = sa + (kGroup + 1) * c + r;
    auto row_sample = [&](int u) -> double {
        return qa[u + (u >= kGroup - kRowsPerWave + 1 ? (r + u >= kGroup ? 1 : 0) : 0)];
    };

    // ---- first memory round trip: the rows' flags, keys and statistics, and
    // the first pass of their windows, which does not depend on the keys ----
    {
        double la[kAL];
        load_rows(0, la);
        store_rows(la);
    }
    const uint8_t fa = i < WA ? aflags[ic] : (uint8_t)kFlagBad;
    const double mai = amu[ic], sai = asig[ic];
    unsigned long long key = 0ull;
    if (part) {
        // the row's key is the largest of its tiles' keys: lane c takes
        // chunks c, c + 16, ..., then the row's 16 lanes combine
        for (int p = c; p < nparts; p += kGroup) {
            const unsigned long long v = part[(int64_t)p * WA + ic];
            key = v > key ? v : key;
        }
        key = row_max_u64(key);
    } else if (keys) {
        key = keys[ic];
    }
    int64_t jb = -1;
    if (i < WA && key && !(fa & (kFlagBad | kFlagFlat))) jb = (int64_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
    int64_t jrows[kRowsPerWave];  // wave-uniform
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) jrows[rr] = lane_i64(jb, rr * kGroup);
    const bool any = jrows[0] >= 0 || jrows[1] >= 0 || jrows[2] >= 0 || jrows[3] >= 0;

    // ---- second round trip: the candidates' statistics and the groups'
    // spans ----
    const int64_t j = jb + c;
    // windows shorter than kFp32SmallM: the key names the best column itself
    const bool cand = jb >= 0 && j < WB && (excl < 0 || j - i > excl || i - j > excl) && (m >= kFp32SmallM || c == 0);
    const int64_t jc = cand ? j : 0;
    const uint8_t fj = cand ? bflags[jc] : (uint8_t)1;
    const double mbj = bmu[jc], sbj = bsig[jc];
    const double mb0 = bmu[jb >= 0 ? jb : 0];
    if (any) {
        double lb[kRowsPerWave][kBL];
        load_spans(0, jrows, lb);
        store_spans(lb);
    }

    // ---- choosing the column: FP32 dots of the row's window minus its mean
    // with the group's span minus the first candidate's mean (the candidates'
    // means differ by little, and the window minus its mean sums to zero, so
    // the dots are the covariances up to rounding); in each pass lane c dots
    // its 16 samples with the 16 shifted spans through a sliding register
    // window, rounding to FP32 as it reads ----
    const double* __restrict__ qb = sb + r * kBSpan + (kGroup + 1) * c;  // row r's sample 16 c + x at pad(x)
    float acc[kGroup];
#pragma unroll
    for (int v = 0; v < kGroup; ++v) acc[v] = 0.f;
    auto dots = [&](int len) {
        const int n16 = len - kSlice * c;  // samples of the lane's slice inside the window
        if (jb < 0 || n16 <= 0) return;
        float av[kSlice], w[kSlice + kGroup - 1];
#pragma unroll
        for (int u = 0; u < kSlice; ++u) av[u] = u < n16 ? (float)(row_sample(u) - mai) : 0.f;
#pragma unroll
        for (int x = 0; x < kSlice + kGroup - 1; ++x) w[x] = (float)(qb[pad(x)] - mb0);
#pragma unroll
        for (int u = 0; u < kSlice; ++u)
#pragma unroll
            for (int x = 0; x < kGroup; ++x) acc[x] = fmaf(av[u], w[u + x], acc[x]);
    };
    // every wave of the block runs the same passes (m is uniform), so all of
    // them reach the barriers
    __syncthreads();
    dots(m < kKC ? m : kKC);
    for (int kc = kKC; kc < m; kc += kKC) {
        __syncthreads();  // this pass overwrites the stage
        if (any) {
            double la[kAL], lb[kRowsPerWave][kBL];
            load_rows(kc, la);
            load_spans(kc, jrows, lb);
            store_rows(la);
            store_spans(lb);
        }
        __syncthreads();
        dots(m - kc < kKC ? m - kc : kKC);
    }
    // halving exchange within the row's 16 lanes: each step pairs lanes that
    // differ in one bit of c (and perhaps lower ones), the lane with the bit
    // set keeping the upper half of the columns, so that afterwards lane c
    // holds the sum of column c
    float h8[8], h4[4], h2[2], dot;
    {
        const bool hi = c & 8;
#pragma unroll
        for (int x = 0; x < 8; ++x) h8[x] = (hi ? acc[x + 8] : acc[x]) + dpp_f32<kDppRor8>(hi ? acc[x] : acc[x + 8]);
    }
    {
        const bool hi = c & 4;
#pragma unroll
        for (int x = 0; x < 4; ++x)
            h4[x] = (hi ? h8[x + 4] : h8[x]) + dpp_f32<kDppHalfMirror>(hi ? h8[x] : h8[x + 4]);
    }
    {
        const bool hi = c & 2;
#pragma unroll
        for (int x = 0; x < 2; ++x) h2[x] = (hi ? h4[x + 2] : h4[x]) + dpp_f32<kDppXor2>(hi ? h4[x] : h4[x + 2]);
    }
    {
        const bool hi = c & 1;
        dot = (hi ? h2[1] : h2[0]) + dpp_f32<kDppXor1>(hi ? h2[0] : h2[1]);
    }
    // score in FP32 like the dot itself (an approximate reciprocal adds an
    // ulp to the dot's own rounding)
    float score = -INFINITY;
    if (cand && fj == 0) score = dot * __builtin_amdgcn_rcpf((float)sbj);
    // best column of the row, in every lane of the row
    int cb = c;
    argmax_step<kDppXor1>(score, cb);
    argmax_step<kDppXor2>(score, cb);
    argmax_step<kDppHalfMirror>(score, cb);
    argmax_step<kDppRor8>(score, cb);
    const int64_t jbest = score == -INFINITY ? -1 : jb + cb;
    // ---- its exact distance in FP64, the norm of the difference of the
    // z-normalised windows, split over the row's 16 lanes ----
    const double mb = __shfl(mbj, r * kGroup + cb, kWave), sbb = __shfl(sbj, r * kGroup + cb, kWave);
    double sq = 0.0;
    if (jbest >= 0) {
        const double ia = 1.0 / sai, ib = 1.0 / sbb;
        if (m <= kKC) {
            // one pass: both windows are still staged; the winner's sample
            // 16 c + u is the span's cb + 16 c + u
            // (a - mu_a) / sigma_a - (b - mu_b) / sigma_b = a ia - b ib + c0
            const int n16 = m - kSlice * c;
            const double c0 = mb * ib - mai * ia;
            double s2[2] = {0.0, 0.0};
            if (n16 > 0) {
#pragma unroll
                for (int u = 0; u < kSlice; ++u) {
                    const double e = fma(row_sample(u), ia, fma(-qb[cb + u + ((cb + u) >> 4)], ib, c0));
                    if (u < n16) s2[u & 1] = fma(e, e, s2[u & 1]);
                }
            }
            sq = s2[0] + s2[1];
        } else {
            // several passes: the windows from memory, lane c taking samples
            // c, c + 16, ...; four independent sums, eight loads in flight
            double s2[4] = {0.0, 0.0, 0.0, 0.0};
            int k = c;
            for (; k + 7 * kGroup < m; k += 8 * kGroup) {
                double av[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    av[u] = axc[i + k + u * kGroup];
                    bv[u] = bxc[jbest + k + u * kGroup];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double e = (av[u] - mai) * ia - (bv[u] - mb) * ib;
                    s2[u & 3] = fma(e, e, s2[u & 3]);
                }
            }
            for (; k < m; k += kGroup) {
                const double e = (axc[i + k] - mai) * ia - (bxc[jbest + k] - mb) * ib;
                s2[0] = fma(e, e, s2[0]);
            }
            sq = (s2[0] + s2[1]) + (s2[2] + s2[3]);
        }
    }
    sq = row_sum_f64(sq);
    const double dist = jbest >= 0 ? sqrt(sq) : INFINITY;

    // ---- conventions: the flat rows and the flat reference rule ----
    const unsigned long long ff0 = WB > 0 ? bfirst[0] : kNone, fv0 = WB > 0 ? bfirst[1] : kNone;
    if (excl < 0) {
        // AB-join: no zone, so every row's 16 lanes settle their own row
        if (i < WA) {
            double pout = NAN;
            int64_t iout = -1;
            if (!(fa & kFlagBad)) {
                if (fa & kFlagFlat) {
                    if (ff0 != kNone) {
                        pout = 0.0;
                        iout = (int64_t)ff0;
                    } else if (fv0 != kNone) {
                        pout = sqrt((double)m);
                        iout = (int64_t)fv0;
                    } else {
                        pout = INFINITY;
                    }
                } else {
                    double d = dist;
                    int64_t jj = jbest;
                    if (ff0 != kNone) {
                        const double sm = sqrt((double)m);
                        if (sm < d || (sm == d && (int64_t)ff0 < jj)) {
                            d = sm;
                            jj = (int64_t)ff0;
                        }
                    }
                    pout = d;
                    iout = jj;
                }
            }
            if (pearson) pout = pearson_of(pout, m);
            if (c == 0) {
                P[i] = (float)pout;
                I[i] = iout;
                if (P64) P64[i] = pout;
            }
        }
        return;
    }
    // self-join: one row at a time (the zone scans use the whole wave)
    for (int rr = 0; rr < kRowsPerWave; ++rr) {
        const int64_t ii = row0 + rr;
        if (ii >= WA) break;
        const uint8_t fr = (uint8_t)__shfl((int)fa, rr * kGroup, kWave);
        double pout = NAN;
        int64_t iout = -1;
        if (!(fr & kFlagBad)) {
            // first valid flat / first valid reference window (outside the
            // row's trivial-match zone in a self-join)
            const unsigned long long ff = outside_zone(ff0, bflags, WB, ii, excl, true, lane);
            if (fr & kFlagFlat) {
                const unsigned long long fv = outside_zone(fv0, bflags, WB, ii, excl, false, lane);
                if (ff != kNone) {
                    pout = 0.0;
                    iout = (int64_t)ff;
                } else if (fv != kNone) {
                    pout = sqrt((double)m);
                    iout = (int64_t)fv;
                } else {
                    pout = INFINITY;
                }
            } else {
                double d = __shfl(dist, rr * kGroup, kWave);
                int64_t jj = __shfl(jbest, rr * kGroup, kWave);
                if (ff != kNone) {
                    const double sm = sqrt((double)m);
                    if (sm < d || (sm == d && (int64_t)ff < jj)) {
                        d = sm;
                        jj = (int64_t)ff;
                    }
                }
                pout = d;
                iout = jj;
            }
        }
        if (pearson) pout = pearson_of(pout, m);
        if (lane == 0) {
            P[ii] = (float)pout;
            I[ii] = iout;
            if (P64) P64[ii] = pout;
        }
    }
}

__global__ __launch_bounds__(kWave * kWavesPerBlock) void k_finalize(
    const double* __restrict__ axc, const double* __restrict__ amu, const double* __restrict__ asig,
    const uint8_t* __restrict__ aflags, int64_t WA, const double* __restrict__ bxc, const double* __restrict__ bmu,
    const double* __restrict__ bsig, const unsigned long long* __restrict__ bfirst,
    const uint8_t* __restrict__ bflags, int64_t WB, int m, int64_t excl, int pearson,
    const unsigned long long* __restrict__ keys, float* __restrict__ P, int64_t* __restrict__ I,
    double* __restrict__ P64, const unsigned long long* __restrict__ part, int nparts)
{
    finalize_body(axc, amu, asig, aflags, WA, bxc, bmu, bsig, bfirst, bflags, WB, m, excl, pearson, keys, P, I, P64,
                  blockIdx.x, part, nparts);
}

// Many joins per launch (a serving batch); workgroups never mix joins, so the
// barriers inside see one window length.
struct FinJobDev {
    const double *axc, *amu, *asig;
    const uint8_t* aflags;
    int64_t WA;
    const double *bxc, *bmu, *bsig;
    const unsigned long long* bfirst;
    const uint8_t* bflags;
    int64_t WB;
    int32_t m, pearson;
    int64_t excl;
    const unsigned long long* keys;
    float* P;
    int64_t* I;
    double* P64;
    int64_t blk0;
};

__global__ __launch_bounds__(kWave * kWavesPerBlock) void k_finalize_many(
    const FinJobDev* __restrict__ jobs, int njobs)
{
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].blk0 <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid;
    }
    const FinJobDev& J = jobs[__builtin_amdgcn_readfirstlane(lo)];
    finalize_body(J.axc, J.amu, J.asig, J.aflags, J.WA, J.bxc, J.bmu, J.bsig, J.bfirst, J.bflags, J.WB, J.m, J.excl,
                  J.pearson, J.keys, J.P, J.I, J.P64, (int64_t)blockIdx.x - J.blk0);
}

}  // namespace

int finalize_launch(const SeriesDev& A, const SeriesDev& B, const unsigned long long* keys, float* P, int64_t* I,
                    hipStream_t stream, double* P64, int64_t excl, bool pearson, const unsigned long long* part,
                    int nparts)
{
    if (A.W <= 0) return ABJ_OK;
    const int64_t rows_per_block = (int64_t)kWavesPerBlock * kRowsPerWave;
    const int64_t g = (A.W + rows_per_block - 1) / rows_per_block;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)g), dim3(kWave * kWavesPerBlock), 0, stream, A.xc, A.mu, A.sig,
                       A.flags, A.W, B.xc, B.mu, B.sig, B.first, B.flags, B.W, (int)A.m, excl, pearson ? 1 : 0, keys, P,
                       I, P64, part, nparts);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

}  // namespace abj

namespace abj {

size_t finalize_job_bytes() { return sizeof(FinJobDev); }

void finalize_job(const SeriesDev& A, const SeriesDev& B, const unsigned long long* keys, float* P, int64_t* I,
                  void* job_host, int64_t* blk)
{
    FinJobDev J = {};
    J.axc = A.xc;
    J.amu = A.mu;
    J.asig = A.sig;
    J.aflags = A.flags;
    J.WA = A.W;
    J.bxc = B.xc;
    J.bmu = B.mu;
    J.bsig = B.sig;
    J.bfirst = B.first;
    J.bflags = B.flags;
    J.WB = B.W;
    J.m = A.m;
    J.pearson = 0;
    J.excl = -1;
    J.keys = keys;
    J.P = P;
    J.I = I;
    J.P64 = nullptr;
    J.blk0 = *blk;
    const int64_t rows_per_block = (int64_t)kWavesPerBlock * kRowsPerWave;
    *blk += (A.W + rows_per_block - 1) / rows_per_block;
    memcpy(job_host, &J, sizeof(J));
}

int finalize_launch_many(const void* jobs_dev, int njobs, int64_t blocks, hipStream_t stream)
{
    if (njobs <= 0 || blocks <= 0) return ABJ_OK;
    hipLaunchKernelGGL(k_finalize_many, dim3((unsigned)blocks), dim3(kWave * kWavesPerBlock), 0, stream,
                       static_cast<const FinJobDev*>(jobs_dev), njobs);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

}  // namespace abj
