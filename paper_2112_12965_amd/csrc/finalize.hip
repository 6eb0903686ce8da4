// Row epilogue of the FP32 join: unpack each row's winning group of 16
// columns, pick the column with the largest correlation among them from FP32
// dot products of the centred windows staged in LDS (one wave per 4 rows, 16
// lanes per row, one lane per candidate column), recompute the winner's
// distance in FP64 from the windows themselves (the norm of the difference of
// the z-normalised windows, so there is no 1 - rho cancellation), and apply
// the flat / non-finite conventions.
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
constexpr int kHalf = 16;                     // samples per lane and sub-pass (the whole slice)
constexpr int kBLen = kKC + kGroup - 1;       // reference samples of one row's group per pass
// LDS index of a staged sample: one pad word per 16 keeps the lanes'
// slices (16 samples apart) on distinct banks
__device__ __forceinline__ int pad(int t) { return t + (t >> 4); }
constexpr int kAPad = kKC + (kKC >> 4) + 1;
constexpr int kBPad = kBLen + (kBLen >> 4) + 1;
constexpr int kStage = kRowsPerWave * (kAPad + kBPad);  // floats per wave

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

__device__ __forceinline__ void finalize_body(
    const double* __restrict__ axc, const double* __restrict__ amu, const double* __restrict__ asig,
    const uint8_t* __restrict__ aflags, int64_t WA, const double* __restrict__ bxc, const double* __restrict__ bmu,
    const double* __restrict__ bsig, const unsigned long long* __restrict__ bfirst,
    const uint8_t* __restrict__ bflags, int64_t WB, int m, int64_t excl, int pearson,
    const unsigned long long* __restrict__ keys, float* __restrict__ P, int64_t* __restrict__ I,
    double* __restrict__ P64, int64_t blk, const unsigned long long* __restrict__ part = nullptr, int nparts = 0)
{
    __shared__ float stage_all[kWavesPerBlock][kStage];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t row0 = (blk * kWavesPerBlock + wave) * kRowsPerWave;
    float* __restrict__ sa = stage_all[wave];                              // per row: its centred window
    float* __restrict__ sb = stage_all[wave] + kRowsPerWave * kAPad;       // per row: its group's span

    // ---- lanes 16 r .. 16 r + 15 serve row row0 + r; lane c scores column
    // jb + c of the row's winning group ----
    const int r = lane / kGroup, c = lane % kGroup;
    const int64_t i = row0 + r;
    const int64_t ic = i < WA ? i : WA - 1;  // rows past the end read a valid row and are masked
    // flags and key together (one memory round trip)
    const uint8_t fa = i < WA ? aflags[ic] : (uint8_t)kFlagBad;
    unsigned long long key = 0ull;
    if (part) {
        // the row's key is the largest of its tiles' keys: lane c takes
        // chunks c, c + 16, ..., then the row's 16 lanes combine
        for (int p = c; p < nparts; p += kGroup) {
            const unsigned long long v = part[(int64_t)p * WA + ic];
            key = v > key ? v : key;
        }
#pragma unroll
        for (int off = 1; off < kGroup; off <<= 1) {
            const unsigned long long o = __shfl_xor(key, off, kWave);
            key = o > key ? o : key;
        }
    } else if (keys) {
        key = keys[ic];
    }
    int64_t jb = -1;
    if (i < WA && key && !(fa & (kFlagBad | kFlagFlat))) jb = (int64_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
    int64_t jrows[kRowsPerWave];
#pragma unroll
    for (int rr = 0; rr < kRowsPerWave; ++rr) jrows[rr] = __shfl(jb, rr * kGroup, kWave);
    const bool any = jrows[0] >= 0 || jrows[1] >= 0 || jrows[2] >= 0 || jrows[3] >= 0;
    // statistics of the lane's candidate and row (one more round trip, which
    // the first pass's window loads below join)
    const int64_t j = jb + c;
    const bool cand = jb >= 0 && j < WB && (excl < 0 || j - i > excl || i - j > excl);
    const int64_t jc = cand ? j : 0;
    const uint8_t fj = cand ? bflags[jc] : (uint8_t)1;
    const double mbj = bmu[jc], sbj = bsig[jc];
    const double mai = amu[ic], sai = asig[ic];
    const double mb0 = bmu[jb >= 0 ? jb : 0];

    // ---- choosing the column: FP32 dots of the row's window minus its mean
    // with the group's span minus the first candidate's mean (the candidates'
    // means differ by little, and the window minus its mean sums to zero, so
    // the dots are the covariances up to rounding); each pass stages 256
    // samples per row in LDS and lane c dots its 16 with the 16 shifted spans
    // through a sliding register window ----
    float acc[kGroup];
#pragma unroll
    for (int v = 0; v < kGroup; ++v) acc[v] = 0.f;
    // every wave of the block runs the same passes (m is uniform), so all of
    // them reach the barriers
    for (int kc = 0; kc < m; kc += kKC) {
        const int len = m - kc < kKC ? m - kc : kKC;
        if (any) {
            // loads are unconditional (rows without a candidate read a valid
            // address and store zeros) and all issued before the first use, so
            // that they are in flight together
            constexpr int kAL = kKC / kWave, kBL = (kBLen + kWave - 1) / kWave;
            double la[kRowsPerWave][kAL], lb[kRowsPerWave][kBL];
            double mas[kRowsPerWave], mbs[kRowsPerWave];
#pragma unroll
            for (int rr = 0; rr < kRowsPerWave; ++rr) {
                const int64_t jr = jrows[rr];
                const double* __restrict__ ar_ = axc + row0 + rr + kc;        // < n + 260: padded copy
                const double* __restrict__ br_ = bxc + (jr >= 0 ? jr : 0) + kc;  // < n + 15: padded copy
#pragma unroll
                for (int x = 0; x < kAL; ++x) la[rr][x] = ar_[lane + x * kWave];
#pragma unroll
                for (int x = 0; x < kBL; ++x) {
                    const int t = lane + x * kWave;
                    lb[rr][x] = br_[t < kBLen ? t : kBLen - 1];
                }
            }
#pragma unroll
            for (int rr = 0; rr < kRowsPerWave; ++rr) {
                mas[rr] = __shfl(mai, rr * kGroup, kWave);
                mbs[rr] = __shfl(mb0, rr * kGroup, kWave);
            }
#pragma unroll
            for (int rr = 0; rr < kRowsPerWave; ++rr) {
                const bool live = jrows[rr] >= 0;
#pragma unroll
                for (int x = 0; x < kAL; ++x) {
                    const int t = lane + x * kWave;
                    sa[rr * kAPad + pad(t)] = (live && t < len) ? (float)(la[rr][x] - mas[rr]) : 0.f;
                }
#pragma unroll
                for (int x = 0; x < kBL; ++x) {
                    const int t = lane + x * kWave;
                    if (t < kBLen)
                        sb[rr * kBPad + pad(t)] = (live && t < len + kGroup - 1) ? (float)(lb[rr][x] - mbs[rr]) : 0.f;
                }
            }
        }
        __syncthreads();
        if (jb >= 0) {
            const float* __restrict__ ra = sa + r * kAPad;
            const float* __restrict__ rb = sb + r * kBPad;
#pragma unroll
            for (int h = 0; h < kSlice; h += kHalf) {
                const int t0 = c * kSlice + h;
                if (t0 < len) {
                    float av[kHalf], w[kHalf + kGroup - 1];
#pragma unroll
                    for (int u = 0; u < kHalf; ++u) av[u] = ra[pad(t0 + u)];
#pragma unroll
                    for (int x = 0; x < kHalf + kGroup - 1; ++x) w[x] = rb[pad(t0 + x)];
#pragma unroll
                    for (int u = 0; u < kHalf; ++u)
#pragma unroll
                        for (int x = 0; x < kGroup; ++x) acc[x] = fmaf(av[u], w[u + x], acc[x]);
                }
            }
        }
        if (kc + kKC < m) __syncthreads();  // the next pass overwrites the stage
    }
    // halving exchange within the row's 16 lanes: after it lane c holds the
    // sum of column 8 bit3 + 4 bit2 + 2 bit1 + bit0 of c, which is c
    float h8[8], h4[4], h2[2], dot;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const bool hi = c & 8;
        h8[x] = (hi ? acc[x + 8] : acc[x]) + __shfl_xor(hi ? acc[x] : acc[x + 8], 8, kWave);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const bool hi = c & 4;
        h4[x] = (hi ? h8[x + 4] : h8[x]) + __shfl_xor(hi ? h8[x] : h8[x + 4], 4, kWave);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        const bool hi = c & 2;
        h2[x] = (hi ? h4[x + 2] : h4[x]) + __shfl_xor(hi ? h4[x] : h4[x + 2], 2, kWave);
    }
    {
        const bool hi = c & 1;
        dot = (hi ? h2[1] : h2[0]) + __shfl_xor(hi ? h2[0] : h2[1], 1, kWave);
    }
    // score in FP32 like the dot itself (an approximate reciprocal adds an
    // ulp to the dot's own rounding)
    float score = -INFINITY;
    if (cand && fj == 0) score = dot * __builtin_amdgcn_rcpf((float)sbj);
    // best column of the row (ties -> smaller column)
    int cb = c;
#pragma unroll
    for (int off = 1; off < kGroup; off <<= 1) {
        const float os = __shfl_xor(score, off, kWave);
        const int oc = __shfl_xor(cb, off, kWave);
        if (os > score || (os == score && oc < cb)) {
            score = os;
            cb = oc;
        }
    }
    const int64_t jbest = score == -INFINITY ? -1 : jb + cb;
    // its exact distance in FP64, the norm of the difference of the
    // z-normalised windows, split over the row's 16 lanes
    const double mb = __shfl(mbj, r * kGroup + cb, kWave), sbb = __shfl(sbj, r * kGroup + cb, kWave);
    double sq = 0.0;
    if (jbest >= 0) {
        const double ia = 1.0 / sai, ib = 1.0 / sbb;
        double s2[4] = {0.0, 0.0, 0.0, 0.0};
        int k = c;
        // four independent sums, loads of eight samples in flight
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
#pragma unroll
    for (int off = 1; off < kGroup; off <<= 1) sq += __shfl_xor(sq, off, kWave);
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

__global__ __launch_bounds__(kWave * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_finalize(
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

__global__ __launch_bounds__(kWave * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_finalize_many(
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
