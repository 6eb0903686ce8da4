// Row epilogue of the FP32 join: unpack each row's winning column, recompute
// its distance in FP64 from the windows themselves (the norm of the difference
// of the z-normalised windows, one wave per row, so there is no 1 - rho
// cancellation), and apply the flat / non-finite conventions.
#include <math.h>

#include "abj_internal.hpp"

namespace abj {

namespace {

constexpr unsigned long long kNone = ~0ull;

constexpr int kWave = 64;
constexpr int kRowsPerBlock = 4;  // one wave per row

// Pearson correlation of a distance, rho = 1 - d^2 / (2m); no window (+inf)
// becomes -inf, NaN stays NaN.
__device__ inline double pearson_of(double d, int m)
{
    if (isnan(d)) return d;
    if (isinf(d)) return -INFINITY;
    return 1.0 - d * d / (2.0 * (double)m);
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Exact FP64 distance of two non-flat windows given their means and
// deviations: the norm of the difference of the z-normalised windows (no
// 1 - rho cancellation), summed across the wave.
__device__ inline double wave_dist(const double* __restrict__ a, double ma, double sa, const double* __restrict__ b,
                                   double mb, double sb, int m, int lane)
{
    const double ia = 1.0 / sa, ib = 1.0 / sb;
    double acc = 0.0;
    for (int k = lane; k < m; k += kWave) {
        const double e = (a[k] - ma) * ia - (b[k] - mb) * ib;
        acc = fma(e, e, acc);
    }
    return sqrt(wave_sum(acc));
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

__global__ __launch_bounds__(kWave * kRowsPerBlock) void k_finalize(
    const double* __restrict__ axc, const double* __restrict__ amu, const double* __restrict__ asig,
    const uint8_t* __restrict__ aflags, int64_t WA, const double* __restrict__ bxc, const double* __restrict__ bmu,
    const double* __restrict__ bsig, const unsigned long long* __restrict__ bfirst,
    const uint8_t* __restrict__ bflags, int64_t WB, int m, int64_t excl, int pearson,
    const unsigned long long* __restrict__ keys, float* __restrict__ P, int64_t* __restrict__ I,
    double* __restrict__ P64)
{
    const int lane = threadIdx.x % kWave;
    const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
    if (i >= WA) return;  // uniform per wave
    const uint8_t fa = aflags[i];
    double pout = NAN;
    int64_t iout = -1;
    if (!(fa & kFlagBad)) {
        // first valid flat / first valid reference window (outside the row's
        // trivial-match zone in a self-join)
        const unsigned long long ff = WB > 0 ? outside_zone(bfirst[0], bflags, WB, i, excl, true, lane) : kNone;
        if (fa & kFlagFlat) {
            const unsigned long long fv =
                WB > 0 ? outside_zone(bfirst[1], bflags, WB, i, excl, false, lane) : kNone;
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
            const unsigned long long key = keys ? keys[i] : 0ull;
            double d = INFINITY;
            int64_t j = -1;
            if (key != 0ull) {
                j = (int64_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
                d = wave_dist(axc + i, amu[i], asig[i], bxc + j, bmu[j], bsig[j], m, lane);
            }
            if (ff != kNone) {
                const double sm = sqrt((double)m);
                if (sm < d || (sm == d && (int64_t)ff < j)) {
                    d = sm;
                    j = (int64_t)ff;
                }
            }
            pout = d;
            iout = j;
        }
    }
    if (pearson) pout = pearson_of(pout, m);
    if (lane == 0) {
        P[i] = (float)pout;
        I[i] = iout;
        if (P64) P64[i] = pout;
    }
}

}  // namespace

int finalize_launch(const SeriesDev& A, const SeriesDev& B, const unsigned long long* keys, float* P, int64_t* I,
                    hipStream_t stream, double* P64, int64_t excl, bool pearson)
{
    if (A.W <= 0) return ABJ_OK;
    const int64_t g = (A.W + kRowsPerBlock - 1) / kRowsPerBlock;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)g), dim3(kWave * kRowsPerBlock), 0, stream, A.xc, A.mu, A.sig,
                       A.flags, A.W, B.xc, B.mu, B.sig, B.first, B.flags, B.W, (int)A.m, excl, pearson ? 1 : 0, keys, P, I, P64);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

}  // namespace abj
