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

__global__ __launch_bounds__(kWave * kRowsPerBlock) void k_finalize(
    const double* __restrict__ axc, const double* __restrict__ amu, const double* __restrict__ asig,
    const uint8_t* __restrict__ aflags, int64_t WA, const double* __restrict__ bxc, const double* __restrict__ bmu,
    const double* __restrict__ bsig, const unsigned long long* __restrict__ bfirst, int64_t WB, int m,
    const unsigned long long* __restrict__ keys, float* __restrict__ P, int64_t* __restrict__ I)
{
    const int lane = threadIdx.x % kWave;
    const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
    if (i >= WA) return;  // uniform per wave
    const uint8_t fa = aflags[i];
    const unsigned long long ff = WB > 0 ? bfirst[0] : kNone;  // first valid flat reference window
    const unsigned long long fv = WB > 0 ? bfirst[1] : kNone;  // first valid reference window
    float pout;
    int64_t iout;
    if (fa & kFlagBad) {
        pout = NAN;
        iout = -1;
    } else if (fa & kFlagFlat) {
        if (ff != kNone) {
            pout = 0.f;
            iout = (int64_t)ff;
        } else if (fv != kNone) {
            pout = (float)sqrt((double)m);
            iout = (int64_t)fv;
        } else {
            pout = INFINITY;
            iout = -1;
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
        pout = (float)d;
        iout = j;
    }
    if (lane == 0) {
        P[i] = pout;
        I[i] = iout;
    }
}

}  // namespace

int finalize_launch(const SeriesDev& A, const SeriesDev& B, const unsigned long long* keys, float* P, int64_t* I,
                    hipStream_t stream)
{
    if (A.W <= 0) return ABJ_OK;
    const int64_t g = (A.W + kRowsPerBlock - 1) / kRowsPerBlock;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)g), dim3(kWave * kRowsPerBlock), 0, stream, A.xc, A.mu, A.sig,
                       A.flags, A.W, B.xc, B.mu, B.sig, B.first, B.W, (int)A.m, keys, P, I);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

}  // namespace abj
