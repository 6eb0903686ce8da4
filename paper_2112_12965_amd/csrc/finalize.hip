// Row epilogue of the FP32 join: unpack each row's winning column, recompute
// its distance exactly in FP64 (two-pass window mean and deviation, direct
// norm of the difference of the z-normalised windows, so no 1 - rho
// cancellation), and apply the flat / non-finite conventions.
#include <math.h>

#include "abj_internal.hpp"

namespace abj {

namespace {

constexpr unsigned long long kNone = ~0ull;

__device__ inline double exact_dist(const double* __restrict__ a, const double* __restrict__ b, int m)
{
    double ma = 0.0, mb = 0.0;
    for (int k = 0; k < m; ++k) {
        ma += a[k];
        mb += b[k];
    }
    ma /= m;
    mb /= m;
    double va = 0.0, vb = 0.0;
    for (int k = 0; k < m; ++k) {
        const double da = a[k] - ma, db = b[k] - mb;
        va = fma(da, da, va);
        vb = fma(db, db, vb);
    }
    if (va == 0.0 && vb == 0.0) return 0.0;
    if (va == 0.0 || vb == 0.0) return sqrt((double)m);
    const double ia = 1.0 / sqrt(va / m), ib = 1.0 / sqrt(vb / m);
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
        const double e = (a[k] - ma) * ia - (b[k] - mb) * ib;
        acc = fma(e, e, acc);
    }
    return sqrt(acc);
}

__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ axc, const uint8_t* __restrict__ aflags,
                                                  int64_t WA, const double* __restrict__ bxc,
                                                  const unsigned long long* __restrict__ bfirst, int64_t WB, int m,
                                                  const unsigned long long* __restrict__ keys, float* __restrict__ P,
                                                  int64_t* __restrict__ I)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= WA) return;
    const uint8_t fa = aflags[i];
    const unsigned long long ff = WB > 0 ? bfirst[0] : kNone;  // first valid flat reference window
    const unsigned long long fv = WB > 0 ? bfirst[1] : kNone;  // first valid reference window
    if (fa & kFlagBad) {
        P[i] = NAN;
        I[i] = -1;
        return;
    }
    if (fa & kFlagFlat) {
        if (ff != kNone) {
            P[i] = 0.f;
            I[i] = (int64_t)ff;
        } else if (fv != kNone) {
            P[i] = (float)sqrt((double)m);
            I[i] = (int64_t)fv;
        } else {
            P[i] = INFINITY;
            I[i] = -1;
        }
        return;
    }
    const unsigned long long key = keys ? keys[i] : 0ull;
    double d = INFINITY;
    int64_t j = -1;
    if (key != 0ull) {
        j = (int64_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
        d = exact_dist(axc + i, bxc + j, m);
    }
    if (ff != kNone) {
        const double sm = sqrt((double)m);
        if (sm < d || (sm == d && (int64_t)ff < j)) {
            d = sm;
            j = (int64_t)ff;
        }
    }
    P[i] = (float)d;
    I[i] = j;
}

}  // namespace

int finalize_launch(const SeriesDev& A, const SeriesDev& B, const unsigned long long* keys, float* P, int64_t* I,
                    hipStream_t stream)
{
    if (A.W <= 0) return ABJ_OK;
    const int64_t g = (A.W + 255) / 256;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)g), dim3(256), 0, stream, A.xc, A.flags, A.W, B.xc, B.first, B.W,
                       (int)A.m, keys, P, I);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

}  // namespace abj
