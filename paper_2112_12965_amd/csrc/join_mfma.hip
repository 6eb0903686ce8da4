// Precision tier of the AB-join: BF16 / FP16 matrix-core window products with
// FP32 accumulation, per-row top-K candidates, FP64 re-check of the candidates.
//
// With z(i)[k] = (x[i+k] - mu(i)) / (sigma(i) sqrt(m)) every window has unit
// norm, so rho(i, j) = z_a(i) . z_b(j) and the nearest neighbour of row i is the
// column with the largest dot product.  Centring and scaling happen in FP64
// before the cast, so the 16-bit operands only carry the shape of the window.
// The dot products are a dense contraction over k = 0..m-1: v_mfma_f32_32x32x16
// tiles, dictionary windows on the M side and query windows on the N side, so
// that each lane's 16 accumulators belong to ONE query window (D row
// 8 (v/4) + 4 (lane/32) + v%4, column lane%32) and the row reduction needs no
// cross-lane traffic until the very end.
//
// Operands are stored pre-swizzled in MFMA fragment order: for each block of
// 32 windows and each 16-wide k step, lane l's 8 elements (window l%32,
// k = 16 ks + 8 (l/32) + e) are 16 contiguous bytes, so a wave loads a whole
// fragment with one coalesced 1 KB access.  Dictionary windows that are
// masked (segment break), flat or non-finite are zero rows and a 0 bit in the
// block's 32-bit validity mask; fully masked blocks are skipped.
#include <math.h>

#include "abj_internal.hpp"

namespace abj {

namespace {

constexpr int kWave = 64;
// waves per workgroup (they share each staged dictionary block): 8 where the
// query fragments are small (m <= 128), 4 for m <= 256
__host__ __device__ constexpr int waves_per_block(int ks) { return ks <= 8 ? 8 : 4; }

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

template <typename T>
struct Vec8;
template <>
struct Vec8<__bf16> {
    using type = bf16x8;
};
template <>
struct Vec8<_Float16> {
    using type = f16x8;
};

__device__ inline f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x16 mfma(f16x8 a, f16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// One thread per (32-window block, k step, lane) fragment of 8 elements.
template <typename T>
__global__ __launch_bounds__(256) void k_make_operand(const double* __restrict__ xc, const double* __restrict__ mu,
                                                      const double* __restrict__ sig,
                                                      const uint8_t* __restrict__ flags, int64_t W, int m, int ks_n,
                                                      int64_t nfrag, typename Vec8<T>::type* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nfrag) return;
    const int lane = (int)(t % kWave);
    const int64_t bk = t / kWave;  // block * ks_n + ks
    const int ks = (int)(bk % ks_n);
    const int64_t blk = bk / ks_n;
    const int64_t i = blk * 32 + (lane % 32);
    const int k0 = ks * 16 + 8 * (lane / 32);
    typename Vec8<T>::type v;
    const bool use = i < W && flags[i] == 0;
    const double mean = use ? mu[i] : 0.0;
    const double scale = use ? 1.0 / (sig[i] * sqrt((double)m)) : 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        const double z = (use && k < m) ? (xc[i + k] - mean) * scale : 0.0;
        v[e] = (T)(float)z;
    }
    out[t] = v;
}

// Validity mask of each 32-window dictionary block (bit r = window 32 b + r usable).
__global__ __launch_bounds__(256) void k_block_mask(const uint8_t* __restrict__ flags, int64_t W, int64_t nblk,
                                                    uint32_t* __restrict__ mask)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    uint32_t msk = 0;
    for (int r = 0; r < 32; ++r) {
        const int64_t i = b * 32 + r;
        if (i < W && flags[i] == 0) msk |= 1u << r;
    }
    mask[b] = msk;
}

__device__ inline unsigned long long pack_key(float s, int j)
{
    unsigned u = __float_as_uint(s);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)j);
}

__device__ inline float unpack_score(unsigned long long key)
{
    unsigned u = (unsigned)(key >> 32);
    u = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    return __uint_as_float(u);
}

// (v, j) ranks before (w, k): larger score first, smaller index on ties.
__device__ inline bool ranks_before(float v, int j, float w, int k) { return v > w || (v == w && j >= 0 && j < k); }

// Candidates of one row are kept pairwise more than kRefineRadius windows
// apart, and the FP64 re-check evaluates every window within that radius of
// each one: neighbouring windows have nearly equal 16-bit scores, so without
// the spacing the K candidates would mostly be one neighbourhood, and the
// re-check of the neighbourhood recovers a best window that the 16-bit
// ranking placed just behind its neighbour.
constexpr int kRefineRadius = 4;

// Inserts (v, j) into a top-K list kept in rank order: skipped if an entry
// within the radius ranks before it; otherwise the entries within the radius
// (all ranking after it) are dropped and (v, j) goes in if it ranks before the
// last entry.  Compile-time indices only (no scratch memory).
template <int K>
__device__ inline void topk_insert(float (&tv)[K], int (&ti)[K], float v, int j)
{
    bool near[K];
    bool dominated = false;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        near[q] = ti[q] >= 0 && (ti[q] - j <= kRefineRadius && j - ti[q] <= kRefineRadius);
        dominated = dominated || (near[q] && ranks_before(tv[q], ti[q], v, j));
    }
    if (dominated) return;
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (near[q]) {
            tv[q] = -INFINITY;
            ti[q] = -1;
        }
    // move the emptied entries behind the others, keeping their order
#pragma unroll
    for (int pass = 0; pass + 1 < K; ++pass)
#pragma unroll
        for (int q = 0; q + 1 < K; ++q)
            if (ti[q] < 0 && ti[q + 1] >= 0) {
                tv[q] = tv[q + 1];
                ti[q] = ti[q + 1];
                tv[q + 1] = -INFINITY;
                ti[q + 1] = -1;
            }
    if (!ranks_before(v, j, tv[K - 1], ti[K - 1])) return;
    int pos = K - 1;
#pragma unroll
    for (int q = K - 2; q >= 0; --q)
        if (ranks_before(v, j, tv[q], ti[q])) pos = q;
#pragma unroll
    for (int q = K - 1; q >= 1; --q) {
        if (q > pos) {
            tv[q] = tv[q - 1];
            ti[q] = ti[q - 1];
        }
    }
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (q == pos) {
            tv[q] = v;
            ti[q] = j;
        }
}

// Largest of 16 values (NaN-free inputs; the compiler forms max3 chains).
__device__ inline float max16(const float (&a)[16])
{
    const float m0 = fmaxf(fmaxf(a[0], a[1]), a[2]);
    const float m1 = fmaxf(fmaxf(a[3], a[4]), a[5]);
    const float m2 = fmaxf(fmaxf(a[6], a[7]), a[8]);
    const float m3 = fmaxf(fmaxf(a[9], a[10]), a[11]);
    const float m4 = fmaxf(fmaxf(a[12], a[13]), a[14]);
    return fmaxf(fmaxf(fmaxf(fmaxf(m0, m1), m2), fmaxf(m3, m4)), a[15]);
}

// Row index (within the 32-window block) of accumulator v in lane `lane`.
__device__ inline int acc_row(int v, int lane) { return 8 * (v / 4) + 4 * (lane / 32) + (v % 4); }

// Grid: chunk-major (all resident workgroups sweep the same dictionary chunk,
// so its operand blocks are shared through L2).  Each wave owns NB query
// blocks (32 NB query windows) whose fragments stay in registers for the whole
// sweep.  The workgroup stages G dictionary blocks (G * KS = 32 fragments of
// 1 KB) at a time in LDS, double-buffered: the global loads of stage s+1 are in
// flight while the waves run the matrix products of stage s.
template <typename T, int KS, int NB, int K, int WPE>
__global__ __launch_bounds__(kWave* waves_per_block(KS)) __attribute__((amdgpu_waves_per_eu(WPE))) void k_join_mfma(
    const typename Vec8<T>::type* __restrict__ zq, int64_t nqblk, const typename Vec8<T>::type* __restrict__ zd,
    const uint32_t* __restrict__ dmask, int64_t ndblk, int64_t npanels, int64_t blk_per_chunk, int nchunks,
    unsigned long long* __restrict__ cand)
{
    using V8 = typename Vec8<T>::type;
    constexpr int kWavesPerBlock = waves_per_block(KS);
    constexpr int G = 32 / KS;                   // dictionary blocks per stage
    constexpr int kFrag = G * KS * kWave;        // 16-byte fragments per stage
    constexpr int kPerThread = kFrag / (kWave * kWavesPerBlock);
    __shared__ V8 stage[2][kFrag];

    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int64_t chunk = blockIdx.x / npanels;
    const int64_t panel = blockIdx.x - chunk * npanels;
    const int64_t qb0 = (panel * kWavesPerBlock + wave) * NB;
    const int64_t db_lo = chunk * blk_per_chunk;
    const int64_t db_hi = db_lo + blk_per_chunk < ndblk ? db_lo + blk_per_chunk : ndblk;
    const int64_t nst = (db_hi - db_lo + G - 1) / G;

    V8 bq[NB][KS];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qb = qb0 + nb < nqblk ? qb0 + nb : nqblk - 1;  // clamp: duplicate work, never stored
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bq[nb][ks] = zq[(qb * KS + ks) * kWave + lane];
    }
    float tv[NB][K];
    int ti[NB][K];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int q = 0; q < K; ++q) {
            tv[nb][q] = -INFINITY;
            ti[nb][q] = -1;
        }

    // stage s holds dictionary blocks db_lo + s G .. + G - 1, fragment order
    // (block, ks, lane) exactly as in global memory, so the copy is linear
    V8 pre[kPerThread];
    auto fetch = [&](int64_t s) {
        const int64_t base = (db_lo + s * G) * KS * kWave;
        const int64_t lim = db_hi * KS * kWave;
#pragma unroll
        for (int e = 0; e < kPerThread; ++e) {
            const int64_t f = base + (int64_t)e * (kWave * kWavesPerBlock) + threadIdx.x;
            pre[e] = f < lim ? zd[f] : V8{};
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < kPerThread; ++e) stage[buf][e * (kWave * kWavesPerBlock) + threadIdx.x] = pre[e];
    };
    if (nst > 0) {
        fetch(0);
        store(0);
    }
    __syncthreads();
    for (int64_t s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nst) fetch(s + 1);
        // two dictionary blocks at a time: 2 NB independent accumulation chains
#pragma unroll
        for (int g0 = 0; g0 < G; g0 += 2) {
            int64_t db[2];
            uint32_t msk[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                db[h] = db_lo + s * G + g0 + h;
                msk[h] = (g0 + h < G && db[h] < db_hi) ? dmask[db[h]] : 0u;
            }
            if ((msk[0] | msk[1]) == 0u) continue;  // both blocks masked or past the end
            f32x16 acc[2][NB];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[h][nb] = f32x16{};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                V8 ad[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) ad[h] = stage[buf][(((g0 + h) % G) * KS + ks) * kWave + lane];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) acc[h][nb] = mfma(ad[h], bq[nb][ks], acc[h][nb]);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (msk[h] == 0u) continue;
                const int jbase = (int)(db[h] * 32);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    float a[16];
#pragma unroll
                    for (int v = 0; v < 16; ++v) a[v] = acc[h][nb][v];
                    if (__builtin_expect(msk[h] != 0xFFFFFFFFu, 0)) {
                        // a block that straddles a segment break (rare): the
                        // opaque copy keeps the per-lane tests inside the branch
                        uint32_t mm = msk[h];
                        asm volatile("" : "+s"(mm));
#pragma unroll
                        for (int v = 0; v < 16; ++v)
                            if (!((mm >> acc_row(v, lane)) & 1u)) a[v] = -INFINITY;
                    }
                    float mx = max16(a);
                    bool hit = mx > tv[nb][K - 1];
                    if (__builtin_expect(__builtin_amdgcn_ballot_w64(hit) != 0, 0)) {
                        // rare (a row's K-th best improves a few dozen times per
                        // chunk): insert the lane's largest value above its K-th
                        // best, one per pass, until no lane of the wave has one
                        asm volatile("" ::: "memory");
                        do {
                            if (hit) {
                                // first (smallest row) position of the lane's largest value
                                int sel = 0;
#pragma unroll
                                for (int v = 15; v >= 0; --v) sel = a[v] == mx ? v : sel;
                                topk_insert<K>(tv[nb], ti[nb], mx, jbase + acc_row(sel, lane));
#pragma unroll
                                for (int v = 0; v < 16; ++v) a[v] = v == sel ? -INFINITY : a[v];
                                mx = max16(a);
                                hit = mx > tv[nb][K - 1];
                            }
                        } while (__builtin_amdgcn_ballot_w64(hit) != 0);
                    }
                }
            }
        }
        if (s + 1 < nst) store(buf ^ 1);
        __syncthreads();
    }
    // merge the two lane halves (same query window, disjoint dictionary rows)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        float ov[K];
        int oi[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            ov[q] = __shfl_xor(tv[nb][q], 32, kWave);
            oi[q] = __shfl_xor(ti[nb][q], 32, kWave);
        }
        if (lane < 32) {
#pragma unroll
            for (int q = 0; q < K; ++q) topk_insert<K>(tv[nb], ti[nb], ov[q], oi[q]);
            const int64_t row = (qb0 + nb) * 32 + lane;
            if (qb0 + nb < nqblk) {
                unsigned long long* dst = cand + (row * nchunks + chunk) * K;
#pragma unroll
                for (int q = 0; q < K; ++q) dst[q] = ti[nb][q] >= 0 ? pack_key(tv[nb][q], ti[nb][q]) : 0ull;
            }
        }
    }
}

constexpr unsigned long long kNone = ~0ull;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

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

// One wave per query row: the row's candidates from every chunk are taken
// best-first, each dropping the others within kRefineRadius of it, up to
// `keep` picks; the FP64 distance of every usable window within the radius of
// a pick is computed and the closest kept (ties: smaller index).  With
// `refine` off, report the distance implied by the best 16-bit score instead.
// Flat / non-finite conventions as in the FP32 tier.
__global__ __launch_bounds__(256) void k_finalize_topk(
    const double* __restrict__ axc, const double* __restrict__ amu, const double* __restrict__ asig,
    const uint8_t* __restrict__ aflags, int64_t WA, const double* __restrict__ bxc, const double* __restrict__ bmu,
    const double* __restrict__ bsig, const uint8_t* __restrict__ bflags, const unsigned long long* __restrict__ bfirst,
    int64_t WB, int m,
    const unsigned long long* __restrict__ cand, int ncand, int keep, int refine, int pearson,
    float* __restrict__ P, int64_t* __restrict__ I)
{
    const int lane = threadIdx.x % kWave;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= WA) return;
    const uint8_t fa = aflags[i];
    const unsigned long long ff = WB > 0 ? bfirst[0] : kNone;
    const unsigned long long fv = WB > 0 ? bfirst[1] : kNone;
    double pout;
    int64_t iout;
    if (fa & kFlagBad) {
        pout = NAN;
        iout = -1;
    } else if (fa & kFlagFlat) {
        if (ff != kNone) {
            pout = 0.0;
            iout = (int64_t)ff;
        } else if (fv != kNone) {
            pout = sqrt((double)m);
            iout = (int64_t)fv;
        } else {
            pout = INFINITY;
            iout = -1;
        }
    } else {
        double d = INFINITY;
        int64_t j = -1;
        const unsigned long long* c = cand + i * ncand;
        // the row's candidates from every chunk, best first (key order =
        // score order, ties -> smaller index), found by repeated wave-wide
        // maxima over the lanes' slices of the list
        constexpr int kMaxPerLane = 8;
        unsigned long long mine[kMaxPerLane];
#pragma unroll
        for (int q = 0; q < kMaxPerLane; ++q) {
            const int t = lane + q * kWave;
            mine[q] = t < ncand ? c[t] : 0ull;
        }
        for (int r = 0; r < keep; ++r) {
            unsigned long long lbest = 0ull;
#pragma unroll
            for (int q = 0; q < kMaxPerLane; ++q) lbest = mine[q] > lbest ? mine[q] : lbest;
            unsigned long long wbest = lbest;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const unsigned long long o = __shfl_xor(wbest, off, kWave);
                wbest = o > wbest ? o : wbest;
            }
            if (wbest == 0ull) break;  // uniform
            const int64_t jj = (int64_t)(0xFFFFFFFFu - (unsigned)(wbest & 0xFFFFFFFFull));
            // the pick and every other candidate within the radius: the
            // re-check below covers them
#pragma unroll
            for (int q = 0; q < kMaxPerLane; ++q) {
                if (mine[q] == 0ull) continue;
                const int64_t jq = (int64_t)(0xFFFFFFFFu - (unsigned)(mine[q] & 0xFFFFFFFFull));
                if (jq - jj <= kRefineRadius && jj - jq <= kRefineRadius) mine[q] = 0ull;
            }
            if (!refine) {
                d = sqrt(fmax(0.0, 2.0 * m * (1.0 - (double)unpack_score(wbest))));
                j = jj;
                break;
            }
            // FP64 distance of every usable window within the radius of the pick
            const int64_t t0 = jj - kRefineRadius > 0 ? jj - kRefineRadius : 0;
            const int64_t t1 = jj + kRefineRadius < WB - 1 ? jj + kRefineRadius : WB - 1;
            for (int64_t t = t0; t <= t1; ++t) {
                if (bflags[t] != 0) continue;  // same t in every lane: uniform
                const double dd = wave_dist(axc + i, amu[i], asig[i], bxc + t, bmu[t], bsig[t], m, lane);
                if (dd < d || (dd == d && t < j)) {
                    d = dd;
                    j = t;
                }
            }
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
    if (pearson) pout = isnan(pout) ? pout : isinf(pout) ? -INFINITY : 1.0 - pout * pout / (2.0 * (double)m);
    if (lane == 0) {
        P[i] = (float)pout;
        I[i] = iout;
    }
}

template <typename T, int KS, int NB, int K>
void launch_main(const MfmaPlan& p, const void* zq, const void* zd, const uint32_t* dmask,
                 unsigned long long* cand, hipStream_t stream)
{
    using V8 = typename Vec8<T>::type;
    // four waves per SIMD where the 8-wave workgroup's 64 KB of LDS allows two
    // workgroups per CU; the 4-wave workgroups of K-step 16 fit two per SIMD
    constexpr int WPE = KS <= 8 ? 4 : 2;
    hipLaunchKernelGGL((k_join_mfma<T, KS, NB, K, WPE>), dim3((unsigned)(p.npanels * p.nchunks)),
                       dim3(kWave * waves_per_block(KS)), 0, stream, reinterpret_cast<const V8*>(zq), p.nqblk,
                       reinterpret_cast<const V8*>(zd), dmask, p.ndblk, p.npanels, p.blk_per_chunk,
                       (int)p.nchunks, cand);
}

template <typename T, int KS, int NB>
int launch_k(const MfmaPlan& p, const void* zq, const void* zd, const uint32_t* dmask, unsigned long long* cand,
             hipStream_t stream)
{
    switch (p.K) {
        case 1: launch_main<T, KS, NB, 1>(p, zq, zd, dmask, cand, stream); break;
        case 2: launch_main<T, KS, NB, 2>(p, zq, zd, dmask, cand, stream); break;
        case 4: launch_main<T, KS, NB, 4>(p, zq, zd, dmask, cand, stream); break;
        case 8: launch_main<T, KS, NB, 8>(p, zq, zd, dmask, cand, stream); break;
        default: return set_error(ABJ_EINVAL, "unsupported candidate count %d", p.K);
    }
    return ABJ_OK;
}

template <typename T>
int launch_ks(const MfmaPlan& p, const void* zq, const void* zd, const uint32_t* dmask, unsigned long long* cand,
              hipStream_t stream)
{
    switch (p.KS) {
        case 2: return launch_k<T, 2, 1>(p, zq, zd, dmask, cand, stream);
        case 4: return launch_k<T, 4, 1>(p, zq, zd, dmask, cand, stream);
        case 8: return launch_k<T, 8, 1>(p, zq, zd, dmask, cand, stream);
        case 16: return launch_k<T, 16, 1>(p, zq, zd, dmask, cand, stream);
        default: return set_error(ABJ_EINVAL, "unsupported k-step count %d", p.KS);
    }
}

template <typename T>
void make_operand(const SeriesDev& s, int ks_n, int64_t nblk, void* out, hipStream_t stream)
{
    using V8 = typename Vec8<T>::type;
    const int64_t nfrag = nblk * ks_n * kWave;
    hipLaunchKernelGGL(k_make_operand<T>, dim3((unsigned)((nfrag + 255) / 256)), dim3(256), 0, stream, s.xc, s.mu,
                       s.sig, s.flags, s.W, (int)s.m, ks_n, nfrag, reinterpret_cast<V8*>(out));
}

}  // namespace

int mfma_plan(int64_t WA, int64_t WB, int32_t m, int tier, int refine_k, MfmaPlan* p)
{
    const int mp = (m + 15) / 16;
    int KS;
    if (mp <= 2) KS = 2;
    else if (mp <= 4) KS = 4;
    else if (mp <= 8) KS = 8;
    else if (mp <= 16) KS = 16;
    else return set_error(ABJ_EINVAL, "the BF16/FP16 tiers support m <= 256 (got %d)", m);
    int K = refine_k <= 0 ? 4 : refine_k;
    K = K <= 1 ? 1 : K <= 2 ? 2 : K <= 4 ? 4 : 8;
    // one query block per wave: it leaves the registers for four waves per
    // SIMD (K-steps <= 8), which hide the LDS and MFMA latencies of the sweep
    const int NB = 1;
    p->tier = tier;
    p->KS = KS;
    p->K = K;
    p->nqblk = (WA + 31) / 32;
    p->ndblk = (WB + 31) / 32;
    const int64_t qblk_per_panel = (int64_t)waves_per_block(KS) * NB;
    p->npanels = (p->nqblk + qblk_per_panel - 1) / qblk_per_panel;
    // split the dictionary sweep until there are enough workgroups to fill the
    // chip, but keep at least 64 blocks (2,048 windows) per chunk
    int64_t nchunks = 1;
    while (p->npanels * nchunks < 2048 && (p->ndblk + nchunks * 2 - 1) / (nchunks * 2) >= 64) nchunks *= 2;
    while (nchunks * K > 512) nchunks /= 2;  // the re-check reads at most 512 candidates per row
    // a reference shorter than m has no block: one empty chunk (no sweep)
    p->blk_per_chunk = p->ndblk > 0 ? (p->ndblk + nchunks - 1) / nchunks : 1;
    p->nchunks = p->ndblk > 0 ? (p->ndblk + p->blk_per_chunk - 1) / p->blk_per_chunk : 1;
    return ABJ_OK;
}

size_t mfma_scratch_bytes(const MfmaPlan& p)
{
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t b = 0;
    b += al((size_t)p.nqblk * p.KS * kWave * 16);  // query operand
    b += al((size_t)p.ndblk * p.KS * kWave * 16);  // dictionary operand
    b += al((size_t)p.ndblk * 4);                  // block masks
    b += al((size_t)p.nqblk * 32 * p.nchunks * p.K * 8);  // candidates
    return b;
}

int join_mfma_run(const SeriesDev& A, const SeriesDev& B, const MfmaPlan& p, int refine, int pearson, float* P,
                  int64_t* I,
                  Arena& ar, hipStream_t stream)
{
    void* zq = ar.take<char>((size_t)p.nqblk * p.KS * kWave * 16);
    void* zd = ar.take<char>((size_t)p.ndblk * p.KS * kWave * 16);
    uint32_t* dmask = ar.take<uint32_t>((size_t)p.ndblk);
    unsigned long long* cand = ar.take<unsigned long long>((size_t)p.nqblk * 32 * p.nchunks * p.K);
    if (A.W <= 0) return ABJ_OK;
    if (B.W > 0) {
        if (p.tier == ABJ_TIER_BF16) {
            make_operand<__bf16>(A, p.KS, p.nqblk, zq, stream);
            make_operand<__bf16>(B, p.KS, p.ndblk, zd, stream);
        } else {
            make_operand<_Float16>(A, p.KS, p.nqblk, zq, stream);
            make_operand<_Float16>(B, p.KS, p.ndblk, zd, stream);
        }
        hipLaunchKernelGGL(k_block_mask, dim3((unsigned)((p.ndblk + 255) / 256)), dim3(256), 0, stream, B.flags, B.W,
                           p.ndblk, dmask);
        ABJ_HIP(hipGetLastError());
        ProfMark mark;
        ABJ_TRY(prof_begin(&mark, stream));
        ABJ_TRY(p.tier == ABJ_TIER_BF16 ? launch_ks<__bf16>(p, zq, zd, dmask, cand, stream)
                                        : launch_ks<_Float16>(p, zq, zd, dmask, cand, stream));
        ABJ_HIP(hipGetLastError());
        ABJ_TRY(prof_end(&mark, stream, A.W * B.nvalid));
    } else {
        ABJ_TRY(fill_u64(cand, p.nqblk * 32 * p.nchunks * p.K, 0ull, stream));
    }
    const int rows_per_block = 4;
    hipLaunchKernelGGL(k_finalize_topk, dim3((unsigned)((A.W + rows_per_block - 1) / rows_per_block)),
                       dim3(kWave * rows_per_block), 0, stream, A.xc, A.mu, A.sig, A.flags, A.W, B.xc, B.mu, B.sig,
                       B.flags, B.first, B.W, (int)A.m, cand, (int)(p.nchunks * p.K), p.K, refine, pearson, P, I);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

}  // namespace abj
