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

// Pointers taken from a job descriptor lose the kernel argument's global
// address space, and the compiler then emits flat accesses, which count on the
// LDS wait counter too (so waiting for one would wait for pending LDS reads):
// give them back the global address space.
template <class T>
__device__ inline const __attribute__((address_space(1))) T* gptr(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline __attribute__((address_space(1))) T* gptr_w(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// Workgroup b of a launch over a job table belongs to the last job whose
// first workgroup blk0 is <= b (blk0 ascending; uniform per workgroup).
template <class J>
__device__ inline int find_job(const J* __restrict__ jobs, int n, int64_t b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One thread per (32-window block, k step, lane) fragment of 8 elements of
// one series (a job): z[k] = (x[i+k] - mu(i)) / (sigma(i) sqrt(m)) in FP64,
// then cast; windows that cannot match (flags) and k >= m are zeros.
template <typename T>
__global__ __launch_bounds__(256) void k_make_operand(MfmaOpJob one, const MfmaOpJob* __restrict__ jobs, int njobs)
{
    const MfmaOpJob J = jobs ? jobs[find_job(jobs, njobs, blockIdx.x)] : one;
    const int64_t t = ((int64_t)blockIdx.x - J.blk0) * blockDim.x + threadIdx.x;
    if (t >= J.nfrag) return;
    const int lane = (int)(t % kWave);
    const int64_t bk = t / kWave;  // block * ks_n + ks
    const int ks = (int)(bk % J.ks_n);
    const int64_t blk = bk / J.ks_n;
    const int64_t i = blk * 32 + (lane % 32);
    const int k0 = ks * 16 + 8 * (lane / 32);
    typename Vec8<T>::type v;
    const bool use = i < J.W && J.flags[i] == 0;
    const double mean = use ? J.mu[i] : 0.0;
    const double scale = use ? 1.0 / (J.sig[i] * sqrt((double)J.m)) : 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        const double z = (use && k < J.m) ? (J.xc[i + k] - mean) * scale : 0.0;
        v[e] = (T)(float)z;
    }
    reinterpret_cast<typename Vec8<T>::type*>(J.out)[t] = v;
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

// The row epilogue takes the candidates best-first, drops the others within
// kRefineRadius windows of each pick, and re-checks every window within that
// radius of a pick in FP64: neighbouring windows have nearly equal 16-bit
// scores, so the best window often ranks just behind a neighbour, and the K
// candidates of a chunk are mostly one neighbourhood.
constexpr int kRefineRadius = 4;

// Inserts (v, j) into a top-K list kept in rank order if it ranks before the
// last entry.  Compile-time indices only (no scratch memory).
template <int K>
__device__ inline void topk_insert(float (&tv)[K], int (&ti)[K], float v, int j)
{
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

// The same for a lane's own sweep, where the scores are stamped (below) and a
// later equal score comes from a later block, hence a larger index: the
// value alone decides.
template <int K>
__device__ inline void topk_insert_stamped(float (&tv)[K], int (&ti)[K], float v, int j)
{
    if (!(v > tv[K - 1])) return;
#pragma unroll
    for (int q = K - 1; q >= 1; --q) {
        const bool shift = v > tv[q - 1];  // v goes at or before q - 1
        const bool here = !shift && v > tv[q];
        tv[q] = shift ? tv[q - 1] : here ? v : tv[q];
        ti[q] = shift ? ti[q - 1] : here ? j : ti[q];
    }
    if (v > tv[0]) {
        tv[0] = v;
        ti[0] = j;
    }
}

// A score below every real one: the top-K lists start with it and masked
// windows take it (finite, so that stamping keeps it a number).
constexpr float kNoScore = -3.0e38f;

// Stamps accumulator v's position into the low 4 bits of its score (15 - v,
// so that equal scores rank the smaller row first): the scores of a lane's
// block become distinct and the largest carries its own position.  It moves a
// score by at most 15 units in the last place, far below the 16-bit inputs'
// resolution.
__device__ inline float stamp(float x, int v)
{
    return __uint_as_float((__float_as_uint(x) & ~15u) | (unsigned)(15 - v));
}

// Largest of 16 values.  The inputs are never NaN (finite matrix-core
// results, their stamped forms, kNoScore), so IEEE maximum (which would
// propagate a NaN) equals the usual fmaxf here; it maps onto gfx950's
// three-input v_maximum3_f32 without the operand canonicalisations fmaxf
// needs: 8 instructions for the 16 values.
__device__ inline float max2(float a, float b) { return __builtin_elementwise_maximum(a, b); }
__device__ inline float max16(const float (&a)[16])
{
    const float m0 = max2(max2(a[0], a[1]), a[2]);
    const float m1 = max2(max2(a[3], a[4]), a[5]);
    const float m2 = max2(max2(a[6], a[7]), a[8]);
    const float m3 = max2(max2(a[9], a[10]), a[11]);
    const float m4 = max2(max2(a[12], a[13]), a[14]);
    return max2(max2(max2(m0, m1), m2), max2(max2(m3, m4), a[15]));
}

// Row index (within the 32-window block) of accumulator v in lane `lane`.
__device__ inline int acc_row(int v, int lane) { return 8 * (v / 4) + 4 * (lane / 32) + (v % 4); }

// Grid: chunk-major within a job (all resident workgroups of a job sweep the
// same dictionary chunk, so its operand blocks are shared through L2).  Each
// wave owns NB query blocks (32 NB query windows) whose fragments stay in
// registers for the whole sweep.  The workgroup of NW waves stages G
// dictionary blocks (G * KS = 32 fragments of 1 KB) at a time in LDS,
// double-buffered: the global loads of stage s+1 are in flight while the
// waves run the matrix products of stage s.  Two dictionary blocks are taken
// per step, for two independent accumulation chains.
//
// Candidates: each lane keeps the KH best (score, window) of its own rows
// (one query window, half of the dictionary windows of every block); the two
// halves are merged into KH per row and chunk at the end.  The per-block test
// against a lane's KH-th best is a wave-wide branch: with 64 lanes and their
// own thresholds some lane passes it in nearly every one of the first 64 KH
// blocks of a sweep, and in about 64 KH / b of the blocks after that, so long
// sweeps (few chunks) keep the insert path rare.
template <typename T, int KS, int NB, int KH, int NW, int WPE>
__global__ __launch_bounds__(kWave* NW) __attribute__((amdgpu_waves_per_eu(WPE))) void k_join_mfma(
    MfmaJoinJob one, const MfmaJoinJob* __restrict__ jobs, int njobs)
{
    using V8 = typename Vec8<T>::type;
    // dictionary blocks per stage: 32 KB of fragments, 64 KB with 2 waves per
    // SIMD (one workgroup per CU then, so the two buffers fit in LDS: fewer
    // barriers)
    constexpr int G = (WPE <= 2 ? 64 : 32) / KS;
    constexpr int kFrag = G * KS * kWave;        // 16-byte fragments per stage
    constexpr int kPerThread = kFrag / (kWave * NW);
    static_assert(G % 2 == 0, "two blocks per step");
    __shared__ V8 stage[2][kFrag];

    const MfmaJoinJob J = jobs ? jobs[find_job(jobs, njobs, blockIdx.x)] : one;
    const auto zq = gptr(reinterpret_cast<const V8*>(J.zq));
    const auto zd = gptr(reinterpret_cast<const V8*>(J.zd));
    const auto dmask = gptr(J.dmask);
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int64_t local = (int64_t)blockIdx.x - J.blk0;
    const int64_t chunk = local / J.npanels;
    const int64_t panel = local - chunk * J.npanels;
    const int64_t qb0 = (panel * NW + wave) * NB;
    const int64_t db_lo = chunk * J.blk_per_chunk;
    const int64_t db_hi = db_lo + J.blk_per_chunk < J.ndblk ? db_lo + J.blk_per_chunk : J.ndblk;
    const int64_t nst = (db_hi - db_lo + G - 1) / G;

    V8 bq[NB][KS];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int64_t qb = qb0 + nb < J.nqblk ? qb0 + nb : J.nqblk - 1;  // clamp: duplicate work, never stored
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) bq[nb][ks] = zq[(qb * KS + ks) * kWave + lane];
    }
    float tv[NB][KH];
    int ti[NB][KH];
    // gate: the larger of the two lane halves' KH-th best scores (lanes l and
    // l ^ 32 hold the same query window).  The row's merged top KH is never
    // below it, so a score below it can be skipped; exchanged after every
    // insert.
    float gate[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        gate[nb] = kNoScore;
#pragma unroll
        for (int q = 0; q < KH; ++q) {
            tv[nb][q] = kNoScore;
            ti[nb][q] = -1;
        }
    }

    // stage s holds dictionary blocks db_lo + s G .. + G - 1, fragment order
    // (block, ks, lane) exactly as in global memory, so the copy is linear.
    // The fragments go from global memory straight into LDS (each wave's 64
    // lanes fill 1 KB): no registers hold them in flight, and they are waited
    // for (vmcnt) before the barrier that ends the stage.  Every lane issues
    // all its loads; past the chunk the address is clamped (those blocks have
    // mask 0 and are never used).
    auto fetch = [&](int64_t s, int into) {
        const int64_t base = (db_lo + s * G) * KS * kWave;
        const int64_t lim = db_hi * KS * kWave;
#pragma unroll
        for (int e = 0; e < kPerThread; ++e) {
            const int64_t f = base + (int64_t)e * (kWave * NW) + threadIdx.x;
            __builtin_amdgcn_global_load_lds(
                (const void*)(zd + (f < lim ? f : lim - 1)),
                (__attribute__((address_space(3))) void*)&stage[into][e * (kWave * NW) + wave * kWave], 16, 0, 0);
        }
    };
    // vmcnt(0), the other counters left alone
    auto wait_loads = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };
    // the masks of a stage's G blocks, one per lane (0 past the chunk),
    // loaded one stage ahead with the fragments and read with readlane (a
    // scalar load per block shares its wait counter with the LDS reads)
    uint32_t smask = 0u, smask_next = 0u;
    auto fetch_mask = [&](int64_t s) {
        const int64_t db = db_lo + s * G + lane;
        smask_next = lane < G && db < db_hi ? dmask[db] : 0u;
    };

    __builtin_assume(nst > 0);  // every chunk holds a block (mfma_plan)
    fetch_mask(0);
    fetch(0, 0);
    wait_loads();
    __syncthreads();
    for (int64_t s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        smask = smask_next;
        if (s + 1 < nst) {
            fetch_mask(s + 1);
            fetch(s + 1, buf ^ 1);  // its readers passed the barrier that ended stage s - 1
        }
        for (int g0 = 0; g0 < G; g0 += 2) {
            uint32_t msk[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) msk[h] = __builtin_amdgcn_readlane(smask, g0 + h);
            if ((msk[0] | msk[1]) == 0u) continue;  // both blocks masked or past the end
            f32x16 acc[2][NB];
            if constexpr (KS <= 4) {
                // every fragment of the step read before the first product, so
                // the LDS latency is paid once per step
                V8 ad[2][KS];
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int h = 0; h < 2; ++h) ad[h][ks] = stage[buf][((g0 + h) * KS + ks) * kWave + lane];
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[h][nb] = mfma(ad[h][ks], bq[nb][ks], ks == 0 ? f32x16{} : acc[h][nb]);
            } else {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    V8 ad[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) ad[h] = stage[buf][((g0 + h) * KS + ks) * kWave + lane];
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[h][nb] = mfma(ad[h], bq[nb][ks], ks == 0 ? f32x16{} : acc[h][nb]);
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (msk[h] == 0u) continue;
                const int jbase = (int)((db_lo + s * G + g0 + h) * 32);
                const bool partial = msk[h] != 0xFFFFFFFFu;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    float mx;
                    {
                        float c[16];
#pragma unroll
                        for (int v = 0; v < 16; ++v) c[v] = acc[h][nb][v];
                        mx = max16(c);
                    }
                    bool hit = mx > gate[nb];
                    if (__builtin_expect(__builtin_amdgcn_ballot_w64(hit) != 0 || partial, 0)) {
                        // insert the lane's values above its KH-th best, the
                        // largest first (at most KH of them can stay); in a
                        // block that straddles a segment break (rare) the
                        // masked windows are removed first.  Stamped scores
                        // give each pass its position without a search.
                        asm volatile("" ::: "memory");
                        float a[16];
#pragma unroll
                        for (int v = 0; v < 16; ++v) a[v] = stamp(acc[h][nb][v], v);
                        if (partial) {
                            uint32_t mm = __builtin_amdgcn_readfirstlane(msk[h]);
                            asm volatile("" : "+s"(mm));  // keeps the per-lane tests inside the branch
#pragma unroll
                            for (int v = 0; v < 16; ++v)
                                if (!((mm >> acc_row(v, lane)) & 1u)) a[v] = kNoScore;
                        }
                        mx = max16(a);
                        hit = mx > gate[nb];
                        constexpr int kPassUnroll = KH <= 4 ? KH : 1;  // a rolled loop for 8 keeps the registers
#pragma unroll kPassUnroll
                        for (int pass = 0; pass < KH; ++pass) {
                            if (__builtin_amdgcn_ballot_w64(hit) == 0) break;
                            if (hit) {
                                const int sel = 15 - (int)(__float_as_uint(mx) & 15u);
                                topk_insert_stamped<KH>(tv[nb], ti[nb], mx, jbase + acc_row(sel, lane));
                                if (pass + 1 < KH) {
                                    // the next largest: everything below this one
#pragma unroll
                                    for (int v = 0; v < 16; ++v) a[v] = a[v] < mx ? a[v] : kNoScore;
                                    mx = max16(a);
                                    hit = mx > fmaxf(gate[nb], tv[nb][KH - 1]);
                                }
                            }
                        }
                        const float own = tv[nb][KH - 1];
                        gate[nb] = fmaxf(own, __shfl_xor(own, 32, kWave));
                    }
                }
            }
        }
        wait_loads();
        __syncthreads();
    }
    // merge the two lane halves (same query window, disjoint dictionary rows)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        float ov[KH];
        int oi[KH];
#pragma unroll
        for (int q = 0; q < KH; ++q) {
            ov[q] = __shfl_xor(tv[nb][q], 32, kWave);
            oi[q] = __shfl_xor(ti[nb][q], 32, kWave);
        }
        if (lane < 32) {
#pragma unroll
            for (int q = 0; q < KH; ++q) topk_insert<KH>(tv[nb], ti[nb], ov[q], oi[q]);
            const int64_t row = (qb0 + nb) * 32 + lane;
            if (qb0 + nb < J.nqblk) {
                auto dst = gptr_w(J.cand + (row * J.nchunks + chunk) * KH);
#pragma unroll
                for (int q = 0; q < KH; ++q) dst[q] = ti[nb][q] >= 0 ? pack_key(tv[nb][q], ti[nb][q]) : 0ull;
            }
        }
    }
}

constexpr unsigned long long kNone = ~0ull;

constexpr int kFinRows = 2;  // query rows (one wave each) per workgroup of the re-check

// Exchanges within a row of 16 lanes on the DPP path: quad_perm xor 1 and
// xor 2, half-row mirror (xor 7), row rotate by 4 and by 8.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRor4 = 0x124, kDppRor8 = 0x128;
template <int kCtrl>
__device__ __forceinline__ unsigned dpp_u32(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xf, 0xf, true);
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
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int l)
{
    // readlane returns int: take both halves as unsigned before widening
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((unsigned)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double lane_f64(double v, int l)
{
    return __longlong_as_double((long long)lane_u64((unsigned long long)__double_as_longlong(v), l));
}
// The largest key of the wave (of its first 16 lanes if kRows is 1), wave-
// uniform: each row of 16 lanes on the DPP path, then the rows' results
// through scalar reads.
template <int kRows>
__device__ inline unsigned long long wave_max_u64(unsigned long long v)
{
    unsigned long long o = dpp_u64<kDppXor1>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppXor2>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppHalfMirror>(v);
    v = o > v ? o : v;
    o = dpp_u64<kDppRor8>(v);
    v = o > v ? o : v;
    unsigned long long w = lane_u64(v, 0);
#pragma unroll
    for (int r = 16; r < 16 * kRows; r += 16) {
        const unsigned long long x = lane_u64(v, r);
        w = x > w ? x : w;
    }
    return w;
}
// One argmin step over (distance, window): the partner's pair if it ranks
// first (smaller distance, then smaller window).
template <int kCtrl>
__device__ __forceinline__ void argmin_step(double& d, int64_t& t)
{
    const double od = dpp_f64<kCtrl>(d);
    const int64_t ot = (int64_t)dpp_u64<kCtrl>((unsigned long long)t);
    if (od < d || (od == d && ot < t)) {
        d = od;
        t = ot;
    }
}

// One wave per query row.  The row's candidates from every chunk are taken
// best-first, each dropping the others within kRefineRadius of it, up to
// `keep` picks.  Then the windows near the picks are re-checked in FP64: with
// L = 64 / (keep rounded up to a power of two) lanes per pick, pick p covers
// the L windows from L/2 - 1 before it to L/2 after it (for 4 picks, 7 before
// to 8 after).  The row's window minus its mean and each pick's span of
// reference samples are staged in LDS, the spans two picks at a time (one
// memory round trip each); the statistics of the windows are fetched while
// the sums run.  A lane takes 4 consecutive windows of its pick and a quarter
// of the samples: a sliding window of 4 reference samples gives 4 FP64 FMAs
// per sample pair, and the quarters are summed across lanes, after which
// each of the four lanes sharing the 4 windows finishes one of them.  The
// distance comes from the covariance, sum (a - mu_a) b (the centred row sums
// to zero, so the reference's mean drops out), as sqrt(2m (1 - rho)).
// Windows outside the reference or that cannot match are skipped.  One
// wave-wide argmin (ties: smaller index) gives the row's result.  Maxima and
// minima across lanes take the DPP path within rows of 16 lanes and scalar
// reads across rows.  With `refine` off, report the distance implied by the
// best 16-bit score instead.  Flat / non-finite conventions as in the FP32
// tier.  kMaxPick: the largest `keep` of the launch's jobs (4 or 8), which
// sizes the stage (10.5 or 18.4 KiB per wave; the larger stage leaves room for
// 2 waves per SIMD, and the register budget follows).
template <int kMaxPick>
__global__ __launch_bounds__(kWave* kFinRows) __attribute__((amdgpu_waves_per_eu(kMaxPick <= 4 ? 4 : 2)))
void k_finalize_topk(MfmaFinJob one, const MfmaFinJob* __restrict__ jobs, int njobs)
{
    // per wave: the row (256 doubles), then kMaxPick spans of up to
    // m + 64 / kMaxPick - 1 reference samples (one pick of 64 lanes: m + 63)
    constexpr int kSpanLen = kMaxPick <= 4 ? 256 + 15 : 256 + 7;
    constexpr int kStage = 256 + (kMaxPick * kSpanLen > 256 + 63 ? kMaxPick * kSpanLen : 256 + 63);
    __shared__ double stage_all[kFinRows][kStage];
    const MfmaFinJob J = jobs ? jobs[find_job(jobs, njobs, blockIdx.x)] : one;
    const int lane = threadIdx.x % kWave;
    const int64_t i = ((int64_t)blockIdx.x - J.blk0) * kFinRows + threadIdx.x / kWave;
    if (i >= J.WA) return;
    double* __restrict__ sa = stage_all[threadIdx.x / kWave];
    double* __restrict__ sb = sa + 256;
    const int m = J.m;
    const auto aflags = gptr(J.aflags);
    const auto bflags = gptr(J.bflags);
    const uint8_t fa = aflags[i];
    const unsigned long long ff = J.WB > 0 ? gptr(J.bfirst)[0] : kNone;
    const unsigned long long fv = J.WB > 0 ? gptr(J.bfirst)[1] : kNone;
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
        const auto c = gptr(J.cand + i * J.ncand);
        // the row's candidates from every chunk, best first (key order =
        // score order, ties -> smaller index), found by repeated wave-wide
        // maxima over the lanes' slices of the list
        constexpr int kMaxPerLane = 8;
        unsigned long long mine[kMaxPerLane];
#pragma unroll
        for (int q = 0; q < kMaxPerLane; ++q) {
            const int t = lane + q * kWave;
            mine[q] = 0ull;
            if (q * kWave < J.ncand && t < J.ncand) mine[q] = c[t];  // first test uniform
        }
        // the row minus its mean, staged while the picks are taken
        const double ma = gptr(J.amu)[i];
        {
            const auto xa = gptr(J.axc + i);
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const int t = lane + x * kWave;
                if (t < m) sa[t] = xa[t] - ma;
            }
        }
        int64_t pick[kMaxPick];
#pragma unroll
        for (int r = 0; r < kMaxPick; ++r) pick[r] = -1;
        int npick = 0;
#pragma unroll
        for (int r = 0; r < kMaxPick; ++r) {
            if (r >= J.keep) continue;
            unsigned long long lbest = mine[0];
#pragma unroll
            for (int q = 1; q < kMaxPerLane; ++q)
                if (q * kWave < J.ncand) lbest = mine[q] > lbest ? mine[q] : lbest;  // uniform guard
            const unsigned long long wbest = J.ncand <= 16 ? wave_max_u64<1>(lbest) : wave_max_u64<4>(lbest);
            if (wbest == 0ull) break;  // uniform
            const int64_t jj = (int64_t)(0xFFFFFFFFu - (unsigned)(wbest & 0xFFFFFFFFull));
            if (!J.refine) {
                d = sqrt(fmax(0.0, 2.0 * m * (1.0 - (double)unpack_score(wbest))));
                j = jj;
                break;
            }
            pick[r] = jj;
            npick = r + 1;
            // the pick and every other candidate within the radius: the
            // re-check below covers them
#pragma unroll
            for (int q = 0; q < kMaxPerLane; ++q) {
                if (q * kWave >= J.ncand) break;  // uniform
                const int64_t jq = (int64_t)(0xFFFFFFFFu - (unsigned)(mine[q] & 0xFFFFFFFFull));
                if (jq - jj <= kRefineRadius && jj - jq <= kRefineRadius) mine[q] = 0ull;
            }
        }
        if (J.refine && npick > 0) {
            const int L = J.keep <= 1 ? 64 : J.keep <= 2 ? 32 : J.keep <= 4 ? 16 : 8;
            const int span = m + L - 1;  // reference samples of a pick's L windows, at most 256 + 63
            // each pick's span, two picks' loads in flight at a time (samples
            // below 0 belong to windows that are skipped: their loads are
            // clamped to 0)
            const auto xb = gptr(J.bxc);
            constexpr int kSpanIt = (256 + 63 + kWave - 1) / kWave;
#pragma unroll
            for (int r0 = 0; r0 < kMaxPick; r0 += 2) {
                if (r0 >= npick) break;  // uniform
                double v[2][kSpanIt];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // s0 >= -L/2 >= -32: only the first load can fall below 0
                    const int64_t s0 = pick[r0 + h] - L / 2 + 1;
                    const int64_t x0 = s0 + lane;
                    v[h][0] = xb[x0 > 0 ? x0 : 0];
                    const auto xu = xb + (x0 + kWave);
#pragma unroll
                    for (int u = 1; u < kSpanIt; ++u) v[h][u] = xu[(u - 1) * kWave];
                }
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int u = 0; u < kSpanIt; ++u) {
                        const int t = lane + u * kWave;
                        if (r0 + h < npick && t < span) sb[(r0 + h) * span + t] = v[h][u];
                    }
            }
            const int pr = lane / L, g = lane % L;
            const int Q = L / 4;          // lanes per sample quarter
            const int kq = g / Q;         // this lane's quarter of the samples
            const int sg = g % Q;         // this lane's 4 windows: 4 sg .. 4 sg + 3 of the pick's L
            int64_t base = -1;
#pragma unroll
            for (int r = 0; r < kMaxPick; ++r)
                if (r == pr && r < npick) base = pick[r];
            const int64_t t0 = base - L / 2 + 1 + 4 * sg;  // first window of the lane
            // after the sums below, the four lanes of a window group (one per
            // quarter) hold the same four sums: lane kq finishes window t0 + kq.
            // Its statistics are fetched before the sums (a window outside the
            // reference is skipped)
            const int64_t tw = t0 + kq;
            const bool fin = base >= 0 && tw >= 0 && tw < J.WB;
            uint8_t wfl = 1;
            double wsig = 1.0;
            if (fin) {
                wfl = bflags[tw];
                wsig = gptr(J.bsig)[tw];
            }
            const double sa_ = gptr(J.asig)[i];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // an odd quarter length puts the quarters' samples on different
            // LDS banks
            const int mq = ((m + 3) / 4) | 1;
            const int k0 = kq * mq, k1 = k0 + mq < m ? k0 + mq : m;
            double cv[4] = {0.0, 0.0, 0.0, 0.0};
            if (base >= 0 && k0 < k1) {
                const double* __restrict__ bw = sb + pr * span + 4 * sg;  // window t0 + r, sample k: bw[r + k]
                double w0 = bw[k0], w1 = bw[k0 + 1], w2 = bw[k0 + 2];
                int k = k0;
#pragma unroll 2
                for (; k + 4 <= k1; k += 4) {
                    const double a0 = sa[k], a1 = sa[k + 1], a2 = sa[k + 2], a3 = sa[k + 3];
                    const double b3 = bw[k + 3], b4 = bw[k + 4], b5 = bw[k + 5], b6 = bw[k + 6];
                    // sample by sample, as the one-step loop below
                    cv[0] = fma(a0, w0, cv[0]);
                    cv[1] = fma(a0, w1, cv[1]);
                    cv[2] = fma(a0, w2, cv[2]);
                    cv[3] = fma(a0, b3, cv[3]);
                    cv[0] = fma(a1, w1, cv[0]);
                    cv[1] = fma(a1, w2, cv[1]);
                    cv[2] = fma(a1, b3, cv[2]);
                    cv[3] = fma(a1, b4, cv[3]);
                    cv[0] = fma(a2, w2, cv[0]);
                    cv[1] = fma(a2, b3, cv[1]);
                    cv[2] = fma(a2, b4, cv[2]);
                    cv[3] = fma(a2, b5, cv[3]);
                    cv[0] = fma(a3, b3, cv[0]);
                    cv[1] = fma(a3, b4, cv[1]);
                    cv[2] = fma(a3, b5, cv[2]);
                    cv[3] = fma(a3, b6, cv[3]);
                    w0 = b4;
                    w1 = b5;
                    w2 = b6;
                }
                for (; k < k1; ++k) {
                    const double av = sa[k], bv = bw[k + 3];
                    cv[0] = fma(av, w0, cv[0]);
                    cv[1] = fma(av, w1, cv[1]);
                    cv[2] = fma(av, w2, cv[2]);
                    cv[3] = fma(av, bv, cv[3]);
                    w0 = w1;
                    w1 = w2;
                    w2 = bv;
                }
            }
            // the four quarters' sums: lanes Q and 2Q apart within the pick
            // (16 lanes per pick: rotations of the DPP row by 4 and 8)
            if (L == 16) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cv[r] += dpp_f64<kDppRor4>(cv[r]);
                    cv[r] += dpp_f64<kDppRor8>(cv[r]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cv[r] += __shfl_xor(cv[r], Q, kWave);
                    cv[r] += __shfl_xor(cv[r], 2 * Q, kWave);
                }
            }
            double dd = INFINITY;
            int64_t tt = INT64_MAX;
            if (fin && wfl == 0) {
                const double cw = kq == 0 ? cv[0] : kq == 1 ? cv[1] : kq == 2 ? cv[2] : cv[3];
                const double rho = cw / ((double)m * sa_ * wsig);
                dd = sqrt(fmax(0.0, 2.0 * (double)m * (1.0 - rho)));
                tt = tw;
            }
            // wave argmin of (distance, window); lanes without a window hold
            // +inf: each row of 16 lanes on the DPP path, then the four rows
            argmin_step<kDppXor1>(dd, tt);
            argmin_step<kDppXor2>(dd, tt);
            argmin_step<kDppHalfMirror>(dd, tt);
            argmin_step<kDppRor8>(dd, tt);
            double bd = lane_f64(dd, 0);
            int64_t bt = (int64_t)lane_u64((unsigned long long)tt, 0);
#pragma unroll
            for (int rr = 16; rr < kWave; rr += 16) {
                const double od = lane_f64(dd, rr);
                const int64_t ot = (int64_t)lane_u64((unsigned long long)tt, rr);
                if (od < bd || (od == bd && ot < bt)) {
                    bd = od;
                    bt = ot;
                }
            }
            if (bt != INT64_MAX) {
                d = bd;
                j = bt;
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
    if (J.pearson) pout = isnan(pout) ? pout : isinf(pout) ? -INFINITY : 1.0 - pout * pout / (2.0 * (double)m);
    if (lane == 0) {
        gptr_w(J.P)[i] = (float)pout;
        gptr_w(J.I)[i] = iout;
    }
}

template <typename T, int KS, int NB, int KH, int NW, int WPE>
void launch_main(const MfmaJoinJob& one, const MfmaJoinJob* jobs, int njobs, int64_t blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((k_join_mfma<T, KS, NB, KH, NW, WPE>), dim3((unsigned)blocks), dim3(kWave * NW), 0, stream,
                       one, jobs, njobs);
}

// K: candidates per row and chunk
template <typename T, int KS, int NB, int NW, int WPE>
int launch_k(int K, const MfmaJoinJob& one, const MfmaJoinJob* jobs, int njobs, int64_t blocks, hipStream_t stream)
{
    switch (K) {
        case 4: launch_main<T, KS, NB, 4, NW, WPE>(one, jobs, njobs, blocks, stream); break;
        case 8: launch_main<T, KS, NB, 8, NW, WPE>(one, jobs, njobs, blocks, stream); break;
        default: return set_error(ABJ_EINVAL, "unsupported candidate count %d", K);
    }
    return ABJ_OK;
}

// Query blocks per wave (NB), waves per workgroup (NW) and the occupancy hint
// (waves per SIMD) of each k-step count, the fastest of the shapes timed on
// 262,144 x 262,144 random walks; must match mfma_shape() below.
template <typename T>
int launch_ks(int KS, int K, const MfmaJoinJob& one, const MfmaJoinJob* jobs, int njobs, int64_t blocks,
              hipStream_t stream)
{
    switch (KS) {
        case 1: return launch_k<T, 1, 1, 8, 4>(K, one, jobs, njobs, blocks, stream);
        case 2: return launch_k<T, 2, 1, 8, 4>(K, one, jobs, njobs, blocks, stream);
        case 4: return launch_k<T, 4, 2, 8, 2>(K, one, jobs, njobs, blocks, stream);
        case 8: return launch_k<T, 8, 2, 8, 2>(K, one, jobs, njobs, blocks, stream);
        case 16: return launch_k<T, 16, 1, 8, 2>(K, one, jobs, njobs, blocks, stream);
        default: return set_error(ABJ_EINVAL, "unsupported k-step count %d", KS);
    }
}

int launch_join(int tier, int KS, int K, const MfmaJoinJob& one, const MfmaJoinJob* jobs, int njobs, int64_t blocks,
                hipStream_t stream)
{
    ABJ_TRY(tier == ABJ_TIER_BF16 ? launch_ks<__bf16>(KS, K, one, jobs, njobs, blocks, stream)
                                  : launch_ks<_Float16>(KS, K, one, jobs, njobs, blocks, stream));
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

int launch_operand(int tier, const MfmaOpJob& one, const MfmaOpJob* jobs, int njobs, int64_t blocks,
                   hipStream_t stream)
{
    if (blocks <= 0) return ABJ_OK;
    if (tier == ABJ_TIER_BF16)
        hipLaunchKernelGGL(k_make_operand<__bf16>, dim3((unsigned)blocks), dim3(256), 0, stream, one, jobs, njobs);
    else
        hipLaunchKernelGGL(k_make_operand<_Float16>, dim3((unsigned)blocks), dim3(256), 0, stream, one, jobs, njobs);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

MfmaOpJob op_job(const SeriesDev& s, int ks_n, int64_t nblk, void* out, int64_t blk0)
{
    MfmaOpJob j{};
    j.xc = s.xc;
    j.mu = s.mu;
    j.sig = s.sig;
    j.flags = s.flags;
    j.out = out;
    j.W = s.W;
    j.nfrag = nblk * ks_n * kWave;
    j.blk0 = blk0;
    j.m = s.m;
    j.ks_n = ks_n;
    return j;
}

int64_t op_blocks(const MfmaOpJob& j) { return (j.nfrag + 255) / 256; }

MfmaJoinJob join_job(const MfmaPlan& p, const void* zq, const MfmaDictOp& dop, unsigned long long* cand,
                     int64_t blk0)
{
    MfmaJoinJob j{};
    j.zq = zq;
    j.zd = dop.zd;
    j.dmask = dop.dmask;
    j.cand = cand;
    j.nqblk = p.nqblk;
    j.ndblk = p.ndblk;
    j.npanels = p.npanels;
    j.blk_per_chunk = p.blk_per_chunk;
    j.nchunks = p.nchunks;
    j.blk0 = blk0;
    return j;
}

MfmaFinJob fin_job(const SeriesDev& A, const SeriesDev& B, const MfmaPlan& p, const unsigned long long* cand,
                   int refine, int pearson, float* P, int64_t* I, int64_t blk0)
{
    MfmaFinJob j{};
    j.axc = A.xc;
    j.amu = A.mu;
    j.asig = A.sig;
    j.aflags = A.flags;
    j.WA = A.W;
    j.bxc = B.xc;
    j.bmu = B.mu;
    j.bsig = B.sig;
    j.bflags = B.flags;
    j.bfirst = B.first;
    j.WB = B.W;
    j.cand = cand;
    j.P = P;
    j.I = I;
    j.blk0 = blk0;
    j.ncand = (int32_t)(p.nchunks * p.K);
    j.keep = p.keep;
    j.m = A.m;
    j.refine = refine;
    j.pearson = pearson;
    return j;
}

int64_t fin_blocks(const MfmaFinJob& j) { return (j.WA + kFinRows - 1) / kFinRows; }

}  // namespace

// NB and NW of each k-step count (see launch_ks).
static void mfma_shape(int KS, int* nb, int* nw)
{
    *nb = KS == 4 || KS == 8 ? 2 : 1;
    *nw = 8;
}

int mfma_plan(int64_t WA, int64_t WB, int32_t m, int tier, int refine_k, MfmaPlan* p)
{
    const int mp = (m + 15) / 16;
    int KS;
    if (mp <= 1) KS = 1;
    else if (mp <= 2) KS = 2;
    else if (mp <= 4) KS = 4;
    else if (mp <= 8) KS = 8;
    else if (mp <= 16) KS = 16;
    else return set_error(ABJ_EINVAL, "the BF16/FP16 tiers support m <= 256 (got %d)", m);
    // keep: distinct picks re-checked per row; K: candidates per row and chunk
    // (at least 4: short windows on quasi-periodic series have many near-equal
    // 16-bit scores, and fewer candidates missed the best there)
    int keep = refine_k <= 0 ? 4 : refine_k;
    keep = keep <= 1 ? 1 : keep <= 2 ? 2 : keep <= 4 ? 4 : 8;
    const int K = keep <= 4 ? 4 : 8;
    int NB, NW;
    mfma_shape(KS, &NB, &NW);
    p->tier = tier;
    p->KS = KS;
    p->K = K;
    p->keep = keep;
    p->nqblk = (WA + 31) / 32;
    p->ndblk = (WB + 31) / 32;
    const int64_t qblk_per_panel = (int64_t)NW * NB;
    p->npanels = (p->nqblk + qblk_per_panel - 1) / qblk_per_panel;
    // split the dictionary sweep until the workgroups fill the chip once (two
    // 8-wave workgroups per CU at KS <= 2, one with the 64 KB stages of KS >= 4:
    // 512 or 256 on 256 CUs), but keep at least 64 blocks (2,048 windows) per
    // chunk: a shorter sweep spends more of its blocks before its top-K
    // thresholds settle, when nearly every block takes the insert path
    const int64_t fill = KS <= 2 ? 512 : 256;
    int64_t nchunks = 1;
    while (p->npanels * nchunks < fill && (p->ndblk + nchunks * 2 - 1) / (nchunks * 2) >= 64) nchunks *= 2;
    while (nchunks * K > 512) nchunks /= 2;  // the re-check reads at most 512 candidates per row
    // a reference shorter than m has no block: one empty chunk (no sweep)
    p->blk_per_chunk = p->ndblk > 0 ? (p->ndblk + nchunks - 1) / nchunks : 1;
    p->nchunks = p->ndblk > 0 ? (p->ndblk + p->blk_per_chunk - 1) / p->blk_per_chunk : 1;
    return ABJ_OK;
}

size_t mfma_query_bytes(const MfmaPlan& p)
{
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return al((size_t)p.nqblk * p.KS * kWave * 16) +          // query operand
           al((size_t)p.nqblk * 32 * p.nchunks * p.K * 8);    // candidates
}

size_t mfma_dict_bytes(const MfmaPlan& p)
{
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return al((size_t)p.ndblk * p.KS * kWave * 16) +  // dictionary operand
           al((size_t)p.ndblk * 4);                   // block masks
}

int mfma_dict_build(const SeriesDev& B, const MfmaPlan& p, Arena& ar, MfmaDictOp* op, hipStream_t stream)
{
    void* zd = ar.take<char>((size_t)p.ndblk * p.KS * kWave * 16);
    uint32_t* dmask = ar.take<uint32_t>((size_t)p.ndblk);
    op->zd = zd;
    op->dmask = dmask;
    if (B.W <= 0 || p.ndblk <= 0) return ABJ_OK;
    const MfmaOpJob oj = op_job(B, p.KS, p.ndblk, zd, 0);
    ABJ_TRY(launch_operand(p.tier, oj, nullptr, 1, op_blocks(oj), stream));
    hipLaunchKernelGGL(k_block_mask, dim3((unsigned)((p.ndblk + 255) / 256)), dim3(256), 0, stream, B.flags, B.W,
                       p.ndblk, dmask);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

int join_mfma_run(const SeriesDev& A, const SeriesDev& B, const MfmaPlan& p, int refine, int pearson, float* P,
                  int64_t* I, Arena& ar, hipStream_t stream, const MfmaDictOp* dop)
{
    void* zq = ar.take<char>((size_t)p.nqblk * p.KS * kWave * 16);
    unsigned long long* cand = ar.take<unsigned long long>((size_t)p.nqblk * 32 * p.nchunks * p.K);
    MfmaDictOp own;
    if (!dop) {
        ABJ_TRY(mfma_dict_build(B, p, ar, &own, stream));
        dop = &own;
    }
    if (A.W <= 0) return ABJ_OK;
    if (B.W > 0) {
        const MfmaOpJob oj = op_job(A, p.KS, p.nqblk, zq, 0);
        ABJ_TRY(launch_operand(p.tier, oj, nullptr, 1, op_blocks(oj), stream));
        const MfmaJoinJob jj = join_job(p, zq, *dop, cand, 0);
        ProfMark mark;
        ABJ_TRY(prof_begin(&mark, stream));
        ABJ_TRY(launch_join(p.tier, p.KS, p.K, jj, nullptr, 1, p.npanels * p.nchunks, stream));
        ABJ_TRY(prof_end(&mark, stream, A.W * B.nvalid));
    } else {
        ABJ_TRY(fill_u64(cand, p.nqblk * 32 * p.nchunks * p.K, 0ull, stream));
    }
    const MfmaFinJob fj = fin_job(A, B, p, cand, refine, pearson, P, I, 0);
    if (p.keep <= 4)
        hipLaunchKernelGGL(k_finalize_topk<4>, dim3((unsigned)fin_blocks(fj)), dim3(kWave * kFinRows), 0, stream,
                           fj, nullptr, 1);
    else
        hipLaunchKernelGGL(k_finalize_topk<8>, dim3((unsigned)fin_blocks(fj)), dim3(kWave * kFinRows), 0, stream,
                           fj, nullptr, 1);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

size_t mfma_batch_table_bytes(int n)
{
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return al(sizeof(MfmaOpJob) * (size_t)n) + al(sizeof(MfmaJoinJob) * (size_t)n) + al(sizeof(MfmaFinJob) * (size_t)n);
}

void mfma_batch_prepare(const MfmaBatchItem* items, int n, int tier, int refine, int pearson, void* host,
                        MfmaBatchLaunch* L)
{
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    char* h = static_cast<char*>(host);
    *L = MfmaBatchLaunch();
    L->tier = tier;
    L->n = n;
    L->off_join = al(sizeof(MfmaOpJob) * (size_t)n);
    L->off_fin = L->off_join + al(sizeof(MfmaJoinJob) * (size_t)n);
    MfmaOpJob* oj = reinterpret_cast<MfmaOpJob*>(h);
    MfmaJoinJob* jj = reinterpret_cast<MfmaJoinJob*>(h + L->off_join);
    MfmaFinJob* fj = reinterpret_cast<MfmaFinJob*>(h + L->off_fin);
    // operand and re-check jobs in item order; join jobs grouped by (k steps,
    // candidates), one launch per group
    int64_t ob = 0, fb = 0;
    for (int a = 0; a < n; ++a) {
        const MfmaBatchItem& it = items[a];
        const bool sweep = it.B->W > 0 && it.A.W > 0;
        oj[a] = op_job(it.A, it.plan.KS, sweep ? it.plan.nqblk : 0, it.zq, ob);
        ob += op_blocks(oj[a]);
        fj[a] = fin_job(it.A, *it.B, it.plan, it.cand, refine, pearson, it.P, it.I, fb);
        fb += fin_blocks(fj[a]);
        if (fj[a].keep > L->max_keep) L->max_keep = fj[a].keep;
        if (!sweep && it.A.W > 0) L->empty.push_back(a);
        if (!sweep) continue;
        size_t g = 0;
        while (g < L->groups.size() && !(L->groups[g].ks == it.plan.KS && L->groups[g].k == it.plan.K)) ++g;
        if (g == L->groups.size()) L->groups.push_back({it.plan.KS, it.plan.K, 0, 0, 0});
    }
    L->op_blocks = ob;
    L->fin_blocks = fb;
    int w = 0;
    for (auto& gr : L->groups) {
        gr.first = w;
        int64_t blk = 0;
        for (int a = 0; a < n; ++a) {
            const MfmaBatchItem& it = items[a];
            if (it.B->W <= 0 || it.A.W <= 0 || it.plan.KS != gr.ks || it.plan.K != gr.k) continue;
            jj[w++] = join_job(it.plan, it.zq, it.dop, it.cand, blk);
            blk += it.plan.npanels * it.plan.nchunks;
        }
        gr.count = w - gr.first;
        gr.blocks = blk;
    }
}

int mfma_batch_launch(const MfmaBatchItem* items, const void* dev, const MfmaBatchLaunch& L, hipStream_t stream)
{
    const char* d = static_cast<const char*>(dev);
    for (int e : L.empty) {
        const MfmaBatchItem& it = items[e];
        ABJ_TRY(fill_u64(it.cand, it.plan.nqblk * 32 * it.plan.nchunks * it.plan.K, 0ull, stream));
    }
    ABJ_TRY(launch_operand(L.tier, MfmaOpJob{}, reinterpret_cast<const MfmaOpJob*>(d), L.n, L.op_blocks, stream));
    const MfmaJoinJob* jj = reinterpret_cast<const MfmaJoinJob*>(d + L.off_join);
    for (const auto& gr : L.groups)
        ABJ_TRY(launch_join(L.tier, gr.ks, gr.k, MfmaJoinJob{}, jj + gr.first, gr.count, gr.blocks, stream));
    if (L.fin_blocks > 0) {
        const auto* fj = reinterpret_cast<const MfmaFinJob*>(d + L.off_fin);
        if (L.max_keep <= 4)
            hipLaunchKernelGGL(k_finalize_topk<4>, dim3((unsigned)L.fin_blocks), dim3(kWave * kFinRows), 0, stream,
                               MfmaFinJob{}, fj, L.n);
        else
            hipLaunchKernelGGL(k_finalize_topk<8>, dim3((unsigned)L.fin_blocks), dim3(kWave * kFinRows), 0, stream,
                               MfmaFinJob{}, fj, L.n);
        ABJ_HIP(hipGetLastError());
    }
    return ABJ_OK;
}

}  // namespace abj
