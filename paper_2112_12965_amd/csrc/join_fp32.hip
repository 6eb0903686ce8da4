// FP32 AB-join by incremental diagonal covariance (the pair loop of Alg. 2).
//
// For query window i and reference window j let
//   cov(i, j) = sum_k (a[i+k] - mu_a(i)) (b[j+k] - mu_b(j)).
// Then rho(i, j) = cov / (m sigma_a(i) sigma_b(j)) and the z-normalised
// distance is d = sqrt(2 m (1 - rho)), so the nearest neighbour of row i is the
// column with the largest cov(i, j) / sigma_b(j) (the row factor drops out).
// Along a diagonal the covariance obeys an O(1) update (derived from the
// definition; see the statistics kernels for df and dg):
//   cov(i+1, j+1) = cov(i, j) + df_a(i) dg_b(j) + df_b(j) dg_a(i).
//
// Work decomposition (one 64-lane wave per tile, no inter-wave traffic):
//   * a tile is 1024 query rows x one chunk of at most 2048 reference columns;
//     chunks come from a host-made list and lie inside one segment's valid
//     windows, so windows that cross a segment break are never swept;
//   * lane l owns rows i0 + 16 l .. i0 + 16 l + 15 and keeps their covariance
//     and running best score in registers;
//   * the wave walks the chunk's columns in order; a column's terms
//     {df_b, dg_b, w_b} are the same for all lanes, so they come from scalar
//     loads (weight w_b = 1/sigma_b, NaN for flat or non-finite windows);
//   * cov(i, j) needs cov(i-1, j-1): for a lane's first row that is the last
//     row of the lane below, moved across with one DPP wave_shr:1; lane 0 takes
//     the tile's top edge instead;
//   * the tile's left column and top row are exact FP64 dot products (so FP32
//     drift is bounded by the tile size);
//   * scores are folded with a max per row within each group of 16 columns and
//     only the group is recorded, so the sweep has no data-dependent branch;
//   * at the end each row's best (score, group) is merged across tiles with a
//     64-bit atomic max on an order-preserving key (ties -> first group), or
//     stored per chunk and reduced in the epilogue, which picks the row's
//     column within the group;
//   * windows shorter than kFp32SmallM take an exact path instead (FP64 dot
//     products per pair, small_m_tile below).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "abj_internal.hpp"

namespace abj {

namespace {

constexpr int kWave = 64;
constexpr int kR = 16;                  // query rows per lane
constexpr int kB = 16;                  // columns per sweep block (= candidate group of the epilogue)
constexpr int kBandRows = kR * kWave;   // query rows per tile
static_assert(kBandRows == kFp32BandRows, "band height is part of the engine's interface");
constexpr int kTC = 2048;               // reference columns per tile
constexpr int kQ = 16;                  // top-edge columns per lane in one pass
constexpr int kEdgePass = kQ * kWave;   // top-edge columns per pass
static_assert(kR == 16 && kQ == 16, "the edge dot products read the 16-row copies: lanes 16 samples apart");
static_assert(kTC % kEdgePass == 0, "whole top-edge passes");
constexpr int kDppWaveShr1 = 0x138;     // DPP control: whole-wave shift right by one lane
constexpr int kG = 16;                  // width of the FP64 edge dot-product groups
constexpr int64_t kGroupBands = 64;     // row bands per group of the tile order

// The slot's arrays live in global memory; saying so keeps their loads global
// (not flat) although the pointers come from a descriptor in memory.
typedef const __attribute__((address_space(1))) double* GDbl;

// acc[g] = sum_{k<m} w[k] * x[B + 16 lane + g + k] for g < G and a
// wave-uniform B, with x read from its 16-row copy xt (x[t] = xt[(t % 16) nb16
// + t / 16]): for one sample offset the 64 lanes, whose windows are 16 samples
// apart, read 64 consecutive doubles of one row, where the series itself would
// have them touch 64 cache lines.  x is read through a G-entry register window
// that slides by one sample per k and is refilled two samples per 2G FMAs.
template <int G>
__device__ inline void sliding_dots_rows(GDbl __restrict__ xt, int64_t nb16, int64_t B, const double* w, int m,
                                         double (&acc)[G])
{
    static_assert(G % 2 == 0, "pairs");
    const int lane = threadIdx.x % kWave;
    // sample B + 16 lane + s of this lane: row (B + s) mod 16, column (B + s) / 16 + lane
    // (a wave-uniform address plus the lane: the loads take a scalar base)
    auto at = [&](int64_t s) {
        const int64_t t = B + s;
        const GDbl __restrict__ p = xt + ((t & 15) * nb16 + (t >> 4));
        return p[lane];
    };
    double win[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        win[g] = at(g);
        acc[g] = 0.0;
    }
    int k0 = 0;
    // Invariant at the top of each block: win[s] holds sample k0 + s.
    for (; k0 + G <= m; k0 += G) {
#pragma unroll
        for (int kk = 0; kk < G; kk += 2) {
            const double n0 = at(k0 + kk + G), n1 = at(k0 + kk + G + 1);
            const double w0 = w[k0 + kk], w1 = w[k0 + kk + 1];
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = fma(w0, win[(kk + g) % G], acc[g]);
            win[kk] = n0;
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = fma(w1, win[(kk + 1 + g) % G], acc[g]);
            win[kk + 1] = n1;
        }
    }
    for (int k = k0; k < m; ++k) {
        const double wk = w[k];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = fma(wk, at(g + k), acc[g]);
    }
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Column records are read-only for a whole launch: reading them through the
// constant address space lets the wave-uniform loads of the sweep be scalar.
typedef float vf4 __attribute__((ext_vector_type(4)));  // same layout as float4
typedef float vf2 __attribute__((ext_vector_type(2)));  // same layout as float2
typedef const __attribute__((address_space(4))) vf4* ColPtr;
typedef const __attribute__((address_space(1))) vf2* GVf2;

__host__ __device__ inline size_t edge_offset(int m) { return ((size_t)m * sizeof(double) + 15) & ~size_t(15); }

__device__ inline unsigned long long pack_key(float s, int j)
{
    unsigned u = __float_as_uint(s);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)j);
}

// Score of logical row r at column j after the step that wrote it (slot
// (r - 1 - U) mod kR): cov times the column's weight (1 / sigma_j, or NaN for
// a reference window that cannot match: maxima drop NaN), and -inf for a
// self-join trivial match.  A product reads one scalar operand where a fused
// bias would need two, which one VALU instruction cannot take.
template <int U, bool kExcl>
__device__ __forceinline__ float step_score(const float (&S)[kR], int r, const vf4& cur, int64_t j, int64_t ibase,
                                            int64_t excl)
{
    float sc = S[(r - 1 - U) & (kR - 1)] * cur[2];
    if (kExcl) {
        // |j - i| <= excl is not a candidate (near the diagonal j - ibase is
        // small, so 32 bits suffice)
        const int rel = (int)(j - ibase) + (int)excl - r;
        if ((unsigned)rel <= 2u * (unsigned)excl) sc = -INFINITY;
    }
    return sc;
}

// One sweep step over column j.  On entry logical row r of this lane lives in
// register slot (r - U) mod kR; the step writes new row r over old row r-1
// (in place, no register moves), so on exit row r lives in slot (r - U - 1).
// blk[r] keeps the best score of row r over the steps of the current block.
template <int U, bool kGuard, bool kExcl>
__device__ __forceinline__ bool sweep_step(int64_t j, int64_t jend, ColPtr __restrict__ bcol, float e,
                                           float (&S)[kR], const float (&pf)[kR], const float (&pg)[kR],
                                           float (&blk)[kR], vf4& prev, int64_t ibase, int64_t excl)
{
    if (kGuard && j >= jend) return false;
    const vf4 cur = bcol[j];
#pragma unroll
    for (int r = kR - 1; r >= 1; --r) {
        float& c = S[(r - 1 - U) & (kR - 1)];
        c = fmaf(pg[r], prev[0], fmaf(pf[r], prev[1], c));
    }
    // row 0: lanes 1..63 take the old last row of the lane below (its slot is
    // the one row 0 overwrites, untouched by the loop above) and lane 0 zero,
    // plus e, which is the edge on lane 0 and zero elsewhere.  The compiler
    // folds the shift into the add (one DPP add into a fresh register, so no
    // row needs a move back at the block's end) only when the two are close
    // and the add's other operand is a whole register, hence their place here
    // and the empty asm.
    asm("" : "+v"(e));
    const float t = e + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(S[(kR - 1 - U) & (kR - 1)]),
                                                                   kDppWaveShr1, 0xf, 0xf, true));
    S[(kR - 1 - U) & (kR - 1)] = fmaf(pg[0], prev[0], fmaf(pf[0], prev[1], t));
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const float sc = step_score<U, kExcl>(S, r, cur, j, ibase, excl);
        blk[r] = U == 0 ? sc : fmaxf(blk[r], sc);
    }
    prev = cur;
    return true;
}

// kB consecutive steps starting at column jb (edge values e[0..kB) belong to
// columns jb .. jb+kB-1), then one update per row: if the block's best score
// beats the row's best, the row remembers the block (the first such block on
// ties).  The epilogue finds the winning column among the block's kB columns
// in FP64, so the sweep itself carries no per-column index and no branch.
template <bool kGuard, bool kExcl>
__device__ __forceinline__ void sweep_block(int64_t jb, int64_t jend, ColPtr __restrict__ bcol,
                                            const float (&e)[kB], float (&S)[kR], const float (&pf)[kR],
                                            const float (&pg)[kR], float (&best)[kR], int (&bidx)[kR],
                                            vf4& prev, int64_t ibase, int64_t excl)
{
    float blk[kR];
#define ABJ_STEP(u) \
    if (!sweep_step<u, kGuard, kExcl>(jb + u, jend, bcol, e[u], S, pf, pg, blk, prev, ibase, excl)) goto done;
    ABJ_STEP(0) ABJ_STEP(1) ABJ_STEP(2) ABJ_STEP(3) ABJ_STEP(4) ABJ_STEP(5) ABJ_STEP(6) ABJ_STEP(7)
    ABJ_STEP(8) ABJ_STEP(9) ABJ_STEP(10) ABJ_STEP(11) ABJ_STEP(12) ABJ_STEP(13) ABJ_STEP(14) ABJ_STEP(15)
#undef ABJ_STEP
done:
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const bool up = blk[r] > best[r];
        best[r] = up ? blk[r] : best[r];
        bidx[r] = up ? (int)jb : bidx[r];
    }
}

// One tile: rows band * 1024 .. +1023 of slot `sl`, the columns of one chunk.
// kExcl: the tile meets the self-join's trivial-match zone.
template <bool kExcl>
__device__ __forceinline__ void join_tile(const Fp32Slot& sl, int64_t band, int64_t chunk, double* lds)
{
    GDbl __restrict__ axc = (GDbl)sl.axc;
    GDbl __restrict__ amu = (GDbl)sl.amu;
    GVf2 __restrict__ adfdg = (GVf2)sl.adfdg;
    GDbl __restrict__ bxc = (GDbl)sl.bxc;
    GDbl __restrict__ axt = (GDbl)sl.axt;
    GDbl __restrict__ bxt = (GDbl)sl.bxt;
    GDbl __restrict__ bmu = (GDbl)sl.bmu;
    ColPtr __restrict__ bcol = (ColPtr)sl.bcol;
    unsigned long long* __restrict__ keys = sl.keys;
    const int64_t WA = sl.WA, WB = sl.WB;
    const int m = sl.m;

    double* wv = lds;                                  // m doubles: one centred window
    // then, 16-byte aligned, kB zeros, which lanes 1..63 read in place of the
    // edge, and the chunk's width + kB floats: edge[t] = cov(i0, j0 + 1 + t)
    float* zeros = reinterpret_cast<float*>(reinterpret_cast<char*>(lds) + edge_offset(m));
    float* edge = zeros + kB;
    if (threadIdx.x < kB) zeros[threadIdx.x] = 0.f;  // the edge's barriers below publish them

    const int lane = threadIdx.x;
    const int64_t i0 = band * kBandRows;
    const int32_t __attribute__((address_space(4)))* ch = (const int32_t __attribute__((address_space(4)))*)sl.chunks;
    const int64_t j0 = ch[2 * chunk];    // at most kTC columns, all valid (host-made list)
    const int64_t jend = ch[2 * chunk + 1];
    const int64_t ibase = i0 + (int64_t)lane * kR;

    // ---- top edge: cov(i0, j) for the tile's columns ------------------------
    {
        const double na = amu[i0];
        double part = 0.0;
        for (int k = lane; k < m; k += kWave) {
            const double v = axc[i0 + k] - na;
            wv[k] = v;
            part += v;
        }
        const double sa = wave_sum(part);
        __syncthreads();
        // kEdgePass columns per pass, kQ consecutive columns per lane
        for (int p = 0; p < kTC / kEdgePass; ++p) {
            const int64_t p0 = j0 + (int64_t)p * kEdgePass;
            if (p0 >= jend) break;  // uniform
            const int64_t cbase = p0 + (int64_t)lane * kQ;
#pragma unroll
            for (int h = 0; h < kQ; h += kG) {
                if (cbase + h >= jend) break;  // columns past the chunk are never swept
                double acc[kG];
                sliding_dots_rows<kG>(bxt, sl.bnb16, p0 + h, wv, m, acc);  // lane's columns from cbase + h
#pragma unroll
                for (int g = 0; g < kG; ++g) {
                    const int64_t j = cbase + h + g;
                    const double mb = j < WB ? bmu[j] : 0.0;
                    const int t = p * kEdgePass + lane * kQ + h + g - 1;  // edge[] starts at column j0 + 1
                    if (t >= 0) edge[t] = (float)(acc[g] - mb * sa);
                }
            }
        }
        __syncthreads();
    }

    float S[kR];
    // ---- left edge: cov(i, j0) for this lane's rows, exact in FP64 ----------
    {
        const double nb = bmu[j0];
        double part = 0.0;
        for (int k = lane; k < m; k += kWave) {
            const double v = bxc[j0 + k] - nb;
            wv[k] = v;
            part += v;
        }
        const double sb = wave_sum(part);
        __syncthreads();
        // cov = sum_k (a - mu_a) bhat_k = sum_k a bhat_k - mu_a sum_k bhat_k
#pragma unroll
        for (int h = 0; h < kR; h += kG) {
            double acc[kG];
            sliding_dots_rows<kG>(axt, sl.anb16, i0 + h, wv, m, acc);  // lane's rows from ibase + h
#pragma unroll
            for (int g = 0; g < kG; ++g) {
                const int64_t i = ibase + h + g;
                const double ma = i < WA ? amu[i] : 0.0;
                S[h + g] = (float)(acc[g] - ma * sb);
            }
        }
        __syncthreads();
    }
    // ---- main sweep -----------------------------------------------------------
    float pf[kR], pg[kR], best[kR];
    int bidx[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int64_t i = ibase + r;
        // terms of the step from row i-1 into row i; zero for the tile's top
        // row (lane 0, r 0) so that lane 0 takes the top edge unchanged
        vf2 t = {0.f, 0.f};
        if (i > i0 && i - 1 < WA - 1) t = adfdg[i - 1];
        pf[r] = t[0];
        pg[r] = t[1];
        best[r] = -INFINITY;
        bidx[r] = -1;
    }
    {
        // column j0 opens the first candidate group [j0, j0 + kB)
        const vf4 c0 = bcol[j0];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            float sc = fmaxf(S[r] * c0[2], -INFINITY);  // NaN (no match) -> -inf
            const int64_t dj = j0 - (ibase + r);
            if (kExcl && dj <= sl.excl && dj >= -sl.excl) sc = -INFINITY;
            best[r] = sc;
            bidx[r] = (int)j0;
        }
    }
    vf4 prev = bcol[j0];
    const int64_t nfull = (jend - j0 - 1) / kB;  // full blocks after column j0
    for (int64_t b = 0; b < nfull; ++b) {
        const int64_t jb = j0 + 1 + b * kB;
        float e[kB];
        const float4* e4 = reinterpret_cast<const float4*>(lane == 0 ? edge + b * kB : zeros);
#pragma unroll
        for (int q = 0; q < kB / 4; ++q) {
            const float4 v = e4[q];
            e[4 * q] = v.x;
            e[4 * q + 1] = v.y;
            e[4 * q + 2] = v.z;
            e[4 * q + 3] = v.w;
        }
        sweep_block<false, kExcl>(jb, jend, bcol, e, S, pf, pg, best, bidx, prev, ibase, sl.excl);
    }
    {
        const int64_t jb = j0 + 1 + nfull * kB;
        if (jb < jend) {
            float e[kB];
            const float* es = lane == 0 ? edge + nfull * kB : zeros;
#pragma unroll
            for (int u = 0; u < kB; ++u) e[u] = es[u];
            sweep_block<true, kExcl>(jb, jend, bcol, e, S, pf, pg, best, bidx, prev, ibase, sl.excl);
        }
    }
    if (sl.part) {
        // every tile writes each of its rows once: plain stores, no atomics
        unsigned long long* __restrict__ pc = sl.part + chunk * WA;
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int64_t i = ibase + r;
            if (i < WA) pc[i] = best[r] > -INFINITY ? pack_key(best[r], bidx[r]) : 0ull;
        }
    } else {
        // the row key only grows, so a tile whose key does not beat the value
        // read back needs no atomic: after the first tiles of a band most
        // rows are already settled, and the atomics (each a read and write
        // beyond the L2) drop from one per row and tile to about the number of
        // improvements.  A stale read only costs an unneeded atomic.
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int64_t i = ibase + r;
            if (i < WA && best[r] > -INFINITY) {
                const unsigned long long k = pack_key(best[r], bidx[r]);
                if (k > keys[i]) atomicMax(&keys[i], k);
            }
        }
    }
}

// Windows shorter than kFp32SmallM: one tile by FP64 dot products.  Lane l
// keeps its 16 rows two at a time, each as the window minus its mean (at most
// 7 samples, zero-padded); the columns stream through scalar loads of their 7
// samples and weight (1/sigma, NaN when the window cannot match), so the
// score sum_k (a_k - mu_a) b_k / sigma_b = m sigma_a rho needs no reference
// mean (the centred row sums to zero).  The row key carries rho in 32-bit
// fixed point (resolution 2^-31) and the column itself, not its group.
typedef const __attribute__((address_space(4))) double* CDbl;
constexpr int kSmallPad = kFp32SmallM - 1;  // samples per window register set

__device__ inline unsigned long long small_key(double rho, int64_t j)
{
    const double r = rho < -1.0 ? -1.0 : rho > 1.0 ? 1.0 : rho;
    const double f = (r + 1.0) * 2147483648.0;  // [0, 2^32]
    const unsigned hi = f >= 4294967295.0 ? 0xFFFFFFFFu : (unsigned)f;
    return ((unsigned long long)hi << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)j);
}

template <bool kExcl>
__device__ __forceinline__ void small_m_tile(const Fp32Slot& sl, int64_t band, int64_t chunk)
{
    GDbl __restrict__ axc = (GDbl)sl.axc;
    GDbl __restrict__ amu = (GDbl)sl.amu;
    GDbl __restrict__ asig = (GDbl)sl.asig;
    CDbl __restrict__ bxc = (CDbl)sl.bxc;
    ColPtr __restrict__ bcol = (ColPtr)sl.bcol;
    const int64_t WA = sl.WA;
    const int m = sl.m;
    const int lane = threadIdx.x;
    const int32_t __attribute__((address_space(4)))* ch = (const int32_t __attribute__((address_space(4)))*)sl.chunks;
    const int64_t j0 = ch[2 * chunk], jend = ch[2 * chunk + 1];
    const int64_t ibase = band * kBandRows + (int64_t)lane * kR;
#pragma unroll 1
    for (int r0 = 0; r0 < kR; r0 += 2) {
        double za[2][kSmallPad], best[2] = {-INFINITY, -INFINITY};
        int64_t bj[2] = {-1, -1};
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int64_t i = ibase + r0 + r;
            const int64_t ic = i < WA ? i : WA - 1;
            const double mu = amu[ic];
#pragma unroll
            for (int k = 0; k < kSmallPad; ++k) za[r][k] = k < m ? axc[ic + k] - mu : 0.0;
        }
        for (int64_t j = j0; j < jend; ++j) {
            const float w = bcol[j][2];
            double b[kSmallPad];
#pragma unroll
            for (int k = 0; k < kSmallPad; ++k) b[k] = bxc[j + k];  // < n + 6: the zero tail
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < kSmallPad; ++k) s = fma(za[r][k], b[k], s);
                double sc = s * (double)w;  // NaN for a window that cannot match
                if (kExcl) {
                    const int64_t d = j - (ibase + r0 + r);
                    if (d <= sl.excl && d >= -sl.excl) sc = -INFINITY;
                }
                if (sc > best[r]) {  // ties keep the smaller column
                    best[r] = sc;
                    bj[r] = j;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int64_t i = ibase + r0 + r;
            if (i >= WA) continue;
            const double rho = bj[r] >= 0 ? best[r] / ((double)m * asig[i]) : NAN;
            const unsigned long long k = rho >= -2.0 && rho <= 2.0 ? small_key(rho, bj[r]) : 0ull;
            if (sl.part) {
                sl.part[chunk * WA + i] = k;
            } else if (k && k > sl.keys[i]) {
                atomicMax(&sl.keys[i], k);
            }
        }
    }
}

// Persistent batch kernel: workgroup w (one wave) first joins tile w, then
// takes tiles from one of kTileQueues interleaved queues of the rest (queue q
// holds tiles grid + q + kTileQueues k; its counter sits on a line of its
// own), so that no single counter serialises the launch.  Device-wide atomics
// are carried out beyond the XCDs' L2 caches, so contended ones cost tens of
// nanoseconds each.  Every queue is finite, so every wave reaches the exit.  Tiles of different slots
// (requests) with different lengths and window lengths share the launch.
// kSelf: self-join launch; tiles that meet a slot's trivial-match zone take the
// masked sweep (a separate instantiation, so the AB-join kernel carries none of it).
template <bool kSelf>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4))) void k_join_fp32_batch(
    const Fp32Slot* __restrict__ slots, int nslots, int64_t ntiles, unsigned long long* __restrict__ counter)
{
    extern __shared__ double lds[];
    const unsigned long long grid = gridDim.x;
    const unsigned q = blockIdx.x % kTileQueues;
    unsigned long long* __restrict__ qc = counter + q * (128 / sizeof(unsigned long long));
    for (unsigned long long t = blockIdx.x;;) {
        if (t >= (unsigned long long)ntiles) break;
        // slot holding tile t: the last slot whose first tile is <= t
        int lo = 0, hi = nslots;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if ((unsigned long long)slots[mid].tile0 <= t) lo = mid;
            else hi = mid;
        }
        const Fp32Slot sl = slots[lo];
        const int64_t lt = (int64_t)t - sl.tile0;
        // a slot with more tiles than the grid runs its tiles in groups of
        // kGroupBands row bands: a group walks the chunks in order with all of
        // its bands per chunk, so the tiles in flight at once (a few thousand)
        // cover a block of bands x chunks whose series data stays in the
        // caches, instead of a few bands against every chunk (1M x 1M: 3.2x
        // less fetched from beyond the L2s).  A slot that fits in one round
        // keeps the plain band-major order, which measured 4% faster there.
        int64_t band, chunk;
        if (sl.nbands * sl.nchunks > (int64_t)grid) {
            const int64_t g = lt / (kGroupBands * sl.nchunks);
            const int64_t in = lt - g * kGroupBands * sl.nchunks;
            const int64_t nb = sl.nbands - g * kGroupBands < kGroupBands ? sl.nbands - g * kGroupBands : kGroupBands;
            chunk = in / nb;
            band = g * kGroupBands + (in - chunk * nb);
        } else {
            band = lt / sl.nchunks;
            chunk = lt - band * sl.nchunks;
        }
        if (kSelf) {
            // does the tile meet the band |j - i| <= excl?
            const int64_t i0 = band * kBandRows, i1 = i0 + kBandRows - 1;
            const int64_t j0 = sl.chunks[2 * chunk], j1 = sl.chunks[2 * chunk + 1] - 1;
            const bool zone = sl.excl >= 0 && j0 - i1 <= sl.excl && j1 - i0 >= -sl.excl;
            if (sl.m < kFp32SmallM)
                small_m_tile<true>(sl, band, chunk);
            else if (zone)
                join_tile<true>(sl, band, chunk, lds);
            else
                join_tile<false>(sl, band, chunk, lds);
        } else if (sl.m < kFp32SmallM) {
            small_m_tile<false>(sl, band, chunk);
        } else {
            join_tile<false>(sl, band, chunk, lds);
        }
        __syncthreads();  // the next tile reuses the LDS buffers
        // next tile of this wave's queue
        if (grid + q >= (unsigned long long)ntiles) break;  // the queue is empty
        unsigned long long k = 0;
        if (threadIdx.x == 0) k = atomicAdd(qc, 1ull);
        // wave-uniform tile index in scalar registers, so that everything derived
        // from it (slot, pointers, column loop) stays scalar
        k = __shfl(k, 0, kWave);
        const unsigned klo = __builtin_amdgcn_readfirstlane((unsigned)k);
        const unsigned khi = __builtin_amdgcn_readfirstlane((unsigned)(k >> 32));
        t = grid + q + kTileQueues * (((unsigned long long)khi << 32) | klo);
    }
}

// keys[i] = the largest of the per-chunk keys of row i (thread per row, so
// each load instruction reads consecutive rows of one chunk).
__global__ __launch_bounds__(256) void k_reduce_parts(const unsigned long long* __restrict__ part, int64_t nparts,
                                                       int64_t WA, unsigned long long* __restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= WA) return;
    unsigned long long k = 0;
    int64_t p = 0;
    for (; p + 8 <= nparts; p += 8) {
        unsigned long long v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(p + u) * WA + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) k = v[u] > k ? v[u] : k;
    }
    for (; p < nparts; ++p) {
        const unsigned long long v = part[p * WA + i];
        k = v > k ? v : k;
    }
    keys[i] = k;
}

}  // namespace

void fp32_slot(const SeriesDev& A, const SeriesDev& B, unsigned long long* keys, int64_t tile0, Fp32Slot* sl)
{
    sl->axc = A.xc;
    sl->amu = A.mu;
    sl->asig = A.sig;
    sl->adfdg = A.dfdg;
    sl->WA = A.W;
    sl->bxc = B.xc;
    sl->bmu = B.mu;
    sl->bcol = B.col;
    sl->WB = B.W;
    sl->axt = A.xt;
    sl->bxt = B.xt;
    sl->anb16 = A.nb16;
    sl->bnb16 = B.nb16;
    sl->m = A.m;
    sl->keys = keys;
    sl->part = nullptr;
    sl->tile0 = tile0;
    sl->nbands = A.W > 0 ? (A.W + kBandRows - 1) / kBandRows : 0;
    sl->chunks = B.chunks;
    sl->nchunks = B.W > 0 ? B.nchunks : 0;
    sl->pairs = A.W * B.nvalid;
    sl->excl = -1;
}

int64_t fp32_slot_tiles(const Fp32Slot& sl) { return sl.nbands * sl.nchunks; }

size_t fp32_partial_bytes(int64_t WA, int64_t nchunks)
{
    if (WA <= 0 || nchunks <= 1) return 0;
    const size_t b = sizeof(unsigned long long) * (size_t)WA * (size_t)nchunks;
    return b <= ((size_t)2 << 30) ? (b + 255) & ~size_t(255) : 0;
}

int fp32_reduce_parts(const unsigned long long* part, int64_t nparts, int64_t WA, unsigned long long* keys,
                      hipStream_t stream)
{
    if (WA <= 0) return ABJ_OK;
    const int64_t g = (WA + 255) / 256;
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)g), dim3(256), 0, stream, part, nparts, WA, keys);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

size_t fp32_chunk_bytes(int32_t n_seg, int64_t n, int32_t max_w)
{
    const int64_t cap = max_w > 0 && max_w < kTC ? max_w : kTC;
    const int64_t most = n / cap + (n_seg > 0 ? n_seg : 1) + 1;
    const size_t bounds = sizeof(int64_t) * (size_t)((n_seg > 0 ? n_seg : 0) + 1);
    return (bounds + sizeof(int32_t) * 2 * (size_t)most + 255) & ~size_t(255);
}

std::vector<int32_t> fp32_chunk_list(const int64_t* bounds, int32_t n_seg, int64_t n, int32_t m, int32_t max_w)
{
    std::vector<int32_t> c;
    const int64_t cap = max_w > 0 && max_w < kTC ? max_w : kTC;
    auto split = [&](int64_t a, int64_t cnt) {
        // equal widths, a multiple of 16 except the last, so that no tile is a sliver
        const int64_t k = (cnt + cap - 1) / cap;
        int64_t w = (cnt + k - 1) / k;
        w = std::min<int64_t>((w + kB - 1) / kB * kB, cap);
        for (int64_t s = 0; s < cnt; s += w) {
            c.push_back((int32_t)(a + s));
            c.push_back((int32_t)(a + std::min(cnt, s + w)));
        }
    };
    if (n_seg <= 0) {
        if (n >= m) split(0, n - m + 1);
    } else {
        for (int32_t s = 0; s < n_seg; ++s) {
            const int64_t len = bounds[s + 1] - bounds[s];
            if (len >= m) split(bounds[s], len - m + 1);
        }
    }
    return c;
}

int fp32_chunks_upload(const int64_t* bounds, int32_t n_seg, int64_t n, int32_t m, Arena& ar, SeriesDev* B,
                       hipStream_t stream, int64_t** dbounds, int32_t max_w)
{
    const std::vector<int32_t> c = fp32_chunk_list(bounds, n_seg, n, m, max_w);
    // one copy: the segment bounds (when asked for), then the chunk list
    const size_t nb = (dbounds && n_seg > 0) ? (size_t)(n_seg + 1) : 0;
    std::vector<int64_t> buf(nb + (c.size() + 1) / 2, 0);
    if (nb) memcpy(buf.data(), bounds, sizeof(int64_t) * nb);
    if (!c.empty()) memcpy(buf.data() + nb, c.data(), sizeof(int32_t) * c.size());
    int64_t* d = ar.take<int64_t>(buf.size() > 0 ? buf.size() : 1);
    if (dbounds) *dbounds = nb ? d : nullptr;
    B->chunks = reinterpret_cast<int32_t*>(d + nb);
    B->nchunks = (int64_t)c.size() / 2;
    B->chunk_w = fp32_chunk_width(c);
    if (!buf.empty())
        ABJ_HIP(hipMemcpyAsync(d, buf.data(), sizeof(int64_t) * buf.size(), hipMemcpyHostToDevice, stream));
    return ABJ_OK;
}

size_t fp32_lds_bytes(int max_m, int max_w)
{
    const int w = max_w > 0 && max_w < kTC ? max_w : kTC;
    return edge_offset(max_m) + sizeof(float) * (w + 2 * kB);
}

int join_fp32_batch(const Fp32Slot* slots_dev, int nslots, int64_t ntiles, int max_m, int max_w, int64_t pairs,
                    unsigned long long* counter_dev, hipStream_t stream, bool self, bool counter_zeroed)
{
    if (ntiles <= 0) return ABJ_OK;
    if (!counter_zeroed) ABJ_TRY(fill_u64(counter_dev, kTileCounterBytes / 8, 0ull, stream));
    // enough one-wave workgroups to fill every SIMD four deep, never more than tiles
    const int64_t grid = ntiles < kFp32Grid ? ntiles : kFp32Grid;
    ProfMark mark;
    ABJ_TRY(prof_begin(&mark, stream));
    if (self)
        hipLaunchKernelGGL(k_join_fp32_batch<true>, dim3((unsigned)grid), dim3(kWave), fp32_lds_bytes(max_m, max_w),
                           stream, slots_dev, nslots, ntiles, counter_dev);
    else
        hipLaunchKernelGGL(k_join_fp32_batch<false>, dim3((unsigned)grid), dim3(kWave), fp32_lds_bytes(max_m, max_w),
                           stream, slots_dev, nslots, ntiles, counter_dev);
    ABJ_HIP(hipGetLastError());
    return prof_end(&mark, stream, pairs);
}

}  // namespace abj
