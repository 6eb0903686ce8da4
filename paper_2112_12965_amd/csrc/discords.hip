// Discords: greedy top-K of a profile, and exact top-K discords from the
// dictionary join (an upper bound of the exact profile, Lemma 1) with exact
// joins against the reference only where they can change the answer.
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

// (value, row) in one orderable 64-bit key: larger values win, ties go to
// the smaller row; 0 = no candidate.
__device__ inline unsigned long long disc_key(float v, int64_t i)
{
    unsigned u = __float_as_uint(v);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)i);
}

inline int64_t key_row(unsigned long long k) { return (int64_t)(0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull)); }

inline float key_value(unsigned long long k)
{
    unsigned u = (unsigned)(k >> 32);
    u = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float v;
    memcpy(&v, &u, sizeof(v));
    return v;
}

// One greedy step: rows within excl of the previous pick (prev, a key; 0 =
// none) die, then the best live finite row is folded into *out.
__global__ __launch_bounds__(kBlock) void k_disc_step(const float* __restrict__ P, int64_t W, int64_t excl,
                                                      const unsigned long long* __restrict__ prev,
                                                      uint8_t* __restrict__ dead, unsigned long long* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long key = 0;
    if (i < W) {
        bool d = dead[i];
        if (prev) {
            const unsigned long long pk = *prev;
            if (pk) {
                const int64_t c = (int64_t)(0xFFFFFFFFu - (unsigned)(pk & 0xFFFFFFFFull));
                if (i - c <= excl && c - i <= excl && !d) {
                    d = true;
                    dead[i] = 1;
                }
            }
        }
        const float v = P[i];
        if (!d && isfinite(v)) key = disc_key(v, i);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off, kWave);
        key = o > key ? o : key;
    }
    if ((threadIdx.x % kWave) == 0 && key) atomicMax(out, key);
}

// flags[band] = 1 for every band holding a row with P >= thr (NaN rows never).
__global__ __launch_bounds__(kBlock) void k_mark_bands(const float* __restrict__ P, int64_t W, float thr,
                                                       uint8_t* __restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < W && P[i] >= thr) flags[i / kFp32BandRows] = 1;
}

__global__ __launch_bounds__(kBlock) void k_fill_i64(int64_t* __restrict__ p, int64_t n, int64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Greedy top-K of P into keys[0..K) (device), dead: W bytes of scratch.
int greedy(const float* P, int64_t W, int32_t K, int64_t excl, uint8_t* dead, unsigned long long* keys,
           hipStream_t stream)
{
    ABJ_HIP(hipMemsetAsync(dead, 0, (size_t)W, stream));
    ABJ_TRY(fill_u64(keys, K, 0ull, stream));
    for (int32_t k = 0; k < K; ++k) {
        hipLaunchKernelGGL(k_disc_step, dim3(grid_of(W)), dim3(kBlock), 0, stream, P, W, excl,
                           k > 0 ? keys + k - 1 : nullptr, dead, keys + k);
        ABJ_HIP(hipGetLastError());
    }
    return ABJ_OK;
}

int read_keys(const unsigned long long* keys_dev, int32_t K, std::vector<unsigned long long>* out,
              hipStream_t stream)
{
    out->assign((size_t)K, 0ull);
    ABJ_HIP(hipMemcpyAsync(out->data(), keys_dev, sizeof(unsigned long long) * (size_t)K, hipMemcpyDeviceToHost,
                           stream));
    ABJ_HIP(hipStreamSynchronize(stream));
    return ABJ_OK;
}

}  // namespace

}  // namespace abj

using namespace abj;

extern "C" int topk_discords(const float* P, int64_t W, int32_t K, int64_t excl, int64_t* rows, float* values,
                             int32_t* n_found, void* hip_stream)
{
    if (W < 1 || W > kMaxN) return set_error(ABJ_EINVAL, "W must be in [1, 2^31-1] (got %lld)", (long long)W);
    if (K < 1) return set_error(ABJ_EINVAL, "K must be >= 1");
    if (excl < 0) return set_error(ABJ_EINVAL, "excl must be >= 0");
    if (!rows || !n_found) return set_error(ABJ_EINVAL, "rows / n_found are required");
    ABJ_TRY(check_dev_buf(P, sizeof(float) * (size_t)W, "P"));
    ABJ_TRY(ensure_device());
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Arena ar(stream);
    ar.reserve((size_t)W);
    ar.reserve(sizeof(unsigned long long) * (size_t)K);
    ABJ_TRY(ar.commit());
    uint8_t* dead = ar.take<uint8_t>((size_t)W);
    unsigned long long* keys = ar.take<unsigned long long>((size_t)K);
    ABJ_TRY(greedy(P, W, K, excl, dead, keys, stream));
    std::vector<unsigned long long> hk;
    ABJ_TRY(read_keys(keys, K, &hk, stream));
    int32_t n = 0;
    for (; n < K && hk[n]; ++n) {
        rows[n] = key_row(hk[n]);
        if (values) values[n] = key_value(hk[n]);
    }
    *n_found = n;
    return ABJ_OK;
}

extern "C" int discords(const double* query, int64_t n_query, int32_t m, const float* P_hat, double e_max,
                        const double* ref, int64_t n_ref, const int64_t* ref_bounds, int32_t n_ref_seg, int32_t K,
                        int64_t excl, int64_t* rows, float* values, int64_t* neighbors, int32_t* n_found,
                        abj_discord_info* info, void* hip_stream)
{
    // ---- validation ----
    if (m < 2 || m > kMaxM) return set_error(ABJ_EINVAL, "m must be in [2, %d] (got %d)", kMaxM, m);
    if (n_query < m || n_query > kMaxN)
        return set_error(ABJ_EINVAL, "n_query must be in [m, 2^31-1] (got %lld)", (long long)n_query);
    if (n_ref < 1 || n_ref > kMaxN)
        return set_error(ABJ_EINVAL, "n_ref must be in [1, 2^31-1] (got %lld)", (long long)n_ref);
    ABJ_TRY(check_bounds(ref_bounds, n_ref_seg, n_ref));
    if (K < 1) return set_error(ABJ_EINVAL, "K must be >= 1");
    if (!rows || !n_found) return set_error(ABJ_EINVAL, "rows / n_found are required");
    if (isnan(e_max)) return set_error(ABJ_EINVAL, "e_max is NaN");
    if (excl < 0) excl = m - 1;
    const int64_t W = n_query - m + 1;
    const int64_t WB = n_ref >= m ? n_ref - m + 1 : 0;
    ABJ_TRY(check_dev_buf(query, sizeof(double) * (size_t)n_query, "query"));
    ABJ_TRY(check_dev_buf(ref, sizeof(double) * (size_t)n_ref, "ref"));
    ABJ_TRY(check_dev_buf(P_hat, sizeof(float) * (size_t)W, "P_hat"));
    ABJ_TRY(ensure_device());

    // ---- workspace ----
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const int64_t nb = (W + kFp32BandRows - 1) / kFp32BandRows;
    const int32_t KK = std::max<int32_t>(K, 2);
    Arena ar(stream);
    ar.reserve(stats_scratch_bytes(n_ref, WB));
    ar.reserve(sizeof(int64_t) * (size_t)(n_ref_seg + 1));
    ar.reserve(fp32_chunk_bytes(n_ref_seg, n_ref));
    ar.reserve(stats_scratch_bytes(n_query, W));
    ar.reserve(sizeof(unsigned long long) * (size_t)W);  // keys
    ar.reserve(sizeof(float) * (size_t)W);               // mixed profile
    ar.reserve(sizeof(int64_t) * (size_t)W);             // exact neighbours
    ar.reserve((size_t)W);                               // dead rows
    ar.reserve((size_t)nb);                              // band flags
    ar.reserve(sizeof(unsigned long long) * (size_t)(KK + 4));
    ar.reserve(sizeof(Fp32Slot) * (size_t)nb);
    ar.reserve(kTileCounterBytes);                        // tile counters
    ABJ_TRY(ar.commit());
    SeriesDev B, A;
    stats_carve(ar, n_ref, m, &B);
    ABJ_TRY(fp32_chunks_upload(ref_bounds, n_ref_seg, n_ref, m, ar, &B, stream));
    for (int32_t s = 0; s < n_ref_seg; ++s) {
        const int64_t len = ref_bounds[s + 1] - ref_bounds[s];
        if (len >= m) B.nvalid += len - m + 1;
    }
    int64_t* dbounds = ar.take<int64_t>((size_t)(n_ref_seg + 1));
    ABJ_HIP(hipMemcpyAsync(dbounds, ref_bounds, sizeof(int64_t) * (size_t)(n_ref_seg + 1), hipMemcpyHostToDevice,
                           stream));
    ABJ_TRY(stats_compute(ref, &B, dbounds, n_ref_seg, ar, stream));
    stats_carve(ar, n_query, m, &A);
    ABJ_TRY(stats_compute(query, &A, nullptr, 0, ar, stream));
    unsigned long long* keys = ar.take<unsigned long long>((size_t)W);
    float* Pmix = ar.take<float>((size_t)W);
    int64_t* Iex = ar.take<int64_t>((size_t)W);
    uint8_t* dead = ar.take<uint8_t>((size_t)W);
    uint8_t* bflag = ar.take<uint8_t>((size_t)nb);
    unsigned long long* pk = ar.take<unsigned long long>((size_t)(KK + 4));
    Fp32Slot* dslots = ar.take<Fp32Slot>((size_t)nb);
    unsigned long long* counter = ar.take<unsigned long long>(kTileCounterBytes / 8);

    ABJ_HIP(hipMemcpyAsync(Pmix, P_hat, sizeof(float) * (size_t)W, hipMemcpyDeviceToDevice, stream));
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_of(W)), dim3(kBlock), 0, stream, Iex, W, (int64_t)-1);
    ABJ_HIP(hipGetLastError());
    ABJ_HIP(hipMemsetAsync(bflag, 0, (size_t)nb, stream));

    // ---- certification tests on P_hat ----
    std::vector<unsigned long long> hk;
    int32_t cert = 0;
    float top = NAN;
    ABJ_TRY(greedy(P_hat, W, 2, 0, dead, pk, stream));
    ABJ_TRY(read_keys(pk, 2, &hk, stream));
    if (hk[0]) {
        top = key_value(hk[0]);
        if (e_max >= 0.0 && (!hk[1] || (double)top - (double)key_value(hk[1]) > e_max)) cert |= 1;
    }
    ABJ_TRY(greedy(P_hat, W, 2, excl, dead, pk, stream));
    ABJ_TRY(read_keys(pk, 2, &hk, stream));
    if (hk[0] && e_max >= 0.0 && (!hk[1] || (double)key_value(hk[1]) < (double)top - e_max)) cert |= 2;

    // ---- round 0: the rows whose bound reaches the K-th greedy pick on P_hat
    // (the loop's first step), and of those only the ones that can hold the
    // top discord when e_max says so (Lemma 2: the top discord's exact value is
    // at least top - e_max).  Rows with no bound (+inf) are always taken.  The
    // loop below makes the result exact whatever this round takes. ----
    {
        std::vector<unsigned long long> first;
        ABJ_TRY(greedy(P_hat, W, K, excl, dead, pk, stream));
        ABJ_TRY(read_keys(pk, K, &first, stream));
        float thr = INFINITY;
        for (int32_t k = 0; k < K && first[k]; ++k) thr = key_value(first[k]);  // the last (lowest) pick
        if (!first[0]) thr = INFINITY;
        if (hk[0] && e_max >= 0.0) thr = std::max(thr, (float)((double)top - e_max));
        // rounding the threshold down keeps every row at or above it
        if (isfinite(thr)) thr = nextafterf(thr, -INFINITY);
        hipLaunchKernelGGL(k_mark_bands, dim3(grid_of(W)), dim3(kBlock), 0, stream, P_hat, W, thr, bflag);
        ABJ_HIP(hipGetLastError());
    }
    std::vector<uint8_t> done((size_t)nb, 0), hflag((size_t)nb);
    int64_t rows_exact = 0;
    int32_t rounds = 0;
    std::vector<unsigned long long> picks;
    for (;;) {
        // join the newly flagged bands
        ABJ_HIP(hipMemcpyAsync(hflag.data(), bflag, (size_t)nb, hipMemcpyDeviceToHost, stream));
        ABJ_HIP(hipStreamSynchronize(stream));
        std::vector<std::pair<int64_t, int64_t>> runs;  // [first band, last band + 1)
        for (int64_t b = 0; b < nb; ++b) {
            if (!hflag[b] || done[b]) continue;
            done[b] = 1;
            if (!runs.empty() && runs.back().second == b)
                runs.back().second = b + 1;
            else
                runs.push_back({b, b + 1});
        }
        if (!runs.empty()) {
            ++rounds;
            std::vector<Fp32Slot> slots;
            std::vector<SeriesDev> views;
            int64_t tiles = 0, pairs = 0;
            for (auto& r : runs) {
                const int64_t r0 = r.first * kFp32BandRows;
                const int64_t nr = std::min(W, r.second * kFp32BandRows) - r0;
                views.push_back(rows_view(A, r0, nr));
                Fp32Slot sl;
                fp32_slot(views.back(), B, keys + r0, tiles, &sl);
                tiles += fp32_slot_tiles(sl);
                pairs += sl.pairs;
                slots.push_back(sl);
                rows_exact += nr;
            }
            ABJ_TRY(fill_u64(keys, W, 0ull, stream));
            ABJ_HIP(hipMemcpyAsync(dslots, slots.data(), sizeof(Fp32Slot) * slots.size(), hipMemcpyHostToDevice,
                                   stream));
            ABJ_TRY(join_fp32_batch(dslots, (int)slots.size(), tiles, m, B.chunk_w, pairs, counter, stream));
            for (size_t k = 0; k < runs.size(); ++k) {
                const int64_t r0 = runs[k].first * kFp32BandRows;
                ABJ_TRY(finalize_launch(views[k], B, keys + r0, Pmix + r0, Iex + r0, stream));
            }
        }
        // greedy on the mixed profile
        ABJ_TRY(greedy(Pmix, W, K, excl, dead, pk, stream));
        ABJ_TRY(read_keys(pk, K, &picks, stream));
        bool all_exact = true;
        float lowest = INFINITY;
        for (int32_t k = 0; k < K && picks[k]; ++k) {
            const int64_t r = key_row(picks[k]);
            lowest = std::min(lowest, key_value(picks[k]));
            if (!done[(size_t)(r / kFp32BandRows)]) all_exact = false;
        }
        if (all_exact) break;
        // every row that could still beat a pick gets its exact value
        hipLaunchKernelGGL(k_mark_bands, dim3(grid_of(W)), dim3(kBlock), 0, stream, Pmix, W, lowest, bflag);
        ABJ_HIP(hipGetLastError());
    }

    // ---- outputs ----
    int32_t n = 0;
    for (; n < K && picks[n]; ++n) {
        const int64_t r = key_row(picks[n]);
        rows[n] = r;
        if (values) values[n] = key_value(picks[n]);
        if (neighbors) ABJ_HIP(hipMemcpyAsync(&neighbors[n], Iex + r, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    }
    ABJ_HIP(hipStreamSynchronize(stream));
    *n_found = n;
    if (info) {
        info->rows_exact = rows_exact;
        info->rounds = rounds;
        info->certified = cert;
    }
    return ABJ_OK;
}
