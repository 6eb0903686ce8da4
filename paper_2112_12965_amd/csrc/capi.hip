// extern "C" entry points of libabjoin.so: argument validation, workspace,
// and the launch sequence of each call.  See include/abjoin.h for the contract.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "abj_internal.hpp"

namespace abj {

namespace {
thread_local char g_err[512] = "";
std::mutex g_init_mu;
int g_inited_dev[64] = {0};

struct ProfRecord {
    hipEvent_t start, stop;
    int64_t pairs;
};
std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof;
}  // namespace

int prof_begin(ProfMark* mark, hipStream_t stream)
{
    mark->start = nullptr;
    if (!g_prof_on.load()) return ABJ_OK;
    ABJ_HIP(hipEventCreate(&mark->start));
    ABJ_HIP(hipEventRecord(mark->start, stream));
    return ABJ_OK;
}

int prof_end(ProfMark* mark, hipStream_t stream, int64_t pairs)
{
    if (!mark->start) return ABJ_OK;
    hipEvent_t stop;
    ABJ_HIP(hipEventCreate(&stop));
    ABJ_HIP(hipEventRecord(stop, stream));
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back({mark->start, stop, pairs});
    mark->start = nullptr;
    return ABJ_OK;
}

int set_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

Arena::~Arena()
{
    if (base_ && !external_) (void)hipFreeAsync(base_, stream_);
}

void Arena::abort_overflow(size_t want, size_t have)
{
    fprintf(stderr, "abjoin: internal workspace overflow (%zu > %zu bytes)\n", want, have);
    abort();
}

int Arena::commit()
{
    if (need_ == 0 || external_) return ABJ_OK;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&base_), need_, stream_);
    if (e != hipSuccess) {
        base_ = nullptr;
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? ABJ_ENOMEM : ABJ_EHIP, "workspace of %zu bytes: %s", need_,
                         hipGetErrorString(e));
    }
    return ABJ_OK;
}

int ensure_device()
{
    int dev = 0;
    ABJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(ABJ_EHIP, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (!g_inited_dev[dev]) {
        // Keep stream-ordered workspace cached between calls instead of
        // releasing it at every synchronisation.
        hipMemPool_t pool;
        ABJ_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
        uint64_t thr = ~0ull;
        ABJ_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
        g_inited_dev[dev] = 1;
    }
    return ABJ_OK;
}

// Checks that [p, p + bytes) lies inside one device (or managed) allocation.
int check_dev_buf(const void* p, size_t bytes, const char* name)
{
    if (!p) return set_error(ABJ_EINVAL, "%s is NULL", name);
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ABJ_EINVAL, "%s is not device memory", name);
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return set_error(ABJ_EINVAL, "%s is not device memory", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return ABJ_OK;  // range unknown (e.g. managed): trust the caller
    }
    const char* b = reinterpret_cast<const char*>(base);
    const char* q = reinterpret_cast<const char*>(p);
    if (q < b || (size_t)(q - b) + bytes > size)
        return set_error(ABJ_EINVAL, "%s: %zu bytes do not fit in its allocation", name, bytes);
    return ABJ_OK;
}

int check_bounds(const int64_t* sb, int32_t n_seg, int64_t n_dict)
{
    if (!sb) return set_error(ABJ_EINVAL, "seg_bounds is NULL");
    if (n_seg < 1) return set_error(ABJ_EINVAL, "n_seg must be >= 1 (got %d)", n_seg);
    if (sb[0] != 0) return set_error(ABJ_EINVAL, "seg_bounds[0] must be 0");
    if (sb[n_seg] != n_dict) return set_error(ABJ_EINVAL, "seg_bounds[n_seg] must equal n_dict");
    for (int32_t s = 0; s < n_seg; ++s)
        if (sb[s + 1] <= sb[s]) return set_error(ABJ_EINVAL, "seg_bounds must be strictly increasing (at %d)", s);
    return ABJ_OK;
}

int check_opts(const abj_opts* opts, abj_opts* out)
{
    abj_opts o = {ABJ_TIER_FP32, 0, 0, 0};
    if (opts) o = *opts;
    if (o.tier != ABJ_TIER_FP32 && o.tier != ABJ_TIER_BF16 && o.tier != ABJ_TIER_FP16)
        return set_error(ABJ_EINVAL, "unknown tier %d", o.tier);
    if (o.refine_k < 0 || o.refine_k > 8) return set_error(ABJ_EINVAL, "refine_k must be in 0..8");
    if ((o.flags & ~(ABJ_FLAG_NO_REFINE | ABJ_FLAG_PEARSON)) != 0 || o.reserved != 0)
        return set_error(ABJ_EINVAL, "unknown opts.flags bits or nonzero opts.reserved");
    *out = o;
    return ABJ_OK;
}

namespace {
size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

size_t query_scratch_bytes(int64_t n, int32_t m, int64_t WB, const abj_opts& o, const MfmaPlan& plan)
{
    (void)WB;
    const int64_t W = n - m + 1;
    size_t b = stats_scratch_bytes(n, W);
    b += al256(sizeof(unsigned long long) * (size_t)W);  // keys
    // upload region: statistics job, slot descriptor, tile counters
    b += al256(stats_job_bytes()) + al256(sizeof(Fp32Slot)) + kTileCounterBytes;
    if (o.tier != ABJ_TIER_FP32) b += mfma_query_bytes(plan);
    return b;
}

// The FP32 column chunks of a join of WA query windows against this
// reference: the wide list, or the narrow one when the wide one gives fewer
// tiles than the grid (fp32_wide_chunks).
std::vector<int32_t> fp32_join_chunks(const int64_t* bounds, int32_t n_seg, int64_t n, int32_t m, int64_t WA)
{
    std::vector<int32_t> c = fp32_chunk_list(bounds, n_seg, n, m);
    if (!fp32_wide_chunks(WA, (int64_t)c.size() / 2)) c = fp32_chunk_list(bounds, n_seg, n, m, kFp32NarrowChunk);
    return c;
}

size_t pair_scratch_bytes(int64_t n_query, int64_t n_ref, int32_t n_seg, int32_t m, const abj_opts& o,
                          const MfmaPlan& plan, size_t part_bytes)
{
    const int64_t WB = n_ref >= m ? n_ref - m + 1 : 0;
    // room for either chunk list (the narrow one is the longer)
    return stats_scratch_bytes(n_ref, WB) + fp32_chunk_bytes(n_seg, n_ref, kFp32NarrowChunk) +
           al256(stats_job_bytes()) + query_scratch_bytes(n_query, m, WB, o, plan) +
           (o.tier != ABJ_TIER_FP32 ? mfma_dict_bytes(plan) : 0) + part_bytes;
}

// The whole path of one join: the statistics of the query (and of the
// reference, when `ref` is given with its host segment bounds; else `Bres`
// holds them) in four launches, the pair scores and the row epilogue.  The
// descriptors, the reference's segment bounds and chunk list and the zeroed
// tile counter are built on the host and uploaded in one copy; the
// per-window statistics pass clears the FP32 keys.
// part_bytes: per-chunk keys (fp32_partial_bytes, reserved by the caller) or 0.
int join_run(const double* query, int64_t n, int32_t m, const double* ref, int64_t n_ref, const int64_t* ref_bounds,
             int32_t n_seg, const SeriesDev* Bres, const abj_opts& o, const MfmaPlan& plan, float* P, int64_t* I,
             Arena& ar, hipStream_t stream, size_t part_bytes, const MfmaDictOp* dop)
{
    const bool fp32 = o.tier == ABJ_TIER_FP32;
    const bool pearson = (o.flags & ABJ_FLAG_PEARSON) != 0;
    const int njobs = ref ? 2 : 1;
    const size_t jb = stats_job_bytes();
    std::vector<int32_t> chunks;
    if (ref) chunks = fp32_join_chunks(ref_bounds, n_seg, n_ref, m, n - m + 1);
    const size_t nb = ref ? (size_t)(n_seg + 1) : 0;
    const size_t o_chunks = sizeof(int64_t) * nb;
    const size_t o_jobs = al256(o_chunks + sizeof(int32_t) * chunks.size());
    const size_t o_slot = o_jobs + al256(jb * (size_t)njobs);
    const size_t o_counter = o_slot + al256(sizeof(Fp32Slot));
    const size_t up = o_counter + kTileCounterBytes;
    char* U = ar.take<char>(up);
    std::vector<char> h(up, 0);
    int64_t bs = 0, bl = 0, bw = 0;
    SeriesDev B;
    if (ref) {
        if (nb) memcpy(h.data(), ref_bounds, o_chunks);
        if (!chunks.empty()) memcpy(h.data() + o_chunks, chunks.data(), sizeof(int32_t) * chunks.size());
        stats_carve_job(ar, ref, n_ref, m, &B, nullptr, h.data() + o_jobs, &bs, &bl, &bw,
                        reinterpret_cast<const int64_t*>(U), n_seg);
        B.chunks = reinterpret_cast<const int32_t*>(U + o_chunks);
        B.nchunks = (int64_t)chunks.size() / 2;
        B.chunk_w = fp32_chunk_width(chunks);
        for (int32_t sgi = 0; sgi < n_seg; ++sgi) {
            const int64_t len = ref_bounds[sgi + 1] - ref_bounds[sgi];
            if (len >= m) B.nvalid += len - m + 1;
        }
    } else {
        B = *Bres;
    }
    SeriesDev A;
    const int64_t WA = n - m + 1;
    unsigned long long* keys = ar.take<unsigned long long>((size_t)WA);
    stats_carve_job(ar, query, n, m, &A, fp32 ? keys : nullptr, h.data() + o_jobs + (size_t)(njobs - 1) * jb, &bs,
                    &bl, &bw);
    Fp32Slot sl = {};
    unsigned long long* part = nullptr;
    if (fp32) {
        fp32_slot(A, B, keys, 0, &sl);
        if (part_bytes && part_bytes == fp32_partial_bytes(A.W, sl.nchunks)) {
            part = ar.take<unsigned long long>(part_bytes / sizeof(unsigned long long));
            sl.part = part;
        }
        memcpy(h.data() + o_slot, &sl, sizeof(sl));
    }
    ABJ_HIP(hipMemcpyAsync(U, h.data(), up, hipMemcpyHostToDevice, stream));
    ABJ_TRY(stats_launch_many(U + o_jobs, njobs, bs, bl, bw, stream));
    if (!fp32)
        return join_mfma_run(A, B, plan, !(o.flags & ABJ_FLAG_NO_REFINE), pearson, P, I, ar, stream, dop);
    ABJ_TRY(join_fp32_batch(reinterpret_cast<const Fp32Slot*>(U + o_slot), 1, fp32_slot_tiles(sl), m, B.chunk_w,
                            sl.pairs, reinterpret_cast<unsigned long long*>(U + o_counter), stream, false, true));
    if (part && sl.nchunks > kEpiloguePartsMax) {
        ABJ_TRY(fp32_reduce_parts(part, sl.nchunks, A.W, keys, stream));
        part = nullptr;
    }
    return finalize_launch(A, B, keys, P, I, stream, nullptr, -1, pearson, part, part ? (int)sl.nchunks : 0);
}

int join_query(const double* query, int64_t n, int32_t m, const SeriesDev& B, const abj_opts& o,
               const MfmaPlan& plan, float* P, int64_t* I, Arena& ar, hipStream_t stream, size_t part_bytes,
               const MfmaDictOp* dop)
{
    return join_run(query, n, m, nullptr, 0, nullptr, 0, &B, o, plan, P, I, ar, stream, part_bytes, dop);
}

int stats_export(const SeriesDev& s, double* mu, double* sig, uint8_t* flags, hipStream_t stream);

}  // namespace abj

using namespace abj;

extern "C" int abj_version(void) { return (0 << 16) | 1; }

extern "C" const char* abj_last_error(void) { return g_err; }

extern "C" int abj_init(int device_ordinal)
{
    int count = 0;
    ABJ_HIP(hipGetDeviceCount(&count));
    if (device_ordinal < 0 || device_ordinal >= count)
        return set_error(ABJ_EHIP, "device %d does not exist (%d visible)", device_ordinal, count);
    ABJ_HIP(hipSetDevice(device_ordinal));
    ABJ_TRY(ensure_device());
    // the device address of ab_join_noalloc's fixed workspace, once per device
    return noalloc_setup(nullptr);
}

extern "C" int abj_profile_enable(int on)
{
    g_prof_on.store(on != 0);
    return ABJ_OK;
}

extern "C" int abj_profile_read(double* kernel_ms, int64_t* launches, int64_t* pairs)
{
    std::vector<ProfRecord> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        recs.swap(g_prof);
    }
    double ms = 0.0;
    int64_t np = 0;
    int rc = ABJ_OK;
    for (auto& r : recs) {
        float e = 0.f;
        hipError_t st = hipEventSynchronize(r.stop);
        if (st == hipSuccess) st = hipEventElapsedTime(&e, r.start, r.stop);
        if (st != hipSuccess && rc == ABJ_OK) rc = set_error(ABJ_EHIP, "profile event: %s", hipGetErrorString(st));
        ms += e;
        np += r.pairs;
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    if (kernel_ms) *kernel_ms = ms;
    if (launches) *launches = (int64_t)recs.size();
    if (pairs) *pairs = np;
    return rc;
}

extern "C" int abj_window_stats(const double* x, int64_t n, int32_t m, double* mu, double* sigma, uint8_t* flags,
                                void* hip_stream)
{
    if (m < 2 || m > kMaxM) return set_error(ABJ_EINVAL, "m must be in [2, %d] (got %d)", kMaxM, m);
    if (n < m || n > kMaxN) return set_error(ABJ_EINVAL, "n must be in [m, 2^31-1] (got %lld)", (long long)n);
    const int64_t W = n - m + 1;
    ABJ_TRY(check_dev_buf(x, sizeof(double) * (size_t)n, "x"));
    ABJ_TRY(check_dev_buf(mu, sizeof(double) * (size_t)W, "mu"));
    ABJ_TRY(check_dev_buf(sigma, sizeof(double) * (size_t)W, "sigma"));
    ABJ_TRY(check_dev_buf(flags, (size_t)W, "flags"));
    ABJ_TRY(ensure_device());
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Arena ar(stream);
    ar.reserve(stats_scratch_bytes(n, W));
    ABJ_TRY(ar.commit());
    SeriesDev s;
    stats_carve(ar, n, m, &s);
    ABJ_TRY(stats_compute(x, &s, nullptr, 0, ar, stream));
    return stats_export(s, mu, sigma, flags, stream);
}

namespace abj {

int ab_join_validate(const double* query, int64_t n_query, const double* dict, int64_t n_dict,
                     const int64_t* seg_bounds, int32_t n_seg, int32_t m, float* P_AB, int64_t* I_AB,
                     const abj_opts* opts, JoinPrep* jp)
{
    abj_opts o;
    ABJ_TRY(check_opts(opts, &o));
    if (m < 2 || m > kMaxM) return set_error(ABJ_EINVAL, "m must be in [2, %d] (got %d)", kMaxM, m);
    if (n_query < m || n_query > kMaxN)
        return set_error(ABJ_EINVAL, "n_query must be in [m, 2^31-1] (got %lld)", (long long)n_query);
    if (n_dict < 1 || n_dict > kMaxN)
        return set_error(ABJ_EINVAL, "n_dict must be in [1, 2^31-1] (got %lld)", (long long)n_dict);
    ABJ_TRY(check_bounds(seg_bounds, n_seg, n_dict));
    const int64_t WA = n_query - m + 1;
    const int64_t WB = n_dict >= m ? n_dict - m + 1 : 0;
    ABJ_TRY(check_dev_buf(query, sizeof(double) * (size_t)n_query, "query"));
    ABJ_TRY(check_dev_buf(dict, sizeof(double) * (size_t)n_dict, "dict"));
    ABJ_TRY(check_dev_buf(P_AB, sizeof(float) * (size_t)WA, "P_AB"));
    ABJ_TRY(check_dev_buf(I_AB, sizeof(int64_t) * (size_t)WA, "I_AB"));
    MfmaPlan plan;
    if (o.tier != ABJ_TIER_FP32) ABJ_TRY(mfma_plan(WA, WB, m, o.tier, o.refine_k, &plan));
    // per-chunk keys instead of atomics when the chunk list is short
    size_t part_bytes = 0;
    if (o.tier == ABJ_TIER_FP32 && WB > 0)
        part_bytes = fp32_partial_bytes(WA, (int64_t)fp32_join_chunks(seg_bounds, n_seg, n_dict, m, WA).size() / 2);
    jp->o = o;
    jp->plan = plan;
    jp->part_bytes = part_bytes;
    jp->scratch = pair_scratch_bytes(n_query, n_dict, n_seg, m, o, plan, part_bytes);
    jp->scratch_atomic = pair_scratch_bytes(n_query, n_dict, n_seg, m, o, plan, 0);
    return ABJ_OK;
}

}  // namespace abj

extern "C" int ab_join(const double* query, int64_t n_query, const double* dict, int64_t n_dict,
                       const int64_t* seg_bounds, int32_t n_seg, int32_t m, float* P_AB, int64_t* I_AB,
                       const abj_opts* opts, void* hip_stream)
{
    // ---- validation: nothing is enqueued or written before this passes ----
    JoinPrep jp;
    ABJ_TRY(ab_join_validate(query, n_query, dict, n_dict, seg_bounds, n_seg, m, P_AB, I_AB, opts, &jp));
    ABJ_TRY(ensure_device());

    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Arena ar(stream);
    ar.reserve(jp.scratch);
    ABJ_TRY(ar.commit());
    return join_run(query, n_query, m, dict, n_dict, seg_bounds, n_seg, nullptr, jp.o, jp.plan, P_AB, I_AB, ar,
                    stream, jp.part_bytes);
}
