// Resident dictionary and the serving scheduler.
//
// The inference phase of the paper (Alg. 2) joins every incoming series with
// the same learned dictionary, so the dictionary and its per-window statistics
// (one set per window length) stay in device memory.  The server turns a
// stream of join requests of uneven lengths into GPU launches:
//   * admission: a queued request is admitted (FIFO) when a slot is free and
//     its device footprint fits in the memory budget;
//   * continuous batching: every request admitted since the last launch goes
//     into the next launch; FP32 requests share ONE persistent tile kernel
//     (each request contributes its row-band x column-chunk tiles), so their
//     work overlaps on the device; two launches are kept in flight, in order
//     on one stream with a buffer set each, so the next batch is queued on
//     the device while one runs and a batch's epilogue never competes with
//     the next batch's tiles;
//   * completion: when a launch's event fires its slots and memory are
//     released, and a completion thread copies the results to the requests'
//     buffers and wakes the waiters.
// The host-simulation backend runs the same scheduler without any GPU call
// (execution time = pairs / configured rate) so that admission, ordering,
// cancellation and statistics can be tested on a machine without a GPU.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "abj_internal.hpp"

using namespace abj;

namespace abj {
struct DictM {
    int32_t m = 0;
    SeriesDev B;  // with the wide FP32 chunk list
    void* mem = nullptr;
    // the narrow FP32 chunk list (kFp32NarrowChunk windows at most)
    const int32_t* narrow_chunks = nullptr;
    int64_t narrow_nchunks = 0;
    int32_t narrow_w = 0;
    // the reference side of an FP32 join of WA query windows (fp32_wide_chunks)
    SeriesDev fp32_side(int64_t WA) const
    {
        SeriesDev b = B;
        if (!fp32_wide_chunks(WA, B.nchunks)) {
            b.chunks = narrow_chunks;
            b.nchunks = narrow_nchunks;
            b.chunk_w = narrow_w;
        }
        return b;
    }
    // the 16-bit tiers' dictionary side (operand fragments and block masks),
    // one per tier (0 = BF16, 1 = FP16), built at its first use
    mutable void* op_mem[2] = {nullptr, nullptr};
    mutable MfmaDictOp op[2];
    mutable hipEvent_t op_ready[2] = {nullptr, nullptr};
};
}  // namespace abj

struct abj_dict {
    int device = 0;
    int64_t n = 0;
    std::vector<int64_t> bounds;
    std::vector<int64_t> orig_start;  // per segment: its first sample in the source series
    double* x = nullptr;
    int64_t* dbounds = nullptr;
    int64_t* dorig = nullptr;  // orig_start on the device
    std::vector<DictM> per_m;
    mutable std::mutex op_mu;  // guards the lazily built 16-bit dictionary sides
    const DictM* find(int32_t m) const
    {
        for (auto& e : per_m)
            if (e.m == m) return &e;
        return nullptr;
    }
};

static void dict_release(abj_dict* d)
{
    if (!d) return;
    for (auto& e : d->per_m) {
        if (e.mem) (void)hipFree(e.mem);
        for (int t = 0; t < 2; ++t) {
            if (e.op_ready[t]) (void)hipEventDestroy(e.op_ready[t]);
            if (e.op_mem[t]) (void)hipFree(e.op_mem[t]);
        }
    }
    if (d->x) (void)hipFree(d->x);
    if (d->dbounds) (void)hipFree(d->dbounds);
    if (d->dorig) (void)hipFree(d->dorig);
    delete d;
}

namespace {
// The 16-bit dictionary side of window length e->m for `tier`: built on
// `stream` at its first use (one device allocation, kept until the dictionary
// is freed); a later caller on another stream waits for the build's event.
int dict_operand(const abj_dict* d, const DictM* e, int tier, hipStream_t stream, MfmaDictOp* out)
{
    const int t = tier == ABJ_TIER_BF16 ? 0 : 1;
    std::lock_guard<std::mutex> lk(d->op_mu);
    if (!e->op_mem[t]) {
        MfmaPlan p;
        ABJ_TRY(mfma_plan(1, e->B.W, e->m, tier, 0, &p));
        const size_t bytes = mfma_dict_bytes(p);
        void* mem = nullptr;
        if (hipMalloc(&mem, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(ABJ_ENOMEM, "dictionary operand of %zu bytes", bytes);
        }
        Arena ar(mem, bytes);
        MfmaDictOp op;
        hipEvent_t ev = nullptr;
        int rc = mfma_dict_build(e->B, p, ar, &op, stream);
        if (rc == ABJ_OK && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            rc = set_error(ABJ_EHIP, "event creation failed");
        if (rc == ABJ_OK && hipEventRecord(ev, stream) != hipSuccess) rc = set_error(ABJ_EHIP, "event record failed");
        if (rc != ABJ_OK) {
            (void)hipStreamSynchronize(stream);
            if (ev) (void)hipEventDestroy(ev);
            (void)hipFree(mem);
            return rc;
        }
        e->op_mem[t] = mem;
        e->op[t] = op;
        e->op_ready[t] = ev;
    } else {
        ABJ_HIP(hipStreamWaitEvent(stream, e->op_ready[t], 0));
    }
    *out = e->op[t];
    return ABJ_OK;
}
}  // namespace

extern "C" int abj_dict_create(const double* dict, int64_t n_dict, const int64_t* seg_bounds, int32_t n_seg,
                               const int64_t* orig_start, const int32_t* ms, int32_t n_ms, abj_dict** out)
{
    if (!out) return set_error(ABJ_EINVAL, "out is NULL");
    if (!dict) return set_error(ABJ_EINVAL, "dict is NULL");
    if (n_dict < 1 || n_dict > kMaxN) return set_error(ABJ_EINVAL, "n_dict out of range");
    ABJ_TRY(check_bounds(seg_bounds, n_seg, n_dict));
    if (orig_start)
        for (int32_t s = 0; s < n_seg; ++s)
            if (orig_start[s] < 0 || orig_start[s] > (int64_t(1) << 62))
                return set_error(ABJ_EINVAL, "orig_start[%d] = %lld out of range", s, (long long)orig_start[s]);
    if (!ms || n_ms < 1 || n_ms > 16) return set_error(ABJ_EINVAL, "n_ms must be in 1..16");
    for (int32_t a = 0; a < n_ms; ++a) {
        if (ms[a] < 2 || ms[a] > kMaxM) return set_error(ABJ_EINVAL, "window length %d out of range", ms[a]);
        for (int32_t b = 0; b < a; ++b)
            if (ms[a] == ms[b]) return set_error(ABJ_EINVAL, "window length %d given twice", ms[a]);
    }
    ABJ_TRY(ensure_device());
    hipPointerAttribute_t at;
    bool on_device = false;
    if (hipPointerGetAttributes(&at, dict) == hipSuccess)
        on_device = at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
    else
        (void)hipGetLastError();

    abj_dict* d = new abj_dict();
    ABJ_HIP(hipGetDevice(&d->device));
    d->n = n_dict;
    d->bounds.assign(seg_bounds, seg_bounds + n_seg + 1);
    if (orig_start)
        d->orig_start.assign(orig_start, orig_start + n_seg);
    else
        d->orig_start.assign(seg_bounds, seg_bounds + n_seg);  // the dictionary is its own source
    int rc = ABJ_OK;
    hipStream_t st = nullptr;
    do {
        if (hipMalloc(&d->x, sizeof(double) * (size_t)n_dict) != hipSuccess ||
            hipMalloc(&d->dbounds, sizeof(int64_t) * (size_t)(n_seg + 1)) != hipSuccess ||
            hipMalloc(&d->dorig, sizeof(int64_t) * (size_t)n_seg) != hipSuccess) {
            rc = set_error(ABJ_ENOMEM, "dictionary allocation failed");
            break;
        }
        if (hipMemcpy(d->x, dict, sizeof(double) * (size_t)n_dict,
                      on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d->dbounds, seg_bounds, sizeof(int64_t) * (size_t)(n_seg + 1), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(d->dorig, d->orig_start.data(), sizeof(int64_t) * (size_t)n_seg, hipMemcpyHostToDevice) !=
                hipSuccess) {
            rc = set_error(ABJ_EHIP, "dictionary copy failed");
            break;
        }
        if (hipStreamCreate(&st) != hipSuccess) {
            rc = set_error(ABJ_EHIP, "stream creation failed");
            break;
        }
        for (int32_t a = 0; a < n_ms && rc == ABJ_OK; ++a) {
            DictM e;
            e.m = ms[a];
            const int64_t W = n_dict >= e.m ? n_dict - e.m + 1 : 0;
            const size_t bytes = stats_scratch_bytes(n_dict, W) + fp32_chunk_bytes(n_seg, n_dict) +
                                 fp32_chunk_bytes(n_seg, n_dict, kFp32NarrowChunk);
            if (hipMalloc(&e.mem, bytes) != hipSuccess) {
                rc = set_error(ABJ_ENOMEM, "dictionary statistics allocation failed");
                break;
            }
            Arena ar(e.mem, bytes);
            stats_carve(ar, n_dict, e.m, &e.B);
            rc = fp32_chunks_upload(seg_bounds, n_seg, n_dict, e.m, ar, &e.B, st);
            if (rc != ABJ_OK) break;
            {
                SeriesDev narrow;
                rc = fp32_chunks_upload(seg_bounds, n_seg, n_dict, e.m, ar, &narrow, st, nullptr, kFp32NarrowChunk);
                if (rc != ABJ_OK) break;
                e.narrow_chunks = narrow.chunks;
                e.narrow_nchunks = narrow.nchunks;
                e.narrow_w = narrow.chunk_w;
            }
            for (int32_t sgi = 0; sgi < n_seg; ++sgi) {
                const int64_t len = seg_bounds[sgi + 1] - seg_bounds[sgi];
                if (len >= e.m) e.B.nvalid += len - e.m + 1;
            }
            rc = stats_compute(d->x, &e.B, d->dbounds, n_seg, ar, st);
            d->per_m.push_back(e);
        }
        if (rc == ABJ_OK && hipStreamSynchronize(st) != hipSuccess) rc = set_error(ABJ_EHIP, "statistics failed");
    } while (0);
    if (st) (void)hipStreamDestroy(st);
    if (rc != ABJ_OK) {
        dict_release(d);
        return rc;
    }
    *out = d;
    return ABJ_OK;
}

namespace {
// One lane per index: the segment holding I[i] by binary search over the
// dictionary's offsets, then the same offset from that segment's source start.
__global__ void k_source_index(const int64_t* __restrict__ I, int64_t n, const int64_t* __restrict__ bounds,
                               const int64_t* __restrict__ orig, int32_t n_seg, int64_t n_dict,
                               int64_t* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t v = I[i];
    if (v < 0 || v >= n_dict) {
        out[i] = -1;
        return;
    }
    int32_t lo = 0, hi = n_seg - 1;  // last segment whose start is <= v
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (bounds[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    out[i] = orig[lo] + (v - bounds[lo]);
}
}  // namespace

extern "C" int abj_dict_source_index(const abj_dict* d, const int64_t* I, int64_t n, int64_t* out,
                                     void* hip_stream)
{
    if (!d) return set_error(ABJ_EINVAL, "dictionary is NULL");
    if (n < 0 || n > kMaxN) return set_error(ABJ_EINVAL, "n out of range");
    if (n == 0) return ABJ_OK;
    ABJ_TRY(check_dev_buf(I, sizeof(int64_t) * (size_t)n, "I"));
    ABJ_TRY(check_dev_buf(out, sizeof(int64_t) * (size_t)n, "out"));
    ABJ_TRY(ensure_device());
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const int32_t n_seg = (int32_t)d->bounds.size() - 1;
    k_source_index<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(I, n, d->dbounds, d->dorig, n_seg, d->n, out);
    ABJ_HIP(hipGetLastError());
    return ABJ_OK;
}

extern "C" int abj_dict_free(abj_dict* d)
{
    if (!d) return set_error(ABJ_EINVAL, "dictionary is NULL");
    dict_release(d);
    return ABJ_OK;
}

extern "C" int ab_join_dict(const abj_dict* d, const double* query, int64_t n_query, int32_t m, float* P_AB,
                            int64_t* I_AB, const abj_opts* opts, void* hip_stream)
{
    if (!d) return set_error(ABJ_EINVAL, "dictionary is NULL");
    abj_opts o;
    ABJ_TRY(check_opts(opts, &o));
    const DictM* e = d->find(m);
    if (!e) return set_error(ABJ_EINVAL, "m = %d is not a window length of this dictionary", m);
    if (n_query < m || n_query > kMaxN)
        return set_error(ABJ_EINVAL, "n_query must be in [m, 2^31-1] (got %lld)", (long long)n_query);
    const int64_t WA = n_query - m + 1;
    ABJ_TRY(check_dev_buf(query, sizeof(double) * (size_t)n_query, "query"));
    ABJ_TRY(check_dev_buf(P_AB, sizeof(float) * (size_t)WA, "P_AB"));
    ABJ_TRY(check_dev_buf(I_AB, sizeof(int64_t) * (size_t)WA, "I_AB"));
    MfmaPlan plan;
    if (o.tier != ABJ_TIER_FP32) ABJ_TRY(mfma_plan(WA, e->B.W, m, o.tier, o.refine_k, &plan));
    ABJ_TRY(ensure_device());
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Arena ar(stream);
    // FP32: the chunk list for this join's size; per-chunk keys instead of
    // atomics when that list is short
    const SeriesDev B = o.tier == ABJ_TIER_FP32 ? e->fp32_side(WA) : e->B;
    const size_t part_bytes = o.tier == ABJ_TIER_FP32 && B.W > 0 ? fp32_partial_bytes(WA, B.nchunks) : 0;
    ar.reserve(query_scratch_bytes(n_query, m, B.W, o, plan) + part_bytes);
    ABJ_TRY(ar.commit());
    MfmaDictOp dop;
    if (o.tier != ABJ_TIER_FP32) ABJ_TRY(dict_operand(d, e, o.tier, stream, &dop));
    return join_query(query, n_query, m, B, o, plan, P_AB, I_AB, ar, stream, part_bytes,
                      o.tier != ABJ_TIER_FP32 ? &dop : nullptr);
}

// ---------------------------------------------------------------------------
// Server
// ---------------------------------------------------------------------------
namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2, kCanceled = 3 };

struct Req {
    uint64_t id = 0;
    std::vector<double> q;
    int64_t n = 0, W = 0;
    int32_t m = 0;
    const DictM* dm = nullptr;
    int state = kQueued;
    size_t mem = 0;
    MfmaPlan plan;
    abj_req_stats st{};
    std::vector<float> P;
    std::vector<int64_t> I;
    // zero-copy requests: the caller's buffers (then q, P and I stay empty)
    const double* q_borrowed = nullptr;
    float* P_out = nullptr;
    int64_t* I_out = nullptr;
    // device side, valid while running (inside the stream's work buffer)
    const double* dq = nullptr;
    char* work = nullptr;
    size_t work_bytes = 0;
    size_t off_P = 0, off_I = 0;  // offsets of the results in the staging buffer
    SeriesDev A;
    unsigned long long* keys = nullptr;
    float* dP = nullptr;
    int64_t* dI = nullptr;
};

struct Batch {
    std::vector<Req*> reqs;
    int set = 0;  // buffer set
    hipEvent_t ev = nullptr;
    char* dout = nullptr;  // results region of the work buffer
    size_t down = 0;
    char* hout = nullptr;  // pinned copy of the results region (from the server's pool)
    size_t hout_bytes = 0;
    double t_sim_done = 0;
    int status = ABJ_OK;
};

// Buffers of one batch in flight, kept for the server's lifetime and grown on
// demand: the device work buffer and pinned staging for the upload.  A set is
// reused only after its previous batch has finished on the device.
struct BufferSet {
    char* dev = nullptr;
    size_t dev_bytes = 0;
    char* hin = nullptr;
    size_t hin_bytes = 0;
};

}  // namespace

struct abj_server {
    const abj_dict* d = nullptr;
    abj_server_opts o{};
    abj_opts jo{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, std::unique_ptr<Req>> reqs;
    std::deque<uint64_t> queue;
    uint64_t next_id = 1;
    int active = 0;
    int64_t mem_used = 0;
    bool stop = false;
    std::thread th;
    hipStream_t stream = nullptr;
    BufferSet bufs[2];  // one set per batch in flight
    // batches finished on the device, whose results the completion thread
    // moves to the requests' buffers; pinned result buffers cycle through a pool
    std::mutex cmu;
    std::condition_variable cv_comp;
    std::deque<Batch> finished;
    bool comp_stop = false;
    std::vector<std::pair<char*, size_t>> out_pool;
    std::vector<char*> retired;  // outgrown pinned buffers, freed at destroy
    int64_t completing = 0;  // requests handed to the completion thread (under mu)
    std::thread comp;
    Clock::time_point t0;
    abj_server_stats stats{};
    double t_first_launch = -1, t_last_done = 0;
    std::vector<double> lat;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    bool sim() const { return o.backend == 1; }
};

namespace {

size_t req_bytes(const abj_server* s, int64_t n, int32_t m, MfmaPlan* plan)
{
    const int64_t W = n - m + 1;
    size_t b = 0;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    b += al((size_t)n * sizeof(double));  // query copy
    b += al((size_t)W * sizeof(float)) + al((size_t)W * sizeof(int64_t));  // outputs
    int64_t WB = 0;
    if (s->sim()) {
        WB = s->o.sim_dict_windows;
    } else {
        const DictM* e = s->d->find(m);
        WB = e ? e->B.W : 0;
    }
    if (s->jo.tier != ABJ_TIER_FP32 && !s->sim()) mfma_plan(W, WB, m, s->jo.tier, 0, plan);
    b += query_scratch_bytes(n, m, WB, s->jo, *plan);
    return b;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Buffers grow geometrically, without any device-wide synchronisation: the
// device buffer is replaced in stream order (the stream's previous batch is
// the last user of the old one), and an outgrown pinned buffer is retired
// until the server is destroyed (freeing pinned memory can wait for the whole
// device).  cap: the largest batch the admission rule allows.
int grow_device(char** p, size_t* have, size_t want, size_t cap, hipStream_t st)
{
    if (*have >= want) return ABJ_OK;
    const size_t bytes = std::max(want, std::min(cap, 2 * *have));
    if (*p) (void)hipFreeAsync(*p, st);
    *p = nullptr;
    *have = 0;
    if (hipMallocAsync(reinterpret_cast<void**>(p), bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(ABJ_ENOMEM, "server work buffer of %zu bytes", bytes);
    }
    *have = bytes;
    return ABJ_OK;
}

int grow_pinned(abj_server* s, char** p, size_t* have, size_t want)
{
    if (*have >= want) return ABJ_OK;
    const size_t bytes = std::max(want, std::max(2 * *have, (size_t)1 << 20));
    if (*p) {
        std::lock_guard<std::mutex> lk(s->cmu);
        s->retired.push_back(*p);
    }
    *p = nullptr;
    *have = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(p), bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(ABJ_ENOMEM, "server staging buffer of %zu bytes", bytes);
    }
    *have = bytes;
    return ABJ_OK;
}

// Launch one batch on the GPU.  The stream's work buffer is laid out as
//   [descriptor tables | queries] [P of every request | I of every request] [work regions]
// so that one copy brings the queries and descriptors in and one copy takes
// the results out.  FP32 requests then take four statistics launches, one
// persistent tile launch and one row-epilogue launch for the whole batch; the
// 16-bit tiers take the same statistics launches, one launch for every query
// operand, one matrix-core sweep per k-step count present in the batch (the
// window lengths of the requests) and one re-check launch.
int launch_batch(abj_server* s, Batch& b)
{
    hipStream_t st = s->stream;
    BufferSet& sb = s->bufs[b.set];
    const size_t k = b.reqs.size();
    const bool fp32 = s->jo.tier == ABJ_TIER_FP32;
    const size_t t_stats = al256(stats_job_bytes() * k), t_slots = al256(sizeof(Fp32Slot) * k),
                 t_fin = al256(finalize_job_bytes() * k);
    const size_t t_mfma = fp32 ? 0 : mfma_batch_table_bytes((int)k);
    const size_t tables = fp32 ? t_stats + t_slots + t_fin + kTileCounterBytes : t_stats + t_mfma;
    size_t qbytes = 0, pbytes = 0, ibytes = 0, work = 0;
    for (Req* r : b.reqs) {
        qbytes += al256(sizeof(double) * (size_t)r->n);
        pbytes += al256(sizeof(float) * (size_t)r->W);
        ibytes += al256(sizeof(int64_t) * (size_t)r->W);
        work += query_scratch_bytes(r->n, r->m, r->dm->B.W, s->jo, r->plan);
    }
    const size_t up = tables + qbytes, down = pbytes + ibytes;
    const size_t slots = (size_t)s->o.max_slots;
    const size_t cap = (size_t)s->o.mem_budget + al256(stats_job_bytes() * slots) + al256(sizeof(Fp32Slot) * slots) +
                       al256(finalize_job_bytes() * slots) + kTileCounterBytes +
                       (fp32 ? 0 : mfma_batch_table_bytes((int)slots));
    ABJ_TRY(grow_device(&sb.dev, &sb.dev_bytes, up + down + work, cap, st));
    ABJ_TRY(grow_pinned(s, &sb.hin, &sb.hin_bytes, up));
    {
        std::lock_guard<std::mutex> lk(s->cmu);
        if (!s->out_pool.empty()) {
            b.hout = s->out_pool.back().first;
            b.hout_bytes = s->out_pool.back().second;
            s->out_pool.pop_back();
        }
    }
    ABJ_TRY(grow_pinned(s, &b.hout, &b.hout_bytes, down));
    char* D = sb.dev;
    char* H = sb.hin;
    b.down = down;
    b.dout = D + up;

    size_t qo = tables, po = up, io = up + pbytes, wo = up + down;
    int64_t blk_sum = 0, blk_loc = 0, blk_win = 0, blk_fin = 0, tiles = 0, pairs = 0;
    int max_m = 2, max_w = 0;
    std::vector<MfmaBatchItem> items(fp32 ? 0 : k);
    for (size_t a = 0; a < k; ++a) {
        Req* r = b.reqs[a];
        memcpy(H + qo, r->q_borrowed ? r->q_borrowed : r->q.data(), sizeof(double) * (size_t)r->n);
        r->dq = reinterpret_cast<const double*>(D + qo);
        qo += al256(sizeof(double) * (size_t)r->n);
        r->dP = reinterpret_cast<float*>(D + po);
        r->off_P = po - up;
        po += al256(sizeof(float) * (size_t)r->W);
        r->dI = reinterpret_cast<int64_t*>(D + io);
        r->off_I = io - up;
        io += al256(sizeof(int64_t) * (size_t)r->W);
        r->work = D + wo;
        r->work_bytes = query_scratch_bytes(r->n, r->m, r->dm->B.W, s->jo, r->plan);
        wo += r->work_bytes;
        Arena ar(r->work, r->work_bytes);
        if (!fp32) {
            // 16-bit tiers: statistics in the batch's statistics launches,
            // then the query operand and candidates; the dictionary side of
            // the request's window length is built once and kept
            stats_carve_job(ar, r->dq, r->n, r->m, &r->A, nullptr, H + a * stats_job_bytes(), &blk_sum, &blk_loc,
                            &blk_win);
            MfmaBatchItem& it = items[a];
            it.A = r->A;
            it.B = &r->dm->B;
            it.plan = r->plan;
            it.zq = ar.take<char>((size_t)r->plan.nqblk * r->plan.KS * 64 * 16);
            it.cand = ar.take<unsigned long long>((size_t)r->plan.nqblk * 32 * r->plan.nchunks * r->plan.K);
            it.P = r->dP;
            it.I = r->dI;
            ABJ_TRY(dict_operand(s->d, r->dm, s->jo.tier, st, &it.dop));
            continue;
        }
        const size_t key_bytes = sizeof(unsigned long long) * (size_t)r->W;
        r->keys = ar.take<unsigned long long>(key_bytes / sizeof(unsigned long long));
        stats_carve_job(ar, r->dq, r->n, r->m, &r->A, r->keys, H + a * stats_job_bytes(), &blk_sum, &blk_loc,
                        &blk_win);
        Fp32Slot sl;
        const SeriesDev side = r->dm->fp32_side(r->W);
        fp32_slot(r->A, side, r->keys, tiles, &sl);
        max_w = std::max(max_w, (int)side.chunk_w);
        tiles += fp32_slot_tiles(sl);
        pairs += sl.pairs;
        max_m = std::max(max_m, (int)r->m);
        memcpy(H + t_stats + a * sizeof(Fp32Slot), &sl, sizeof(sl));
        finalize_job(r->A, r->dm->B, r->keys, r->dP, r->dI, H + t_stats + t_slots + a * finalize_job_bytes(),
                     &blk_fin);
    }
    if (fp32) memset(H + tables - kTileCounterBytes, 0, kTileCounterBytes);  // tile counters
    MfmaBatchLaunch L;
    if (!fp32) mfma_batch_prepare(items.data(), (int)k, s->jo.tier, 1, 0, H + t_stats, &L);
    ABJ_HIP(hipMemcpyAsync(D, H, up, hipMemcpyHostToDevice, st));
    if (fp32) {
        ABJ_TRY(stats_launch_many(D, (int)k, blk_sum, blk_loc, blk_win, st));
        ABJ_TRY(join_fp32_batch(reinterpret_cast<const Fp32Slot*>(D + t_stats), (int)k, tiles, max_m, max_w, pairs,
                                reinterpret_cast<unsigned long long*>(D + tables - kTileCounterBytes), st, false,
                                true));
        ABJ_TRY(finalize_launch_many(D + t_stats + t_slots, (int)k, blk_fin, st));
    } else {
        ABJ_TRY(stats_launch_many(D, (int)k, blk_sum, blk_loc, blk_win, st));
        ABJ_TRY(mfma_batch_launch(items.data(), D + t_stats, L, st));
    }
    ABJ_HIP(hipMemcpyAsync(b.hout, b.dout, down, hipMemcpyDeviceToHost, st));
    ABJ_HIP(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
    ABJ_HIP(hipEventRecord(b.ev, st));
    return ABJ_OK;
}

// Move a finished batch's results out of its pinned buffer (completion
// thread; the batch's event has fired).
int collect_batch(Batch& b)
{
    int rc = b.status;
    if (rc == ABJ_OK && b.ev && hipEventSynchronize(b.ev) != hipSuccess) rc = set_error(ABJ_EHIP, "batch failed");
    for (Req* r : b.reqs) {
        if (rc != ABJ_OK) continue;
        if (!r->P_out) {
            r->P.resize((size_t)r->W);
            r->I.resize((size_t)r->W);
        }
        memcpy(r->P_out ? r->P_out : r->P.data(), b.hout + r->off_P, sizeof(float) * (size_t)r->W);
        memcpy(r->I_out ? r->I_out : r->I.data(), b.hout + r->off_I, sizeof(int64_t) * (size_t)r->W);
    }
    if (b.ev) (void)hipEventDestroy(b.ev);
    b.ev = nullptr;
    return rc;
}

void sim_fill(abj_server* s, Req* r)
{
    if (!r->P_out) {
        r->P.resize((size_t)r->W);
        r->I.resize((size_t)r->W);
    }
    float* P = r->P_out ? r->P_out : r->P.data();
    int64_t* I = r->I_out ? r->I_out : r->I.data();
    const int64_t wb = s->o.sim_dict_windows > 0 ? s->o.sim_dict_windows : 1;
    for (int64_t i = 0; i < r->W; ++i) {
        P[i] = (float)((i * 7 + (int64_t)r->id) % 100) * 0.1f;
        I[i] = i % wb;
    }
}

void scheduler(abj_server* s)
{
    if (!s->sim()) (void)hipSetDevice(s->device);
    std::deque<Batch> inflight;
    int next_set = 0;
    int64_t batch_no = 0;
    for (;;) {
        Batch b;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            auto admissible = [&] {
                if (s->queue.empty() || s->active >= s->o.max_slots) return false;
                const Req* r = s->reqs[s->queue.front()].get();
                return s->mem_used + (int64_t)r->mem <= s->o.mem_budget;
            };
            if (inflight.empty()) {
                s->cv_work.wait(lk, [&] { return s->stop || admissible(); });
                if (s->stop && !admissible()) break;
            } else if (inflight.size() < 2 && !admissible()) {
                // keep polling the running launches, but wake at once for arrivals
                s->cv_work.wait_for(lk, std::chrono::microseconds(50), [&] { return s->stop || admissible(); });
            }
            if (inflight.size() < 2) {
                // half of the slots and of the budget per batch, so that the
                // next batch can be formed while this one runs
                const int slot_cap = std::max(1, s->o.max_slots / 2);
                const int64_t mem_cap = s->o.mem_budget / 2;
                int64_t batch_mem = 0;
                while (admissible()) {
                    const Req* nx = s->reqs[s->queue.front()].get();
                    if (!b.reqs.empty() &&
                        ((int)b.reqs.size() >= slot_cap || batch_mem + (int64_t)nx->mem > mem_cap))
                        break;
                    batch_mem += (int64_t)nx->mem;
                    Req* r = s->reqs[s->queue.front()].get();
                    s->queue.pop_front();
                    s->active += 1;
                    s->mem_used += (int64_t)r->mem;
                    r->state = kRunning;
                    r->st.t_admit = s->now();
                    b.reqs.push_back(r);
                }
            }
        }
        if (!b.reqs.empty()) {
            b.set = next_set;
            next_set ^= 1;
            const double t = s->now();
            int64_t pairs = 0;
            for (Req* r : b.reqs) {
                r->st.t_start = t;
                r->st.batch = (int32_t)batch_no;
                pairs += r->st.pairs;
            }
            ++batch_no;
            if (s->t_first_launch < 0) s->t_first_launch = t;
            if (s->sim()) {
                const double start = inflight.empty() ? t : std::max(t, inflight.back().t_sim_done);
                b.t_sim_done = start + (double)pairs / (s->o.sim_pairs_per_s > 0 ? s->o.sim_pairs_per_s : 1e12);
            } else {
                b.status = launch_batch(s, b);
            }
            inflight.push_back(std::move(b));
        }
        // completion: oldest launch first
        while (!inflight.empty()) {
            Batch& ob = inflight.front();
            bool done;
            if (s->sim()) {
                done = s->now() >= ob.t_sim_done;
                if (!done && inflight.size() >= 2) {
                    std::this_thread::sleep_for(std::chrono::duration<double>(ob.t_sim_done - s->now()));
                    done = true;
                }
            } else if (ob.status != ABJ_OK || !ob.ev) {
                done = true;
            } else {
                hipError_t q = hipEventQuery(ob.ev);
                if (q == hipErrorNotReady) (void)hipGetLastError();  // not an error: do not leave it pending
                done = q != hipErrorNotReady;
                if (!done && inflight.size() >= 2) {
                    (void)hipEventSynchronize(ob.ev);
                    done = true;
                }
            }
            if (!done) break;
            // the device is done with this batch: free its slots and memory
            // now, and let the completion thread deliver the results
            if (!s->sim() && ob.status != ABJ_OK) (void)hipStreamSynchronize(s->stream);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                const double t = s->now();
                for (Req* r : ob.reqs) {
                    r->st.t_device_done = t;
                    s->active -= 1;
                    s->mem_used -= (int64_t)r->mem;
                }
                s->completing += (int64_t)ob.reqs.size();
            }
            {
                std::lock_guard<std::mutex> lk(s->cmu);
                s->finished.push_back(std::move(ob));
            }
            s->cv_comp.notify_one();
            inflight.pop_front();
        }
    }
    for (int k = 0; k < 2; ++k) {
        BufferSet& sb = s->bufs[k];
        if (sb.dev) (void)hipFreeAsync(sb.dev, s->stream);
        if (s->stream) (void)hipStreamSynchronize(s->stream);
        if (sb.hin) (void)hipHostFree(sb.hin);
        sb = BufferSet();
    }
}

void completer(abj_server* s)
{
    if (!s->sim()) (void)hipSetDevice(s->device);
    for (;;) {
        Batch b;
        {
            std::unique_lock<std::mutex> lk(s->cmu);
            s->cv_comp.wait(lk, [&] { return s->comp_stop || !s->finished.empty(); });
            if (s->finished.empty()) break;
            b = std::move(s->finished.front());
            s->finished.pop_front();
        }
        int rc = b.status;
        if (s->sim()) {
            for (Req* r : b.reqs) sim_fill(s, r);
        } else {
            rc = collect_batch(b);
        }
        if (b.hout) {
            std::lock_guard<std::mutex> lk(s->cmu);
            s->out_pool.emplace_back(b.hout, b.hout_bytes);
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const double t = s->now();
            for (Req* r : b.reqs) {
                r->state = kDone;
                r->st.status = rc;
                r->st.t_done = t;
                r->q.clear();
                r->q.shrink_to_fit();
                if (rc == ABJ_OK) {
                    s->stats.completed += 1;
                    s->stats.pairs += r->st.pairs;
                    s->lat.push_back(r->st.t_done - r->st.t_arrive);
                }
            }
            s->completing -= (int64_t)b.reqs.size();
            s->stats.batches += 1;
            s->t_last_done = t;
        }
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" int abj_server_create(const abj_dict* d, const abj_server_opts* opts, abj_server** out)
{
    if (!opts || !out) return set_error(ABJ_EINVAL, "opts and out must not be NULL");
    const abj_server_opts& o = *opts;
    if (o.max_slots < 1) return set_error(ABJ_EINVAL, "max_slots must be >= 1");
    if (o.mem_budget <= 0) return set_error(ABJ_EINVAL, "mem_budget must be > 0");
    if (o.backend != 0 && o.backend != 1) return set_error(ABJ_EINVAL, "unknown backend %d", o.backend);
    abj_opts jo = {o.tier, 0, 0, 0};
    ABJ_TRY(check_opts(&jo, &jo));
    if (o.backend == 0 && !d) return set_error(ABJ_EINVAL, "the GPU backend needs a dictionary");
    if (o.backend == 1) {
        if (d) return set_error(ABJ_EINVAL, "the simulation backend takes no dictionary");
        if (o.sim_n_ms < 1 || o.sim_n_ms > 8) return set_error(ABJ_EINVAL, "sim_n_ms must be in 1..8");
    }
    abj_server* s = new abj_server();
    s->d = d;
    s->o = o;
    s->jo = jo;
    s->t0 = Clock::now();
    if (o.backend == 0) {
        int rc = ensure_device();
        if (rc == ABJ_OK && hipGetDevice(&s->device) != hipSuccess) rc = set_error(ABJ_EHIP, "hipGetDevice failed");
        if (rc == ABJ_OK && hipStreamCreate(&s->stream) != hipSuccess)
            rc = set_error(ABJ_EHIP, "stream creation failed");
        if (rc != ABJ_OK) {
            delete s;
            return rc;
        }
    }
    s->comp = std::thread(completer, s);
    s->th = std::thread(scheduler, s);
    *out = s;
    return ABJ_OK;
}

static int submit(abj_server* s, const double* query_host, int64_t n_query, int32_t m, float* P_out, int64_t* I_out,
                  uint64_t* req_id)
{
    if (!s || !query_host || !req_id) return set_error(ABJ_EINVAL, "NULL argument");
    int64_t WB = 0;
    bool m_ok = false;
    if (s->sim()) {
        for (int a = 0; a < s->o.sim_n_ms; ++a) m_ok |= s->o.sim_ms[a] == m;
        WB = s->o.sim_dict_windows;
    } else if (const DictM* e = s->d->find(m)) {
        m_ok = true;
        WB = e->B.W;
    }
    auto reject = [&](int code, const char* msg) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.rejected += 1;
        return set_error(code, "%s", msg);
    };
    if (!m_ok) return reject(ABJ_EINVAL, "m is not a window length of the dictionary");
    if (n_query < m || n_query > kMaxN) return reject(ABJ_EINVAL, "n_query must be >= m");
    auto r = std::make_unique<Req>();
    r->n = n_query;
    r->m = m;
    r->W = n_query - m + 1;
    r->dm = s->sim() ? nullptr : s->d->find(m);
    r->mem = req_bytes(s, n_query, m, &r->plan);
    if ((int64_t)r->mem > s->o.mem_budget) return reject(ABJ_ENOMEM, "request exceeds the memory budget");
    const int64_t nvalid = s->sim() ? WB : r->dm->B.nvalid;
    r->st.pairs = r->W * nvalid;
    if (P_out) {
        r->q_borrowed = query_host;
        r->P_out = P_out;
        r->I_out = I_out;
    } else {
        r->q.assign(query_host, query_host + n_query);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return set_error(ABJ_EINVAL, "server is shutting down");
        r->id = s->next_id++;
        r->st.t_arrive = s->now();
        r->st.batch = -1;
        *req_id = r->id;
        s->queue.push_back(r->id);
        s->stats.submitted += 1;
        s->reqs[r->id] = std::move(r);
    }
    s->cv_work.notify_all();
    return ABJ_OK;
}

extern "C" int abj_submit(abj_server* s, const double* query_host, int64_t n_query, int32_t m, uint64_t* req_id)
{
    return submit(s, query_host, n_query, m, nullptr, nullptr, req_id);
}

extern "C" int abj_submit_borrowed(abj_server* s, const double* query_host, int64_t n_query, int32_t m,
                                   float* P_host, int64_t* I_host, uint64_t* req_id)
{
    if (!P_host || !I_host) return set_error(ABJ_EINVAL, "P_host and I_host must not be NULL");
    return submit(s, query_host, n_query, m, P_host, I_host, req_id);
}

extern "C" int abj_wait(abj_server* s, uint64_t id, int32_t timeout_ms)
{
    if (!s) return set_error(ABJ_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_error(ABJ_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
    Req* r = it->second.get();
    auto fin = [&] { return r->state == kDone || r->state == kCanceled; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, fin);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), fin)) {
        return set_error(ABJ_ETIMEOUT, "request %llu not finished", (unsigned long long)id);
    }
    if (r->state == kCanceled) return set_error(ABJ_ECANCELED, "request %llu was canceled", (unsigned long long)id);
    return r->st.status;
}

extern "C" int abj_result(abj_server* s, uint64_t id, float* P_host, int64_t* I_host, abj_req_stats* st)
{
    if (!s) return set_error(ABJ_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_error(ABJ_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
    Req* r = it->second.get();
    if (r->state != kDone && r->state != kCanceled)
        return set_error(ABJ_EBUSY, "request %llu is not finished", (unsigned long long)id);
    if (st) *st = r->st;
    if (r->state == kDone && r->st.status == ABJ_OK) {
        const float* P = r->P_out ? r->P_out : r->P.data();
        const int64_t* I = r->I_out ? r->I_out : r->I.data();
        if (P_host && P_host != P) memcpy(P_host, P, sizeof(float) * (size_t)r->W);
        if (I_host && I_host != I) memcpy(I_host, I, sizeof(int64_t) * (size_t)r->W);
    }
    const int rc = r->state == kCanceled ? ABJ_ECANCELED : r->st.status;
    s->reqs.erase(it);
    if (rc != ABJ_OK) return set_error(rc, "request %llu did not complete", (unsigned long long)id);
    return ABJ_OK;
}

extern "C" int abj_cancel(abj_server* s, uint64_t id)
{
    if (!s) return set_error(ABJ_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return set_error(ABJ_ENOTFOUND, "unknown request %llu", (unsigned long long)id);
        Req* r = it->second.get();
        if (r->state != kQueued) return set_error(ABJ_EBUSY, "request %llu is already running", (unsigned long long)id);
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
        r->state = kCanceled;
        r->st.status = ABJ_ECANCELED;
        r->st.t_done = s->now();
        s->stats.canceled += 1;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
    return ABJ_OK;
}

extern "C" int abj_server_drain(abj_server* s, int32_t timeout_ms)
{
    if (!s) return set_error(ABJ_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto idle = [&] { return s->queue.empty() && s->active == 0 && s->completing == 0; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, idle);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle)) {
        return set_error(ABJ_ETIMEOUT, "server still busy");
    }
    return ABJ_OK;
}

extern "C" int abj_server_stats_get(abj_server* s, abj_server_stats* out)
{
    if (!s || !out) return set_error(ABJ_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    abj_server_stats st = s->stats;
    st.busy_s = s->t_first_launch >= 0 ? s->t_last_done - s->t_first_launch : 0.0;
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        size_t k = (size_t)ceil(p * (double)v.size()) - 1;
        return v[std::min(k, v.size() - 1)];
    };
    st.p50_s = pct(0.50);
    st.p99_s = pct(0.99);
    st.max_s = v.empty() ? 0.0 : v.back();
    *out = st;
    return ABJ_OK;
}

extern "C" int abj_server_destroy(abj_server* s)
{
    if (!s) return set_error(ABJ_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (uint64_t id : s->queue) {
            Req* r = s->reqs[id].get();
            r->state = kCanceled;
            r->st.status = ABJ_ECANCELED;
            s->stats.canceled += 1;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->th.joinable()) s->th.join();
    {
        std::lock_guard<std::mutex> lk(s->cmu);
        s->comp_stop = true;
    }
    s->cv_comp.notify_all();
    if (s->comp.joinable()) s->comp.join();
    for (auto& e : s->out_pool) (void)hipHostFree(e.first);
    for (char* p : s->retired) (void)hipHostFree(p);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return ABJ_OK;
}
