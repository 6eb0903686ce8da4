// Internal declarations shared by the HIP sources of libabjoin.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "abjoin.h"

namespace abj {

// Records `code` with a printf-style message as the calling thread's last error
// and returns `code`.
int set_error(int code, const char* fmt, ...);

#define ABJ_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::abj::set_error(ABJ_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define ABJ_TRY(expr)              \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != ABJ_OK) return rc_; \
    } while (0)

// Samples of zero padding after every centred series copy, so that the
// register-window loads of the edge dot products never leave the buffer.
constexpr int64_t kSeriesPad = 4096;

// Flat-window threshold: population variance <= kFlatRel x series variance.
constexpr double kFlatRel = 1e-10;

// Window flag bits (also the public abj_window_stats flags).
constexpr uint8_t kFlagFlat = 1;
constexpr uint8_t kFlagBad = 2;
constexpr uint8_t kFlagInvalid = 4;  // reference window that crosses a segment break

// Device-side statistics of one series for one window length m.
struct SeriesDev {
    int64_t n = 0;         // samples
    int64_t W = 0;         // windows, n - m + 1 (0 if n < m)
    int32_t m = 0;
    int64_t nvalid = 0;    // reference side: windows inside one segment (host-computed)
    double* xc = nullptr;  // n + kSeriesPad: x - mean(x), non-finite -> 0, zero tail
    // the same samples (zero past n) in 16 rows: xt[(t % 16) * nb16 + t / 16] =
    // xc[t] for t < 16 nb16, so that 64 lanes reading samples 16 apart (the FP32
    // engine's edge dot products) read 64 consecutive doubles
    double* xt = nullptr;
    int64_t nb16 = 0;      // (n + kSeriesPad + 15) / 16
    double* mu = nullptr;  // W: window mean of xc
    double* sig = nullptr; // W: window population deviation
    float2* dfdg = nullptr;// W: {df(i), dg(i)} for the diagonal recurrence (last entry 0)
    float4* col = nullptr; // W: {df, dg, 1/sigma or NaN when excluded, 0}
    uint8_t* flags = nullptr;  // W
    double* scal = nullptr;    // device scalars: [0] mean, [1] variance, [2] finite count
    unsigned long long* first = nullptr;  // [0] first valid flat window, [1] first valid window (~0 = none)
    // reference side: column chunks of the FP32 engine, [chunks[2c], chunks[2c+1]),
    // each inside the valid windows of one segment (see fp32_chunks_upload)
    const int32_t* chunks = nullptr;
    int64_t nchunks = 0;
    int32_t chunk_w = 0;  // the widest chunk (windows), which sizes the tile kernel's LDS
};

// Stream-ordered scratch arena: one hipMallocAsync block carved into aligned
// pieces, released with hipFreeAsync on the same stream.
class Arena {
  public:
    explicit Arena(hipStream_t s) : stream_(s) {}
    // Carves from caller-owned memory of `bytes` bytes (commit() is then a no-op
    // and nothing is freed).
    Arena(void* base, size_t bytes) : base_(static_cast<char*>(base)), need_(bytes), external_(true) {}
    ~Arena();
    void reserve(size_t bytes) { need_ += (bytes + 255) & ~size_t(255); }
    int commit();
    template <class T>
    T* take(size_t count) {
        size_t b = (count * sizeof(T) + 255) & ~size_t(255);
        if (used_ + b > need_) abort_overflow(used_ + b, need_);
        char* p = base_ + used_;
        used_ += b;
        return reinterpret_cast<T*>(p);
    }
    size_t size() const { return need_; }

  private:
    [[noreturn]] static void abort_overflow(size_t want, size_t have);
    hipStream_t stream_ = nullptr;
    char* base_ = nullptr;
    size_t need_ = 0, used_ = 0;
    bool external_ = false;
};

// Bytes of scratch that stats_compute needs for a series of n samples.
size_t stats_scratch_bytes(int64_t n, int64_t W);

// Carves the SeriesDev arrays for (n, m) out of the arena (after commit()).
void stats_carve(Arena& a, int64_t n, int32_t m, SeriesDev* s);

// Runs the statistics pipeline: centred copy, FP64 prefix sums, per-window
// mean / deviation / flags, recurrence terms and column records.  When
// seg_bounds_dev is non-null the windows crossing a segment break are marked
// invalid and first-flat / first-valid indices are computed.
int stats_compute(const double* x, SeriesDev* s, const int64_t* seg_bounds_dev, int32_t n_seg, Arena& a,
                  hipStream_t stream);

// Statistics of many query series in four launches (a serving batch): each
// series' descriptor is written to job_host (stats_job_bytes() bytes) with its
// arrays carved from `ar`; the block counters accumulate the launch grids.
// clear: keys of the join to zero in the per-window pass (may be NULL).
// bounds_dev / n_seg: segment bounds of a reference series (device), which
// mask segment-crossing windows and find the first flat / valid window.
size_t stats_job_bytes();
void stats_carve_job(Arena& a, const double* x_dev, int64_t n, int32_t m, SeriesDev* s, unsigned long long* clear,
                     void* job_host, int64_t* blk_sum, int64_t* blk_loc, int64_t* blk_win,
                     const int64_t* bounds_dev = nullptr, int32_t n_seg = 0);
int stats_launch_many(const void* jobs_dev, int njobs, int64_t blk_sum, int64_t blk_loc, int64_t blk_win,
                      hipStream_t stream);

// Query rows per tile of the FP32 engine: slots whose rows start at a multiple
// of this share the engine's tiling of the whole series.
constexpr int64_t kFp32BandRows = 1024;

// Windows shorter than this take the FP32 engine's exact path: every pair's
// correlation from an FP64 dot product instead of the FP32 recurrence, whose
// absolute error is too coarse for the tiny distances of very short windows,
// and a row key that names the best column itself rather than its group.
constexpr int kFp32SmallM = 8;

// A view of rows [r0, r0 + rows) of the query statistics A, for joining or
// finishing a subset of bands (the copy behind xc keeps its zero tail).  r0
// is a multiple of 16 (the callers pass band starts), so that the 16-row copy
// is the same rows shifted by r0 / 16 columns, with the same row length.
inline SeriesDev rows_view(const SeriesDev& A, int64_t r0, int64_t rows)
{
    SeriesDev v = A;
    v.W = rows;
    v.n = rows + A.m - 1;
    v.xc = A.xc + r0;
    v.xt = A.xt + r0 / 16;
    v.mu = A.mu + r0;
    v.sig = A.sig + r0;
    v.dfdg = A.dfdg + r0;
    v.col = A.col + r0;
    v.flags = A.flags + r0;
    return v;
}

// One query series (a "slot") of an FP32 batch launch: its statistics, the
// reference statistics for the same m, its key array, and its tiles
// (nbands x nchunks, numbered from tile0 in the launch's tile list).
struct Fp32Slot {
    const double* axc;
    const double* amu;
    const double* asig;
    const float2* adfdg;
    int64_t WA;
    const double* bxc;
    const double* bmu;
    const float4* bcol;
    int64_t WB;
    const double* axt;  // the series in 16 rows (SeriesDev::xt) and their length
    const double* bxt;
    int64_t anb16, bnb16;
    const int32_t* chunks;  // reference column chunks [c0, c1) (device)
    unsigned long long* keys;
    // when set, tiles store their row keys here (one WA-entry row per chunk,
    // no atomics) and the row epilogue reduces them; else atomicMax into keys
    unsigned long long* part;
    int64_t tile0;
    int64_t nbands, nchunks;
    int64_t pairs;  // valid pairs (for timing records)
    int64_t excl;   // self-join trivial-match zone: pairs with |i - j| <= excl are skipped (-1: none)
    int32_t m;
    int32_t pad;
};
void fp32_slot(const SeriesDev& A, const SeriesDev& B, unsigned long long* keys, int64_t tile0, Fp32Slot* sl);
// Column chunks of a reference of n samples with these segments (host
// bounds; n_seg = 0 means one segment): every valid window of a segment
// falls in one of its chunks, chunks hold at most 2048 windows (max_w, when
// positive and smaller), and windows that cross a segment break belong to
// none, so the engine never sweeps them.  Carves the list from `ar` and
// copies it to the device for B; with dbounds the same copy also brings the
// segment bounds (*dbounds points at them).
size_t fp32_chunk_bytes(int32_t n_seg, int64_t n, int32_t max_w = 0);
// The chunk list itself (pairs [start, end) of reference windows), host side.
std::vector<int32_t> fp32_chunk_list(const int64_t* bounds, int32_t n_seg, int64_t n, int32_t m, int32_t max_w = 0);
int fp32_chunks_upload(const int64_t* bounds, int32_t n_seg, int64_t n, int32_t m, Arena& ar, SeriesDev* B,
                       hipStream_t stream, int64_t** dbounds = nullptr, int32_t max_w = 0);
// One wave sweeps a tile of 1024 query rows by one chunk; a tile's FP64 edges
// cost its rows plus its columns, so wider chunks cost fewer edge products per
// pair, but give fewer tiles.  A join takes the 2048-window chunks when they
// still give at least one tile per workgroup of the persistent grid
// (kFp32Grid), else chunks of at most kFp32NarrowChunk windows.  The choice
// depends on the join's own sizes only, so a request joins the same way on its
// own, through a resident dictionary and served in a batch.
constexpr int64_t kFp32Grid = 4096;
constexpr int32_t kFp32NarrowChunk = 1024;
inline bool fp32_wide_chunks(int64_t WA, int64_t wide_nchunks)
{
    return ((WA + kFp32BandRows - 1) / kFp32BandRows) * wide_nchunks >= kFp32Grid;
}
int64_t fp32_slot_tiles(const Fp32Slot& sl);
size_t fp32_lds_bytes(int max_m, int max_w);
// FP32 diagonal join of every tile of every slot (persistent workgroups, one
// atomic tile counter); writes one packed (score, group) key per query row.
// self: the slots are self-joins whose excl fields are honoured.
// counter_zeroed: the caller already cleared the tile counter on the stream.
// Bytes of the tile counters of one FP32 launch (zero before the launch).
constexpr int kTileQueues = 16;
constexpr size_t kTileCounterBytes = kTileQueues * 128;
// max_m / max_w: the largest window length and chunk width (chunk_w) of the
// slots, which size the LDS of the launch.
int join_fp32_batch(const Fp32Slot* slots_dev, int nslots, int64_t ntiles, int max_m, int max_w, int64_t pairs,
                    unsigned long long* counter_dev, hipStream_t stream, bool self = false,
                    bool counter_zeroed = false);
// The widest chunk of a chunk list (pairs [start, end)).
inline int32_t fp32_chunk_width(const std::vector<int32_t>& c)
{
    int32_t w = 0;
    for (size_t k = 0; k + 1 < c.size(); k += 2) w = std::max(w, c[k + 1] - c[k]);
    return w;
}

// Turns packed keys into P (FP64 re-check, flat conventions) and I; P64
// (optional) receives the same values unrounded.  excl >= 0 makes it a
// self-join epilogue: the flat conventions then only take reference windows
// outside |j - i| <= excl.  pearson: report 1 - d^2 / (2m) instead of d.
// part / nparts: per-chunk keys of the tiles (Fp32Slot::part), reduced here
// instead of reading `keys`.
int finalize_launch(const SeriesDev& A, const SeriesDev& B, const unsigned long long* keys, float* P, int64_t* I,
                    hipStream_t stream, double* P64 = nullptr, int64_t excl = -1, bool pearson = false,
                    const unsigned long long* part = nullptr, int nparts = 0);

// Bytes of per-chunk keys for a join of WA rows over `nchunks` column chunks,
// or 0 when the join should combine its tiles with atomics instead (the buffer
// would exceed 2 GiB: then there are so many tiles per row band that the
// atomics are spread over a long launch anyway).
size_t fp32_partial_bytes(int64_t WA, int64_t nchunks);
// Up to this many chunks the row epilogue reduces the per-chunk keys itself;
// beyond, fp32_reduce_parts writes the row keys first.
constexpr int64_t kEpiloguePartsMax = 64;
int fp32_reduce_parts(const unsigned long long* part, int64_t nparts, int64_t WA, unsigned long long* keys,
                      hipStream_t stream);

// Row epilogues of many joins in one launch (a serving batch): one descriptor
// per join (finalize_job_bytes() bytes, AB-join conventions), blocks counted in *blk.
size_t finalize_job_bytes();
void finalize_job(const SeriesDev& A, const SeriesDev& B, const unsigned long long* keys, float* P, int64_t* I,
                  void* job_host, int64_t* blk);
int finalize_launch_many(const void* jobs_dev, int njobs, int64_t blocks, hipStream_t stream);

int fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t stream);

// Launch plan of the BF16/FP16 tier.
struct MfmaPlan {
    int tier = 0;
    int KS = 0;                 // 16-wide k steps (m padded with zeros)
    int K = 0;                  // candidates stored per row and chunk
    int keep = 0;               // distinct candidates re-checked per row
    int64_t nqblk = 0, ndblk = 0;  // 32-window blocks of query / dictionary
    int64_t npanels = 0;        // query panels (one workgroup each per chunk)
    int64_t blk_per_chunk = 0, nchunks = 0;  // dictionary split of the sweep
};
int mfma_plan(int64_t WA, int64_t WB, int32_t m, int tier, int refine_k, MfmaPlan* p);
// Device bytes of the query side (16-bit operand, candidates) and of the
// dictionary side (16-bit operand, block masks) of a plan.
size_t mfma_query_bytes(const MfmaPlan& p);
size_t mfma_dict_bytes(const MfmaPlan& p);

// The dictionary side of the 16-bit tiers, built once per (window length,
// tier) for a resident dictionary or per call otherwise.
struct MfmaDictOp {
    const void* zd = nullptr;        // operand fragments (32-window blocks x k steps x 64 lanes x 16 B)
    const uint32_t* dmask = nullptr; // per block: bit r set = window 32 b + r can match
};
// Carves mfma_dict_bytes(p) from `ar` and enqueues the build on `stream`.
int mfma_dict_build(const SeriesDev& B, const MfmaPlan& p, Arena& ar, MfmaDictOp* op, hipStream_t stream);

// Operand, matrix-core sweep, FP64 re-check of the candidates (or, with
// refine = 0, the distance implied by the best 16-bit score), conventions.
// dop: a prebuilt dictionary side, or NULL to build it from `ar`.
int join_mfma_run(const SeriesDev& A, const SeriesDev& B, const MfmaPlan& p, int refine, int pearson, float* P,
                  int64_t* I, Arena& ar, hipStream_t stream, const MfmaDictOp* dop = nullptr);

// Job descriptors of the 16-bit tier's kernels: a one-shot join passes one by
// value, a serving batch uploads a table (blk0 = the job's first workgroup
// in its launch, ascending).
struct MfmaOpJob {
    const double* xc;
    const double* mu;
    const double* sig;
    const uint8_t* flags;
    void* out;
    int64_t W, nfrag, blk0;
    int32_t m, ks_n;
};
struct MfmaJoinJob {
    const void* zq;
    const void* zd;
    const uint32_t* dmask;
    unsigned long long* cand;
    int64_t nqblk, ndblk, npanels, blk_per_chunk, nchunks, blk0;
};
struct MfmaFinJob {
    const double *axc, *amu, *asig;
    const uint8_t* aflags;
    int64_t WA;
    const double *bxc, *bmu, *bsig;
    const uint8_t* bflags;
    const unsigned long long* bfirst;
    int64_t WB;
    const unsigned long long* cand;
    float* P;
    int64_t* I;
    int64_t blk0;
    int32_t ncand, keep, m, refine, pearson, pad;
};

// One query of a 16-bit serving batch: its statistics, the dictionary side
// for its window length, its plan and its device buffers.
struct MfmaBatchItem {
    SeriesDev A;
    const SeriesDev* B = nullptr;
    MfmaDictOp dop;
    MfmaPlan plan;
    void* zq = nullptr;                 // mfma_query_bytes(plan) bytes: operand, then candidates
    unsigned long long* cand = nullptr;
    float* P = nullptr;
    int64_t* I = nullptr;
};
struct MfmaBatchLaunch {
    struct Group {
        int ks, k, first, count;
        int64_t blocks;
    };
    int tier = 0, n = 0;
    std::vector<Group> groups;  // one sweep launch per (k steps, candidates)
    std::vector<int> empty;     // items whose dictionary has no window
    int64_t op_blocks = 0, fin_blocks = 0;
    int max_keep = 0;           // the largest re-check pick count of the items (sizes the re-check's stage)
    size_t off_join = 0, off_fin = 0;
};
// Device bytes of the job tables of n items.
size_t mfma_batch_table_bytes(int n);
// Writes the job tables to `host` (later copied to the device) and the launch shape to *L.
void mfma_batch_prepare(const MfmaBatchItem* items, int n, int tier, int refine, int pearson, void* host,
                        MfmaBatchLaunch* L);
// Enqueues the batch: every query operand in one launch, one sweep per group, every re-check in one launch.
int mfma_batch_launch(const MfmaBatchItem* items, const void* tables_dev, const MfmaBatchLaunch& L,
                      hipStream_t stream);

int ensure_device();

// The whole path of one join (see capi.hip): statistics of the query (and of
// `ref` with its host segment bounds, else `Bres` holds the reference), pair
// scores of the selected tier and row epilogue, all scratch from `ar`.
// part_bytes: per-chunk FP32 keys (fp32_partial_bytes) or 0 for atomics.
int join_run(const double* query, int64_t n, int32_t m, const double* ref, int64_t n_ref, const int64_t* ref_bounds,
             int32_t n_seg, const SeriesDev* Bres, const abj_opts& o, const MfmaPlan& plan, float* P, int64_t* I,
             Arena& ar, hipStream_t stream, size_t part_bytes = 0, const MfmaDictOp* dop = nullptr);

// ab_join's argument checks and plan: everything is checked before anything
// is enqueued.  scratch: workspace bytes of the join with per-chunk FP32
// keys (part_bytes of them); scratch_atomic: without them (atomic merge).
struct JoinPrep {
    abj_opts o;
    MfmaPlan plan;
    size_t part_bytes = 0;
    size_t scratch = 0, scratch_atomic = 0;
};
int ab_join_validate(const double* query, int64_t n_query, const double* dict, int64_t n_dict,
                     const int64_t* seg_bounds, int32_t n_seg, int32_t m, float* P_AB, int64_t* I_AB,
                     const abj_opts* opts, JoinPrep* jp);

// Device address of the fixed workspace of ab_join_noalloc on the current
// device (looked up once per device; *out may be NULL to only set it up).
int noalloc_setup(void** out);

// Argument checks shared by the entry points (set the error text).
int check_dev_buf(const void* p, size_t bytes, const char* name);
int check_bounds(const int64_t* sb, int32_t n_seg, int64_t n_dict);
int check_opts(const abj_opts* opts, abj_opts* out);
constexpr int32_t kMaxM = 4096;
constexpr int64_t kMaxN = (1LL << 31) - 1;

// Device bytes that join_query needs for one query of n samples (statistics,
// keys, the upload region and, in the 16-bit tiers, the query operand and
// candidates; the dictionary side comes prebuilt, see join_query).
size_t query_scratch_bytes(int64_t n, int32_t m, int64_t WB, const abj_opts& o, const MfmaPlan& plan);
// Query-side join against reference statistics B: query statistics, pair loop
// of the selected tier, row epilogue.  All scratch comes from `ar`; the 16-bit
// tiers take the dictionary side from `dop` (if NULL, `ar` must also hold
// mfma_dict_bytes(plan) for it).
int join_query(const double* query, int64_t n, int32_t m, const SeriesDev& B, const abj_opts& o,
               const MfmaPlan& plan, float* P, int64_t* I, Arena& ar, hipStream_t stream,
               size_t part_bytes = 0, const MfmaDictOp* dop = nullptr);

// Benchmark timing hooks (no-ops unless abj_profile_enable(1) was called):
// prof_begin records a start event on the stream, prof_end the stop event and
// the number of valid pairs the launch covers.
struct ProfMark {
    hipEvent_t start = nullptr;
};
int prof_begin(ProfMark* mark, hipStream_t stream);
int prof_end(ProfMark* mark, hipStream_t stream, int64_t pairs);

}  // namespace abj
