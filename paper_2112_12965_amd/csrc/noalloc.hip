// ab_join_noalloc: the AB-join with its workspace in a fixed device array of
// the library instead of the stream-ordered allocator, for callers that cannot
// allocate device memory during the call.
//
// The array is a file-scope __device__ variable, so every GPU the library runs
// on holds its own copy, at its own device address, until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// the name is a stand-in, not a device address): set-up looks the address up
// with hipGetSymbolAddress, once per device with that device current, and the
// join carves its workspace from that address.
#include <mutex>

#include "abj_internal.hpp"

namespace abj {

namespace {

// Workspace limit of one call (the value ab_join_noalloc's declaration states).
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static_assert(kNoAllocBytes == (size_t)ABJ_NOALLOC_SCRATCH_BYTES, "workspace limit differs from the header");

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_scratch_dev[64] = {};

}  // namespace

int noalloc_setup(void** out)
{
    int dev = 0;
    ABJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(ABJ_EHIP, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(ABJ_EHIP, "device address of the fixed workspace on device %d: %s", dev,
                             hipGetErrorString(e));
        }
        g_scratch_dev[dev] = p;
    }
    if (out) *out = g_scratch_dev[dev];
    return ABJ_OK;
}

}  // namespace abj

using namespace abj;

extern "C" int ab_join_noalloc(const double* query, int64_t n_query, const double* dict, int64_t n_dict,
                               const int64_t* seg_bounds, int32_t n_seg, int32_t m, float* P_AB, int64_t* I_AB,
                               const abj_opts* opts, void* hip_stream)
{
    // ---- validation: nothing is enqueued or written before this passes ----
    JoinPrep jp;
    ABJ_TRY(ab_join_validate(query, n_query, dict, n_dict, seg_bounds, n_seg, m, P_AB, I_AB, opts, &jp));
    // the FP32 tiles store per-chunk keys when they fit, else merge by atomics
    // (the same row keys either way, so the results equal ab_join's)
    size_t part_bytes = jp.part_bytes;
    if (jp.scratch > kNoAllocBytes) part_bytes = 0;
    const size_t need = part_bytes ? jp.scratch : jp.scratch_atomic;
    if (need > kNoAllocBytes)
        return set_error(ABJ_EINVAL,
                         "ab_join_noalloc: this join needs %zu bytes of workspace, more than the fixed %zu bytes "
                         "(use ab_join)",
                         need, kNoAllocBytes);
    ABJ_TRY(ensure_device());
    void* base = nullptr;
    ABJ_TRY(noalloc_setup(&base));
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    Arena ar(base, kNoAllocBytes);
    return join_run(query, n_query, m, dict, n_dict, seg_bounds, n_seg, nullptr, jp.o, jp.plan, P_AB, I_AB, ar,
                    stream, part_bytes);
}
