// Many MPHFs in one launch without any allocation: the batch table of
// ptrhash_query_multi lives in a fixed device array of this library instead
// of a plan allocated on first use, for callers that cannot allocate (HIP
// graph capture aside, tight serving loops, harnesses that forbid hipMalloc).
//
// The array is one file-scope __device__ symbol, so each GPU the library
// runs on holds its own copy for the life of the process. Host code never
// passes the symbol itself to a kernel or a copy: on the first call on a
// device, hipGetSymbolAddress gives that device's address, which is kept per
// device and used from then on. The host side builds the table in a fixed
// host array (so the host side does not allocate either) and copies it to
// the device array on the caller's stream, ahead of the launch.
//
// Every call on one GPU shares that GPU's array, and each call overwrites
// it: calls that overlap on one GPU (on different streams, or from
// different host threads before the earlier launch has read its table) race.
#include <mutex>

#include "errors.h"
#include "internal.h"
#include "ptrhash.h"

namespace ptrhash {
namespace {

constexpr int kNoAllocBatches = 256;
constexpr size_t kNoAllocBytes = (multi_table_capacity(kNoAllocBatches) + 255) / 256 * 256;
constexpr int kMaxDevices = 64;
constexpr uint32_t kHandleSlots = 2 * kNoAllocBatches;

__device__ __align__(256) uint8_t scratch[kNoAllocBytes];

std::mutex g_mu;                 // guards everything below
void *g_scratch[kMaxDevices];    // scratch's address on each device (null until the first call there)
alignas(256) uint8_t g_stage[kNoAllocBytes];  // the table as the host builds it
MultiSpan g_outs[kNoAllocBatches];
const ptrhash_handle *g_handles[kHandleSlots];
uint32_t g_index[kHandleSlots];
uint32_t g_batch_mphf[kNoAllocBatches];
uint32_t g_mphf_start[kNoAllocBatches + 1];

}  // namespace
}  // namespace ptrhash

extern "C" {

PTRHASH_API int ptrhash_query_multi_noalloc(const ptrhash_query_desc *descs, int k, hipStream_t stream) {
    using namespace ptrhash;
    if (k < 0 || (k > 0 && !descs)) return set_error(PTRHASH_E_INVAL, "bad descriptor array");
    if (k > kNoAllocBatches)
        return set_error(PTRHASH_E_RANGE, "%d batches exceed the %d of the fixed table", k, kNoAllocBatches);
    if (k == 0) return PTRHASH_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return set_error(PTRHASH_E_HIP, "hipStreamIsCapturing: %s", hipGetErrorString(e));
    if (cs != hipStreamCaptureStatusNone)
        return set_error(PTRHASH_E_STATE, "stream is capturing: capture a multi plan instead");
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess)
        return set_error(PTRHASH_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(PTRHASH_E_RANGE, "device %d out of range", dev);

    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess || !ptr)
            return set_error(PTRHASH_E_HIP, "hipGetSymbolAddress of the batch table: %s", hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    const MultiTuning t = multi_default_tuning();
    MultiTable *stage = reinterpret_cast<MultiTable *>(g_stage);
    MultiWork w{g_outs, g_handles, g_index, kHandleSlots, g_batch_mphf, g_mphf_start};
    const int rc = fill_multi_table_ws(stage, descs, k, multi_tile(t), w);
    if (rc) return rc;
    if (stage->tiles == 0) return PTRHASH_OK;
    const size_t bytes = multi_table_bytes(stage->count, stage->mphfs);
    // g_stage is pageable host memory, which HIP copies synchronously: the
    // table has left it when the call returns, so the next call may reuse it
    if ((e = hipMemcpyAsync(g_scratch[dev], g_stage, bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
        return set_error(PTRHASH_E_HIP, "batch table copy: %s", hipGetErrorString(e));
    e = launch_query_multi(static_cast<const MultiTable *>(g_scratch[dev]), t, multi_grid(t), stream);
    return e == hipSuccess ? PTRHASH_OK : set_error(PTRHASH_E_HIP, "query_multi launch: %s", hipGetErrorString(e));
}

}  // extern "C"
