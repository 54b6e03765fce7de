// Construction front half on the device (Section 3.1 "Construction": hash,
// sort, partition): hash every key, radix-sort the hashes, copy them to the
// host. Sorted hashes are grouped by part and by bucket, because the part
// hi(P*h) and the bucket within it are non-decreasing in h; the host pilot
// search then takes each part's hashes as they are.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "builder.h"
#include "errors.h"
#include "internal.h"

namespace {

__global__ void hash_keys_k(const uint64_t *__restrict__ keys, uint64_t n, uint64_t *__restrict__ out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = ptrhash::hash_u64(keys[i]);
}

struct DeviceBuffers {
    void *p[3] = {nullptr, nullptr, nullptr};
    ~DeviceBuffers() {
        for (void *x : p)
            if (x) (void)hipFree(x);
    }
};

}  // namespace

extern "C" {

PTRHASH_API int ptrhash_build_u64_device(const uint64_t *keys, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                                         void *remap, int threads, ptrhash_build_info *info, hipStream_t stream) {
    using ptrhash::set_error;
    if (!keys || !params || !pilots) return set_error(PTRHASH_E_INVAL, "NULL argument");
    if (n == 0 || params->n != n) return set_error(PTRHASH_E_INVAL, "params->n must equal n > 0");
    if (params->key_kind != PTRHASH_KEY_U64) return set_error(PTRHASH_E_INVAL, "device front half takes u64 keys");
    const bool timing = std::getenv("PTRHASH_BUILD_TIMING") != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    DeviceBuffers buf;
    uint64_t *a = nullptr, *b = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&buf.p[0], n * sizeof(uint64_t))) != hipSuccess ||
        (e = hipMalloc(&buf.p[1], n * sizeof(uint64_t))) != hipSuccess)
        return set_error(PTRHASH_E_NOMEM, "device buffers for the sort: %s", hipGetErrorString(e));
    a = static_cast<uint64_t *>(buf.p[0]);
    b = static_cast<uint64_t *>(buf.p[1]);
    hipLaunchKernelGGL(hash_keys_k, dim3(8192), dim3(256), 0, stream, keys, n, a);
    if ((e = hipGetLastError()) != hipSuccess) return set_error(PTRHASH_E_HIP, "hash launch: %s", hipGetErrorString(e));
    hipcub::DoubleBuffer<uint64_t> db(a, b);
    size_t temp = 0;
    if ((e = hipcub::DeviceRadixSort::SortKeys(nullptr, temp, db, (size_t)n, 0, 64, stream)) != hipSuccess)
        return set_error(PTRHASH_E_HIP, "sort sizing: %s", hipGetErrorString(e));
    if ((e = hipMalloc(&buf.p[2], temp)) != hipSuccess)
        return set_error(PTRHASH_E_NOMEM, "sort scratch: %s", hipGetErrorString(e));
    if ((e = hipcub::DeviceRadixSort::SortKeys(buf.p[2], temp, db, (size_t)n, 0, 64, stream)) != hipSuccess)
        return set_error(PTRHASH_E_HIP, "sort: %s", hipGetErrorString(e));
    std::vector<uint64_t> sorted;
    try {
        sorted.resize(n);
    } catch (const std::bad_alloc &) {
        return set_error(PTRHASH_E_NOMEM, "host buffer for the sorted hashes");
    }
    if ((e = hipMemcpyAsync(sorted.data(), db.Current(), n * sizeof(uint64_t), hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return set_error(PTRHASH_E_HIP, "sorted hashes to host: %s", hipGetErrorString(e));
    if (timing)
        std::fprintf(stderr, "[build] device    %8.3f s (hash, sort, copy out)\n",
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    for (void *&x : buf.p) {
        if (x) (void)hipFree(x);
        x = nullptr;
    }
    return ptrhash::build_from_sorted(std::move(sorted), n, params, pilots, remap, threads, info);
}

}  // extern "C"
