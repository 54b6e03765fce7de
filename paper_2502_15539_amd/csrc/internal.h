// Internal interfaces between the C ABI layer, the kernels and the builder.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mphf_device.h"

namespace ptrhash {

enum : int { kKernelPlain = 0, kKernelPipelined = 1 };

struct Tuning {
    int kernel = kKernelPipelined;
    int keys_per_lane = 4;
    int block = 256;
};

bool valid_tuning(int kernel, int keys_per_lane, int block);

hipError_t launch_query_u64(const DevMphf &m, const uint64_t *keys, uint64_t nq, void *out, bool out64,
                            const Tuning &t, hipStream_t s);
hipError_t launch_query_bytes(const DevMphf &m, const uint8_t *data, const uint64_t *offsets, uint64_t nq,
                              void *out, bool out64, const Tuning &t, hipStream_t s);

hipError_t launch_bench_gather(const uint64_t *keys, uint64_t nq, const uint8_t *table, uint64_t table_len,
                               uint64_t *out, int keys_per_lane, int block, hipStream_t s);
hipError_t launch_bench_copy(const uint64_t *keys, uint64_t nq, uint64_t *out, int keys_per_lane, int block,
                             hipStream_t s);

}  // namespace ptrhash
