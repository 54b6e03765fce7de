// Internal interfaces between the C ABI layer, the kernels and the builder.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mphf_device.h"
#include "ptrhash.h"

namespace ptrhash {

enum : int { kKernelPlain = 0, kKernelPipelined = 1 };

struct Tuning {
    int kernel = kKernelPipelined;
    int keys_per_lane = 4;
    int block = 256;
    uint32_t lds_bytes = 0;  // dynamic LDS reserved per workgroup: caps resident workgroups per CU
};

bool valid_tuning(int kernel, int keys_per_lane, int block);

// Persistent multi-batch launch. A tile is keys_per_lane * block keys of one
// batch; the grid is CUs x resident workgroups per CU (blocks_per_cu, or the
// most the kernel allows when 0).
struct MultiTuning {
    int keys_per_lane = 4;
    int block = 256;
    int blocks_per_cu = 0;
};
bool valid_multi_tuning(int keys_per_lane, int block, int blocks_per_cu);
inline uint32_t multi_tile(const MultiTuning &t) { return (uint32_t)t.keys_per_lane * (uint32_t)t.block; }
MultiTuning multi_default_tuning();  // the process-wide default (ptrhash_set_multi_kernel)

struct MultiDesc {
    DevMphf m;
    const uint64_t *keys;     // u64 keys (bytes == 0)
    const uint8_t *data;      // byte keys (bytes == 1)
    const uint64_t *offsets;
    void *out;
    uint64_t nq;
    uint64_t tile_begin;      // first global tile of this batch
    uint32_t bytes, out64;
};

struct MultiTable {
    uint32_t count;           // batches (>= 1)
    uint32_t tile;            // keys per tile the table was numbered with
    uint64_t tiles;           // total tiles
    MultiDesc descs[1];       // count entries follow
};

inline size_t multi_table_bytes(int max_descs) {
    return sizeof(MultiTable) + sizeof(MultiDesc) * (size_t)(max_descs > 1 ? max_descs - 1 : 0);
}

// The table must have been filled with multi_tile(t); grid from multi_grid(t).
hipError_t launch_query_multi(const MultiTable *table, const MultiTuning &t, uint32_t grid, hipStream_t s);
int multi_blocks_per_cu(const MultiTuning &t);  // most resident workgroups of the kernel per compute unit
uint32_t multi_grid(const MultiTuning &t);      // persistent grid size on the current device
// Validate k batches and write them (and the tile prefix sums for tiles of
// `tile` keys) into t.
int fill_multi_table(MultiTable *t, const ptrhash_query_desc *descs, int k, uint32_t tile);

hipError_t launch_query_u64(const DevMphf &m, const uint64_t *keys, uint64_t nq, void *out, bool out64,
                            const Tuning &t, hipStream_t s);
hipError_t launch_query_bytes(const DevMphf &m, const uint8_t *data, const uint64_t *offsets, uint64_t nq,
                              void *out, bool out64, const Tuning &t, hipStream_t s);

hipError_t launch_bench_gather(const uint64_t *keys, uint64_t nq, const uint8_t *table, uint64_t table_len,
                               uint64_t *out, int keys_per_lane, int block, uint32_t lds_bytes, hipStream_t s);
hipError_t launch_bench_gather_pure(uint64_t n, const uint8_t *table, uint64_t T, uint32_t *sink, uint32_t grid,
                                    hipStream_t s);
hipError_t launch_bench_gather_pair(uint64_t n, const uint8_t *table, uint64_t T, uint32_t D, uint32_t *sink,
                                    uint32_t grid, hipStream_t s);
hipError_t launch_bench_copy(const uint64_t *keys, uint64_t nq, uint64_t *out, int keys_per_lane, int block,
                             hipStream_t s);

}  // namespace ptrhash
