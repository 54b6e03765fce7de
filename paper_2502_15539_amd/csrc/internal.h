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

// One batch of a multi-MPHF launch (48 bytes).
struct MultiBatch {
    const void *keys;         // u64 keys, or the packed bytes of byte keys
    const uint64_t *offsets;  // byte keys: nq + 1 offsets into keys
    void *out;
    uint64_t nq;
    uint64_t end_limit;       // byte keys: largest string end offset that can be read safely
    uint32_t mphf;            // index into the table's MPHF array
    uint32_t flags;           // kBatchBytes | kBatchOut64
};
enum : uint32_t { kBatchBytes = 1, kBatchOut64 = 2 };

// Compute dies (XCDs) of the device, each with its own L2; the dispatcher
// hands consecutive workgroups to them in turn (workgroup i to die i mod 8).
constexpr uint32_t kDies = 8;

// The batches of one multi-MPHF launch, laid out back to back after this
// header: tile_begin[count] (first global tile of each batch, ascending),
// batch[count], then mphf[mphfs] (each distinct MPHF once). The kernel's
// binary search touches only the compact tile_begin array, and a table of
// many batches over few MPHFs stays small to upload. Batches are grouped by
// MPHF (in the order the MPHFs first appear), so that a contiguous range of
// tiles touches few MPHFs. die_first splits the tiles into one contiguous
// range per die, of about equal estimated work (multi_batch_cost).
struct MultiTable {
    uint32_t count;  // batches
    uint32_t tile;   // keys per tile the table was numbered with
    uint64_t tiles;  // total tiles
    uint32_t mphfs;  // distinct MPHFs
    uint32_t pad_;
    uint64_t die_first[kDies + 1];  // die x takes tiles [die_first[x], die_first[x + 1])
};
static_assert(sizeof(MultiTable) == 96 && sizeof(MultiBatch) == 48, "multi table layout");

__host__ __device__ inline uint64_t *multi_tile_begin(MultiTable *t) { return reinterpret_cast<uint64_t *>(t + 1); }
__host__ __device__ inline const uint64_t *multi_tile_begin(const MultiTable *t) {
    return reinterpret_cast<const uint64_t *>(t + 1);
}
__host__ __device__ inline MultiBatch *multi_batches(MultiTable *t) {
    return reinterpret_cast<MultiBatch *>(multi_tile_begin(t) + t->count);
}
__host__ __device__ inline const MultiBatch *multi_batches(const MultiTable *t) {
    return reinterpret_cast<const MultiBatch *>(multi_tile_begin(t) + t->count);
}
__host__ __device__ inline DevMphf *multi_mphfs(MultiTable *t) {
    return reinterpret_cast<DevMphf *>(multi_batches(t) + t->count);
}
__host__ __device__ inline const DevMphf *multi_mphfs(const MultiTable *t) {
    return reinterpret_cast<const DevMphf *>(multi_batches(t) + t->count);
}

// Bytes of a table of `count` batches over `mphfs` distinct MPHFs, and the
// most a table of up to max_batches batches can take.
constexpr size_t multi_table_bytes(uint32_t count, uint32_t mphfs) {
    return sizeof(MultiTable) + (size_t)count * (sizeof(uint64_t) + sizeof(MultiBatch)) + (size_t)mphfs * sizeof(DevMphf);
}
constexpr size_t multi_table_capacity(int max_batches) {
    const uint32_t m = max_batches > 0 ? (uint32_t)max_batches : 0;
    return multi_table_bytes(m, m);
}

// LDS of the packed remap decode: 64 u64 per wavefront of a workgroup of
// `block` threads. The single-MPHF kernels pack from kPackMinKeys keys per
// lane on (with fewer, a wavefront has at most one or two decode passes to
// merge), the multi-MPHF kernel always.
constexpr int kPackMinKeys = 4;
inline uint32_t pack_lds_bytes(uint32_t block) { return block / 64u * 64u * 8u; }
inline uint32_t multi_lds_bytes(const MultiTuning &t) { return pack_lds_bytes((uint32_t)t.block); }
// The table must have been filled with multi_tile(t); grid from multi_grid(t).
hipError_t launch_query_multi(const MultiTable *table, const MultiTuning &t, uint32_t grid, hipStream_t s);
// Copy bytes (rounded up to a multiple of 16, which both buffers must hold)
// from mapped host memory src to device memory dst with a kernel on s.
hipError_t launch_stage_in(const void *src, void *dst, size_t bytes, hipStream_t s);
int multi_blocks_per_cu(const MultiTuning &t);  // most resident workgroups of the kernel per compute unit
uint32_t multi_grid(const MultiTuning &t);      // persistent grid size on the current device
// Validate k batches and write them (and the tile prefix sums for tiles of
// `tile` keys) into t.
int fill_multi_table(MultiTable *t, const ptrhash_query_desc *descs, int k, uint32_t tile);

// The same with a caller-provided host workspace, so that the fill itself
// allocates nothing: room for k output spans, and an open-addressing table
// of hcap handle slots (hcap a power of two, at least 2k).
struct MultiSpan {
    uintptr_t lo, hi;  // [lo, hi)
    int batch;
};
struct MultiWork {
    MultiSpan *outs;                 // k
    const ptrhash_handle **handles;  // hcap
    uint32_t *index;                 // hcap
    uint32_t hcap;
    uint32_t *batch_mphf;            // k: MPHF of each non-empty batch
    uint32_t *mphf_start;            // k + 1: first slot of each MPHF's batches in the table
};
int fill_multi_table_ws(MultiTable *t, const ptrhash_query_desc *descs, int k, uint32_t tile, MultiWork &w);

hipError_t launch_query_u64(const DevMphf &m, const uint64_t *keys, uint64_t nq, void *out, bool out64,
                            const Tuning &t, hipStream_t s);
// Byte keys: a string may end at most at end_limit (see bytes_end_limit);
// a key whose offsets decrease or pass it is not read and gets an index of
// all ones.
hipError_t launch_query_bytes(const DevMphf &m, const uint8_t *data, uint64_t end_limit, const uint64_t *offsets,
                              uint64_t nq, void *out, bool out64, const Tuning &t, hipStream_t s);

// The string hash reads aligned 8-byte words up to 15 bytes past a string's
// end, so a string in a buffer of data_len bytes may end at data_len - 16.
constexpr uint64_t kBytesReadSlack = 16;
constexpr uint64_t kBytesPadding = 64;  // readable bytes the ABI asks for after the last string
inline uint64_t bytes_end_limit(uint64_t data_len) { return data_len - kBytesReadSlack; }

// [a, a + na) and [b, b + nb) share a byte.
inline bool ranges_overlap(const void *a, uint64_t na, const void *b, uint64_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na && nb && x < y + nb && y < x + na;
}

hipError_t launch_bench_gather(const uint64_t *keys, uint64_t nq, const uint8_t *table, uint64_t table_len,
                               uint64_t *out, int keys_per_lane, int block, uint32_t lds_bytes, hipStream_t s);
hipError_t launch_bench_gather_pure(uint64_t n, const uint8_t *table, uint64_t T, uint32_t *sink, uint32_t grid,
                                    hipStream_t s);
hipError_t launch_bench_gather_pair(uint64_t n, const uint8_t *table, uint64_t T, uint32_t D, uint32_t *sink,
                                    uint32_t grid, hipStream_t s);
hipError_t launch_bench_copy(const uint64_t *keys, uint64_t nq, uint64_t *out, int keys_per_lane, int block,
                             hipStream_t s);
hipError_t launch_bench_gather_bucket(const uint64_t *keys, uint64_t nq, const DevMphf &m, uint64_t *out,
                                      int keys_per_lane, int block, uint32_t lds_bytes, hipStream_t s);
hipError_t launch_bench_gather_bytes(const uint8_t *data, uint64_t end_limit, const uint64_t *offsets, uint64_t nq,
                                     const DevMphf &m, uint32_t *out, int keys_per_lane, int block,
                                     uint32_t lds_bytes, hipStream_t s);
hipError_t launch_bench_scatter(const uint64_t *in, uint32_t log2_n, uint64_t *out, hipStream_t s);

}  // namespace ptrhash
