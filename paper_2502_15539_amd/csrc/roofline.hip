// Roofline microbenchmarks: the memory pattern of a query with none of its
// arithmetic. gather: stream a u64 key in, read one byte at a random index
// hi(key * T) of a T-byte table, stream a u64 out. gather_bucket: the same
// with the query's own part/bucket index into a loaded MPHF's pilots.
// gather_bytes: the string workload's streams plus that gather. copy: stream
// in, stream out. Same tiling, non-temporal streams and keys-per-lane knob as
// the pipelined query kernel, so a query's time can be compared with these.
#include "internal.h"

namespace ptrhash {

template <int K>
__global__ void __launch_bounds__(1024) bench_gather_k(const uint64_t *__restrict__ keys, uint64_t nq,
                                                       const uint8_t *__restrict__ table, uint64_t T,
                                                       uint64_t *__restrict__ out) {
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * K + threadIdx.x;
    uint64_t k[K];
    bool ok[K];
    // unconditional loads, as in the query kernel: a lane past the end reads
    // key 0 (nq >= 1), and hi(k * T) < T for every k
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        ok[j] = i < nq;
        k[j] = __builtin_nontemporal_load(keys + (ok[j] ? i : 0));
    }
    uint32_t b[K];
#pragma unroll
    for (int j = 0; j < K; ++j) b[j] = table[__umul64hi(k[j], T)];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        if (ok[j]) __builtin_nontemporal_store(k[j] ^ b[j], out + i);
    }
}

template <int K>
__global__ void __launch_bounds__(1024) bench_copy_k(const uint64_t *__restrict__ keys, uint64_t nq,
                                                     uint64_t *__restrict__ out) {
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * K + threadIdx.x;
    uint64_t k[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        k[j] = __builtin_nontemporal_load(keys + (i < nq ? i : 0));
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        if (i < nq) __builtin_nontemporal_store(k[j], out + i);
    }
}

// Random byte gathers with no streams: index i is hi(mix(i) * T) (SplitMix64
// output mixer), four gathers in flight per lane per step, one u32 sum per
// lane written at the end so the loads stay live. hi(x * T) < T for every x,
// so the loads past the end are in bounds and only their values are dropped.
__device__ inline uint64_t sm_mix(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    z ^= z >> 31;
    return z;
}

__global__ void __launch_bounds__(256) bench_gather_pure_k(uint64_t n, const uint8_t *__restrict__ table, uint64_t T,
                                                           uint32_t *__restrict__ sink) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (uint64_t i = t; i < n; i += 4 * stride) {
        uint32_t b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t k = i + j * stride;
            b[j] = table[__umul64hi(sm_mix(k), T)];
            b[j] = k < n ? b[j] : 0;
        }
        acc += b[0] + b[1] + b[2] + b[3];
    }
    sink[t] = acc;
}

// Line-size probe: as the pure gather, plus a second byte at o xor D for
// each random offset o (D = 32: same 64-byte half, 64: other half of the
// same 128-byte line, 128: the neighbouring line). T is a multiple of 256,
// so o xor D < T.
__global__ void __launch_bounds__(256) bench_gather_pair_k(uint64_t n, const uint8_t *__restrict__ table,
                                                           uint64_t T, uint32_t D, uint32_t *__restrict__ sink) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (uint64_t i = t; i < n; i += 4 * stride) {
        uint32_t b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t k = i + j * stride;
            const uint64_t o = __umul64hi(sm_mix(k), T);
            b[j] = table[o] + table[o ^ D];
            b[j] = k < n ? b[j] : 0;
        }
        acc += b[0] + b[1] + b[2] + b[3];
    }
    sink[t] = acc;
}

// Like-for-like gather: the query's own pilot index. Each key is hashed and
// sent to its part and global bucket exactly as a query does (so the gathers
// have the cubic bucket function's skew and hit the caches as often as the
// query's do), the bucket's pilot byte is read and the key xor that byte is
// streamed out; the slot hash and the remap are left out.
template <int K>
__global__ void __launch_bounds__(1024) bench_gather_bucket_k(const uint64_t *__restrict__ keys, uint64_t nq,
                                                              DevMphf m, uint64_t *__restrict__ out) {
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * K + threadIdx.x;
    uint64_t k[K];
    bool ok[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        ok[j] = i < nq;
        k[j] = __builtin_nontemporal_load(keys + (ok[j] ? i : 0));
    }
    uint32_t b[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        uint32_t part;
        b[j] = m.pilots[bucket_of(m, hash_u64(k[j]), part)];
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        if (ok[j]) __builtin_nontemporal_store(k[j] ^ b[j], out + i);
    }
}

// String-stream gather: the memory pattern of a byte-key query. Each key's
// two offsets and its aligned 8-byte words are read (the words the string
// hash reads), the words are folded by xor and mixed once, the result goes
// through the MPHF's part/bucket map, the pilot byte is read, and a u32 is
// streamed out. A key whose offsets decrease or pass end_limit is skipped.
template <int K>
__global__ void __launch_bounds__(1024) bench_gather_bytes_k(const uint8_t *__restrict__ data, uint64_t end_limit,
                                                             const uint64_t *__restrict__ offsets, uint64_t nq,
                                                             DevMphf m, uint32_t *__restrict__ out) {
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * K + threadIdx.x;
    uint64_t x[K];
    bool ok[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        ok[j] = i < nq;
        x[j] = 0;
        if (ok[j]) {
            const uint64_t o0 = offsets[i], o1 = offsets[i + 1];
            if (o1 >= o0 && o1 <= end_limit) {
                const uint64_t *W = reinterpret_cast<const uint64_t *>(data + (o0 & ~7ull));
                const uint64_t nw = ((o1 - o0) + 7) >> 3;
                uint64_t f = o1 - o0;
                for (uint64_t w = 0; w <= nw; ++w) f ^= W[w];
                x[j] = fmix64(f);
            }
        }
    }
    uint32_t b[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        uint32_t part;
        b[j] = m.pilots[bucket_of(m, x[j], part)];
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * blockDim.x;
        if (ok[j]) __builtin_nontemporal_store((uint32_t)x[j] ^ b[j], out + i);
    }
}

// Un-permute probe: out[(i * A) mod 2^L] = in[i] for i < 2^L, A odd (a
// bijection of [0, 2^L)): a streamed 8-byte read and a random 8-byte write
// per element, the cost of putting indices computed in some other order
// back into query order.
__global__ void __launch_bounds__(256) bench_scatter_k(const uint64_t *__restrict__ in, uint32_t log2_n,
                                                       uint64_t *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t mask = (1ull << log2_n) - 1;
    if (i > mask) return;
    const uint64_t v = __builtin_nontemporal_load(in + i);
    out[(i * 0x9E3779B97F4A7C15ull) & mask] = v;
}

static inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

hipError_t launch_bench_gather_bucket(const uint64_t *keys, uint64_t nq, const DevMphf &m, uint64_t *out, int K,
                                      int block, uint32_t lds, hipStream_t s) {
    const dim3 grid((uint32_t)ceil_div(nq, (uint64_t)block * K)), blk((uint32_t)block);
    switch (K) {
    case 1: hipLaunchKernelGGL(bench_gather_bucket_k<1>, grid, blk, lds, s, keys, nq, m, out); break;
    case 2: hipLaunchKernelGGL(bench_gather_bucket_k<2>, grid, blk, lds, s, keys, nq, m, out); break;
    case 4: hipLaunchKernelGGL(bench_gather_bucket_k<4>, grid, blk, lds, s, keys, nq, m, out); break;
    case 8: hipLaunchKernelGGL(bench_gather_bucket_k<8>, grid, blk, lds, s, keys, nq, m, out); break;
    case 16: hipLaunchKernelGGL(bench_gather_bucket_k<16>, grid, blk, lds, s, keys, nq, m, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bench_gather_bytes(const uint8_t *data, uint64_t end_limit, const uint64_t *offsets, uint64_t nq,
                                     const DevMphf &m, uint32_t *out, int K, int block, uint32_t lds, hipStream_t s) {
    const dim3 grid((uint32_t)ceil_div(nq, (uint64_t)block * K)), blk((uint32_t)block);
    switch (K) {
    case 1: hipLaunchKernelGGL(bench_gather_bytes_k<1>, grid, blk, lds, s, data, end_limit, offsets, nq, m, out); break;
    case 2: hipLaunchKernelGGL(bench_gather_bytes_k<2>, grid, blk, lds, s, data, end_limit, offsets, nq, m, out); break;
    case 4: hipLaunchKernelGGL(bench_gather_bytes_k<4>, grid, blk, lds, s, data, end_limit, offsets, nq, m, out); break;
    case 8: hipLaunchKernelGGL(bench_gather_bytes_k<8>, grid, blk, lds, s, data, end_limit, offsets, nq, m, out); break;
    case 16: hipLaunchKernelGGL(bench_gather_bytes_k<16>, grid, blk, lds, s, data, end_limit, offsets, nq, m, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bench_scatter(const uint64_t *in, uint32_t log2_n, uint64_t *out, hipStream_t s) {
    const uint64_t n = 1ull << log2_n;
    hipLaunchKernelGGL(bench_scatter_k, dim3((uint32_t)ceil_div(n, 256)), dim3(256), 0, s, in, log2_n, out);
    return hipGetLastError();
}

hipError_t launch_bench_gather_pair(uint64_t n, const uint8_t *table, uint64_t T, uint32_t D, uint32_t *sink,
                                    uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(bench_gather_pair_k, dim3(grid), dim3(256), 0, s, n, table, T, D, sink);
    return hipGetLastError();
}

hipError_t launch_bench_gather_pure(uint64_t n, const uint8_t *table, uint64_t T, uint32_t *sink, uint32_t grid,
                                    hipStream_t s) {
    hipLaunchKernelGGL(bench_gather_pure_k, dim3(grid), dim3(256), 0, s, n, table, T, sink);
    return hipGetLastError();
}

hipError_t launch_bench_gather(const uint64_t *keys, uint64_t nq, const uint8_t *table, uint64_t T, uint64_t *out,
                               int K, int block, uint32_t lds, hipStream_t s) {
    const dim3 grid((uint32_t)ceil_div(nq, (uint64_t)block * K)), blk((uint32_t)block);
    switch (K) {
    case 1: hipLaunchKernelGGL(bench_gather_k<1>, grid, blk, lds, s, keys, nq, table, T, out); break;
    case 2: hipLaunchKernelGGL(bench_gather_k<2>, grid, blk, lds, s, keys, nq, table, T, out); break;
    case 4: hipLaunchKernelGGL(bench_gather_k<4>, grid, blk, lds, s, keys, nq, table, T, out); break;
    case 8: hipLaunchKernelGGL(bench_gather_k<8>, grid, blk, lds, s, keys, nq, table, T, out); break;
    case 16: hipLaunchKernelGGL(bench_gather_k<16>, grid, blk, lds, s, keys, nq, table, T, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bench_copy(const uint64_t *keys, uint64_t nq, uint64_t *out, int K, int block, hipStream_t s) {
    const dim3 grid((uint32_t)ceil_div(nq, (uint64_t)block * K)), blk((uint32_t)block);
    switch (K) {
    case 1: hipLaunchKernelGGL(bench_copy_k<1>, grid, blk, 0, s, keys, nq, out); break;
    case 2: hipLaunchKernelGGL(bench_copy_k<2>, grid, blk, 0, s, keys, nq, out); break;
    case 4: hipLaunchKernelGGL(bench_copy_k<4>, grid, blk, 0, s, keys, nq, out); break;
    case 8: hipLaunchKernelGGL(bench_copy_k<8>, grid, blk, 0, s, keys, nq, out); break;
    case 16: hipLaunchKernelGGL(bench_copy_k<16>, grid, blk, 0, s, keys, nq, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ptrhash
