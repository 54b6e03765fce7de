// Seeded synthetic inputs on the device: the same counter-based generators
// as the host-side generator module (SplitMix64 of Steele, Lea and Flood,
// OOPSLA 2014, and a 4-round Feistel permutation with cycle walking), so a
// benchmark can create 10^9 keys or a shuffled member stream in place.
// Holds no hash-function arithmetic of the MPHF itself.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "errors.h"
#include "ptrhash.h"

namespace {

constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ull;

__host__ __device__ inline uint64_t sm_mix(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    z ^= z >> 31;
    return z;
}

__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t idx) {
    return sm_mix(seed + (idx + 1) * kGolden);
}

struct Feistel {
    uint64_t n, mask, keys[4];
    uint32_t half, pad_;
};

__device__ inline uint64_t feistel_round(const Feistel &f, uint64_t x) {
    uint64_t left = x >> f.half, right = x & f.mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t g = sm_mix(right ^ f.keys[r]) & f.mask;
        const uint64_t t = left ^ g;
        left = right;
        right = t;
    }
    return (left << f.half) | right;
}

// Cycle walking ends: i < n lies on its own cycle of the bijection.
__device__ inline uint64_t permute(const Feistel &f, uint64_t i) {
    uint64_t x = feistel_round(f, i);
    while (x >= f.n) x = feistel_round(f, x);
    return x;
}

__global__ void gen_keys_k(uint64_t seed, uint64_t start, uint64_t count, uint64_t *out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = splitmix64(seed, start + i);
}

__global__ void gen_query_k(uint64_t key_seed, Feistel f, uint64_t start, uint64_t count, uint64_t *out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = splitmix64(key_seed, permute(f, start + i));
}

// String i of a set: length 10 + (r mod 41), byte j = 0x20 + ((r_j & 0xff) mod 95)
// with r = SplitMix64(seed, i) and r_j = SplitMix64(seed ^ kByteSalt, 64 i + j).
constexpr uint64_t kByteSalt = 0x2545F4914F6CDD1Dull;

__device__ inline uint64_t string_of(bool shuffled, const Feistel &f, uint64_t i) {
    return shuffled ? permute(f, i) : i;
}

__global__ void gen_str_len_k(uint64_t seed, Feistel f, int shuffled, uint64_t start, uint64_t count,
                              uint64_t *lengths) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = string_of(shuffled, f, start + i);
        lengths[i] = 10 + splitmix64(seed, s) % 41;
    }
}

__global__ void gen_str_bytes_k(uint64_t seed, Feistel f, int shuffled, uint64_t start, uint64_t count,
                                const uint64_t *offsets, uint8_t *data) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = string_of(shuffled, f, start + i);
        const uint64_t len = offsets[i + 1] - offsets[i];
        uint8_t *dst = data + offsets[i];
        for (uint64_t j = 0; j < len; ++j)
            dst[j] = (uint8_t)(0x20 + (splitmix64(seed ^ kByteSalt, s * 64 + j) & 0xff) % 95);
    }
}

Feistel make_feistel(uint64_t n, uint64_t order_seed) {
    Feistel f{};
    uint32_t bits = 2;
    while (bits < 64 && ((n - 1) >> bits)) ++bits;
    bits += bits & 1u;
    f.n = n;
    f.half = bits / 2;
    f.mask = (1ull << f.half) - 1;
    for (int r = 0; r < 4; ++r) f.keys[r] = splitmix64(order_seed, (uint64_t)r);
    return f;
}

int launch_err(hipError_t e, const char *what) {
    return e == hipSuccess ? PTRHASH_OK : ptrhash::set_error(PTRHASH_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" {

PTRHASH_API int ptrhash_gen_u64_keys(uint64_t seed, uint64_t start, uint64_t count, uint64_t *out,
                                     hipStream_t stream) {
    if (count == 0) return PTRHASH_OK;
    if (!out) return ptrhash::set_error(PTRHASH_E_INVAL, "out is NULL");
    hipLaunchKernelGGL(gen_keys_k, dim3(8192), dim3(256), 0, stream, seed, start, count, out);
    return launch_err(hipGetLastError(), "gen_keys launch");
}

PTRHASH_API int ptrhash_gen_query_stream(uint64_t n, uint64_t key_seed, uint64_t order_seed, uint64_t start,
                                         uint64_t count, uint64_t *out, hipStream_t stream) {
    if (count == 0) return PTRHASH_OK;
    if (!out || n == 0 || start > n || count > n - start)
        return ptrhash::set_error(PTRHASH_E_INVAL, "bad query-stream range");
    const Feistel f = make_feistel(n, order_seed);
    hipLaunchKernelGGL(gen_query_k, dim3(8192), dim3(256), 0, stream, key_seed, f, start, count, out);
    return launch_err(hipGetLastError(), "gen_query launch");
}

PTRHASH_API int ptrhash_gen_string_lengths(uint64_t n, uint64_t seed, uint64_t order_seed, int shuffled,
                                           uint64_t start, uint64_t count, uint64_t *lengths, hipStream_t stream) {
    if (count == 0) return PTRHASH_OK;
    if (!lengths || n == 0 || start > n || count > n - start)
        return ptrhash::set_error(PTRHASH_E_INVAL, "bad string range");
    hipLaunchKernelGGL(gen_str_len_k, dim3(8192), dim3(256), 0, stream, seed, make_feistel(n, order_seed),
                       shuffled, start, count, lengths);
    return launch_err(hipGetLastError(), "gen_string_lengths launch");
}

PTRHASH_API int ptrhash_gen_string_bytes(uint64_t n, uint64_t seed, uint64_t order_seed, int shuffled,
                                         uint64_t start, uint64_t count, const uint64_t *offsets, uint8_t *data,
                                         hipStream_t stream) {
    if (count == 0) return PTRHASH_OK;
    if (!offsets || !data || n == 0 || start > n || count > n - start)
        return ptrhash::set_error(PTRHASH_E_INVAL, "bad string range");
    hipLaunchKernelGGL(gen_str_bytes_k, dim3(8192), dim3(256), 0, stream, seed, make_feistel(n, order_seed),
                       shuffled, start, count, offsets, data);
    return launch_err(hipGetLastError(), "gen_string_bytes launch");
}

}  // extern "C"
