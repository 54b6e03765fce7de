// Query kernels for gfx950 and their launchers.
//
// The query of one key is: stream the key in, hash it, find its part and
// bucket, gather the bucket's 8-bit pilot from a table that is usually far
// larger than the L2 caches, compute the slot, decode the remap line for the
// rare slot >= n, stream the index out (Appendix A describes the same
// pipeline on a CPU with software prefetching; here the latency of the
// random pilot gathers is hidden by many independent loads in flight per
// wavefront instead).
//
//  - query_plain: one key per lane, the straightforward form.
//  - query_pipelined<K>: K keys per lane in a tile of K*blockDim keys; all
//    K key loads, then all K pilot gathers, are issued before any result is
//    used (both unconditionally, so that none waits inside a branch). The
//    rare remap reads stay under their slot >= n branch; from 4 keys per
//    lane on, the wavefront's remapped keys are first packed onto its lanes
//    (finish_packed). Keys and indices are streamed with non-temporal loads
//    and stores so that they do not evict pilots from the L2 and MALL.
//  - query_bytes<K>: the same for packed byte-string keys.
//  - query_multi: a persistent launch over many batches, each against its
//    own resident MPHF, described by a table in device memory (stage_in_k
//    copies a plan's table there from mapped host memory).
#include "internal.h"
#include "mphf_device.h"

namespace ptrhash {

template <typename T>
__device__ __forceinline__ T nt_load(const T *p) { return __builtin_nontemporal_load(gbl(p)); }

template <typename OutT>
__device__ __forceinline__ void nt_store(OutT v, OutT *p) { __builtin_nontemporal_store(v, gbl(p)); }

template <typename OutT>
__global__ void __launch_bounds__(1024) query_plain(const uint64_t *__restrict__ keys, uint64_t nq,
                                                    OutT *__restrict__ out, DevMphf m) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint64_t h = hash_u64(gbl(keys)[i]);
    uint32_t part;
    const uint64_t b = bucket_of(m, h, part);
    uint64_t v = slot_of(m, h, part, gbl(m.pilots)[b]);
    if (m.remap_kind != kRemapNone && v >= m.n) v = remap_lookup(m, v);
    out[i] = (OutT)v;
}

// Slots of K keys (already hashed) -> indices: keys with slot >= n read and
// decode their remap entry (divergent; about 1 % of the keys).
template <int K>
__device__ __forceinline__ void finish_k(const DevMphf &m, uint64_t (&v)[K], const bool (&ok)[K]) {
    if (m.remap_kind == kRemapNone) return;
    bool need[K];
#pragma unroll
    for (int j = 0; j < K; ++j) need[j] = ok[j] && v[j] >= m.n;
    if (m.remap_kind == kRemapU32) {
        const uint32_t *R = reinterpret_cast<const uint32_t *>(m.remap);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (need[j]) v[j] = gbl(R)[v[j] - m.n];
        return;
    }
    ClefRead r[K];
    uint32_t idx[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (need[j]) {
            uint64_t line;
            clef_index(v[j] - m.n, line, idx[j]);
            r[j] = clef_load(m.remap, line, idx[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (need[j]) v[j] = clef_value(r[j], idx[j]);
}

// The same with the wavefront's keys that need a remap entry packed onto
// consecutive lanes: each round decodes up to 64 of them with every lane
// busy, instead of one divergent pass per key slot j. When a few percent of
// the keys are remapped (9 % over a fleet of small MPHFs), nearly every
// wavefront has some lane to decode in every pass, so this saves K - 1 of
// K passes. pack: 64 u64 of LDS owned by the wavefront; all its lanes must
// be active.
template <int K>
__device__ __forceinline__ void finish_packed(const DevMphf &m, uint64_t (&v)[K], const bool (&ok)[K],
                                              uint64_t *pack) {
    if (m.remap_kind == kRemapNone) return;
    bool need[K];
    uint32_t pos[K];  // place in the wavefront's list of keys to decode
    uint32_t total = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        need[j] = ok[j] && v[j] >= m.n;
        const uint64_t mask = __ballot(need[j]);
        pos[j] = total + __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        total += (uint32_t)__popcll(mask);
    }
    const uint32_t lane = __lane_id();
    for (uint32_t r0 = 0; r0 < total; r0 += 64) {
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (need[j] && pos[j] - r0 < 64u) pack[pos[j] - r0] = v[j];
        __builtin_amdgcn_wave_barrier();
        if (r0 + lane < total) pack[lane] = remap_lookup(m, pack[lane]);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (need[j] && pos[j] - r0 < 64u) v[j] = pack[pos[j] - r0];
        __builtin_amdgcn_wave_barrier();
    }
}

// One tile of K*stride keys starting at base: lane tid handles keys
// base + tid + j*stride, j < K. Bytes selects packed byte-string keys; a
// string may end at most at end_limit, and one whose offsets decrease or
// pass that limit is not read and gets an index of all ones. Packed decodes
// the remap entries with finish_packed (pack: the wavefront's 64 u64 of
// LDS).
template <int K, typename OutT, bool Bytes, bool Packed = false>
__device__ __forceinline__ void process_tile(const DevMphf &m, const uint64_t *__restrict__ keys,
                                             const uint8_t *__restrict__ data, const uint64_t *__restrict__ offsets,
                                             uint64_t end_limit, uint64_t nq, OutT *__restrict__ out, uint64_t base,
                                             uint32_t stride, uint64_t *pack = nullptr) {
    uint64_t h[K], hs[K];  // hash for part/bucket, hash for the slot
    bool ok[K], bad[K];
    if (Bytes) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint64_t i = base + (uint64_t)j * stride;
            ok[j] = i < nq;
            bad[j] = false;
            h[j] = hs[j] = 0;
            if (ok[j]) {
                const uint64_t o0 = gbl(offsets)[i], o1 = gbl(offsets)[i + 1];
                bad[j] = o1 < o0 || o1 > end_limit;
                if (!bad[j]) h[j] = hash_bytes(m.seed, data, o0, o1 - o0, m.hash128 != 0, hs[j]);
            }
        }
    } else {
        // Every lane loads all K keys unconditionally (a lane past the end
        // reads key 0; nq >= 1), so that the K loads are issued back to back
        // and waited for once: a load under a branch is waited for inside
        // the branch.
        uint64_t key[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint64_t i = base + (uint64_t)j * stride;
            ok[j] = i < nq;
            bad[j] = false;
            key[j] = nt_load(keys + (ok[j] ? i : 0));
        }
#pragma unroll
        for (int j = 0; j < K; ++j) h[j] = hs[j] = hash_u64(key[j]);
    }
    // Any hash maps to a bucket inside the table, so the K pilot gathers are
    // unconditional too.
    uint32_t part[K], pil[K];
#pragma unroll
    for (int j = 0; j < K; ++j) pil[j] = gbl(m.pilots)[bucket_of(m, h[j], part[j])];
    uint64_t v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = slot_of(m, hs[j], part[j], pil[j]);
    if (Packed)
        finish_packed<K>(m, v, ok, pack);
    else
        finish_k<K>(m, v, ok);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t i = base + (uint64_t)j * stride;
        if (ok[j]) nt_store(Bytes && bad[j] ? (OutT)~0ull : (OutT)v[j], out + i);
    }
}

template <int K, typename OutT>
__global__ void __launch_bounds__(1024) query_pipelined(const uint64_t *__restrict__ keys, uint64_t nq,
                                                        OutT *__restrict__ out, DevMphf m) {
    extern __shared__ uint64_t tile_pack[];  // 64 u64 per wavefront when packing
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * K + threadIdx.x;
    process_tile<K, OutT, false, (K >= kPackMinKeys)>(m, keys, nullptr, nullptr, 0, nq, out, base, blockDim.x,
                                                      tile_pack + (threadIdx.x / 64u) * 64u);
}

template <int K, typename OutT>
__global__ void __launch_bounds__(1024) query_bytes_k(const uint8_t *__restrict__ data, uint64_t end_limit,
                                                      const uint64_t *__restrict__ offsets, uint64_t nq,
                                                      OutT *__restrict__ out, DevMphf m) {
    extern __shared__ uint64_t tile_pack[];  // 64 u64 per wavefront when packing
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * K + threadIdx.x;
    process_tile<K, OutT, true, (K >= kPackMinKeys)>(m, nullptr, data, offsets, end_limit, nq, out, base, blockDim.x,
                                                     tile_pack + (threadIdx.x / 64u) * 64u);
}

// Persistent launch over a table of query batches (each against its own
// resident MPHF). Every batch is cut into tiles of K*blockDim keys (the
// table records the tile size it was numbered with); tiles are numbered
// globally (tile_begin is a prefix sum), so batches of any mix of sizes
// share one launch. The table groups the batches by MPHF, and the workgroups
// of each die take one contiguous range of the tiles (an eighth of the
// estimated work, die_first), so a die's L2 holds the pilots and remap lines
// of about an eighth of the MPHFs instead of all of them. The header (batch
// count, tile count, the dies' ranges) lives in device memory next to the
// batches, so a captured launch can be replayed over new batches. Remap
// entries are decoded packed (finish_packed), in 64 u64 of dynamic LDS per
// wavefront (multi_lds_bytes).
template <int K>
__global__ void __launch_bounds__(1024) query_multi(const MultiTable *__restrict__ table) {
    const uint32_t count = table->count;
    const uint64_t tiles = table->tiles;
    const uint32_t tile = table->tile;
    if (tile != (uint32_t)K * blockDim.x) return;  // table numbered for another launch shape
    extern __shared__ uint64_t multi_pack[];
    uint64_t *pack = multi_pack + (threadIdx.x / 64u) * 64u;
    const uint64_t *__restrict__ tb = multi_tile_begin(table);
    const MultiBatch *__restrict__ bt = multi_batches(table);
    const DevMphf *__restrict__ mp = multi_mphfs(table);
    uint64_t first = blockIdx.x, end = tiles, step = gridDim.x;
    if (gridDim.x % kDies == 0) {
        const uint32_t x = blockIdx.x % kDies;
        first = table->die_first[x] + blockIdx.x / kDies;
        end = table->die_first[x + 1];
        step = gridDim.x / kDies;
    }
    const uint32_t lane = __lane_id();
    for (uint64_t t = first; t < end; t += step) {
        // The last batch whose first tile is <= t, found by each wavefront
        // with 64 reads in parallel per round: the lanes read every
        // stride-th first tile of the remaining range and the highest lane
        // whose tile is <= t narrows it to one stride (two rounds for 4096
        // batches instead of twelve dependent reads). tb[0] = 0 <= t, so the
        // ballot is never empty.
        uint32_t lo = 0, n = count;
        while (n > 1) {
            const uint32_t stride = (n + 63) / 64;
            const uint32_t off = lane * stride;
            const bool le = off < n && tb[lo + off] <= t;
            const uint64_t mask = __ballot(le);
            const uint32_t hit = 63u - (uint32_t)__clzll(mask);
            lo += hit * stride;
            n = n - hit * stride < stride ? n - hit * stride : stride;
        }
        const MultiBatch &q = bt[lo];
        const DevMphf &m = mp[q.mphf];
        const uint64_t base = (t - tb[lo]) * (uint64_t)tile + threadIdx.x;
        if (q.flags & kBatchBytes) {
            const uint8_t *data = static_cast<const uint8_t *>(q.keys);
            if (q.flags & kBatchOut64)
                process_tile<K, uint64_t, true, true>(m, nullptr, data, q.offsets, q.end_limit, q.nq,
                                                      static_cast<uint64_t *>(q.out), base, blockDim.x, pack);
            else
                process_tile<K, uint32_t, true, true>(m, nullptr, data, q.offsets, q.end_limit, q.nq,
                                                      static_cast<uint32_t *>(q.out), base, blockDim.x, pack);
        } else {
            const uint64_t *keys = static_cast<const uint64_t *>(q.keys);
            if (q.flags & kBatchOut64)
                process_tile<K, uint64_t, false, true>(m, keys, nullptr, nullptr, 0, q.nq,
                                                       static_cast<uint64_t *>(q.out), base, blockDim.x, pack);
            else
                process_tile<K, uint32_t, false, true>(m, keys, nullptr, nullptr, 0, q.nq,
                                                       static_cast<uint32_t *>(q.out), base, blockDim.x, pack);
        }
    }
}

// The batch table copied from mapped host memory into device memory by a
// kernel on the launch's own stream. A copy-engine transfer instead needs a
// hand-off between the copy and compute queues before every launch (about
// 20-60 us per step, the copy itself being 10 us).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) stage_in_k(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, uint64_t n16) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
        gbl(dst)[i] = gbl(src)[i];
}

// ---- launchers ----

static inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// A dispatch holds fewer than 2^32 work-items (grid times block), so a large
// batch is split into launches of at most 2^31 / block workgroups each, one
// after the other on the same stream.
static inline uint64_t keys_per_launch(uint32_t block, int K) {
    return (uint64_t)(0x80000000u / block) * block * (uint64_t)K;
}

// Dynamic LDS of a single-MPHF launch: the occupancy cap's reservation, at
// least the packed decode's 64 u64 per wavefront when the kernel packs.
static inline uint32_t launch_lds(const Tuning &t, int K) {
    const uint32_t pack = K >= kPackMinKeys ? pack_lds_bytes((uint32_t)t.block) : 0u;
    return t.lds_bytes > pack ? t.lds_bytes : pack;
}

template <typename OutT>
static hipError_t launch_u64_t(const DevMphf &m, const uint64_t *keys, uint64_t nq, void *out, const Tuning &t,
                               hipStream_t s) {
    OutT *o = static_cast<OutT *>(out);
    const uint32_t blk = (uint32_t)t.block;
    const int K = t.kernel == kKernelPlain ? 1 : t.keys_per_lane;
    const uint64_t chunk = keys_per_launch(blk, K);
    const uint32_t lds = launch_lds(t, K);
    for (uint64_t s0 = 0; s0 < nq; s0 += chunk) {
        const uint64_t n = nq - s0 < chunk ? nq - s0 : chunk;
        const dim3 grid((uint32_t)ceil_div(n, (uint64_t)blk * K));
        if (t.kernel == kKernelPlain) {
            hipLaunchKernelGGL(query_plain<OutT>, grid, dim3(blk), t.lds_bytes, s, keys + s0, n, o + s0, m);
        } else {
            switch (K) {
#define PTRHASH_CASE(KK)                                                                                      \
    case KK:                                                                                                  \
        hipLaunchKernelGGL((query_pipelined<KK, OutT>), grid, dim3(blk), lds, s, keys + s0, n, o + s0, m);         \
        break;
                PTRHASH_CASE(1)
                PTRHASH_CASE(2)
                PTRHASH_CASE(4)
                PTRHASH_CASE(8)
                PTRHASH_CASE(16)
#undef PTRHASH_CASE
            default:
                return hipErrorInvalidValue;
            }
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_query_u64(const DevMphf &m, const uint64_t *keys, uint64_t nq, void *out, bool out64,
                            const Tuning &t, hipStream_t s) {
    return out64 ? launch_u64_t<uint64_t>(m, keys, nq, out, t, s) : launch_u64_t<uint32_t>(m, keys, nq, out, t, s);
}

template <typename OutT>
static hipError_t launch_bytes_t(const DevMphf &m, const uint8_t *data, uint64_t end_limit, const uint64_t *offsets,
                                 uint64_t nq, void *out, const Tuning &t, hipStream_t s) {
    OutT *o = static_cast<OutT *>(out);
    const uint32_t blk = (uint32_t)t.block;
    const int K = t.kernel == kKernelPlain ? 1 : t.keys_per_lane;
    const uint64_t chunk = keys_per_launch(blk, K);
    const uint32_t lds = launch_lds(t, K);
    for (uint64_t s0 = 0; s0 < nq; s0 += chunk) {
        const uint64_t n = nq - s0 < chunk ? nq - s0 : chunk;
        const dim3 grid((uint32_t)ceil_div(n, (uint64_t)blk * K));
        switch (K) {
#define PTRHASH_CASE(KK)                                                                                      \
    case KK:                                                                                                  \
        hipLaunchKernelGGL((query_bytes_k<KK, OutT>), grid, dim3(blk), lds, s, data, end_limit,               \
                           offsets + s0, n, o + s0, m);                                                       \
        break;
            PTRHASH_CASE(1)
            PTRHASH_CASE(2)
            PTRHASH_CASE(4)
            PTRHASH_CASE(8)
            PTRHASH_CASE(16)
#undef PTRHASH_CASE
        default:
            return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_query_bytes(const DevMphf &m, const uint8_t *data, uint64_t end_limit, const uint64_t *offsets,
                              uint64_t nq, void *out, bool out64, const Tuning &t, hipStream_t s) {
    return out64 ? launch_bytes_t<uint64_t>(m, data, end_limit, offsets, nq, out, t, s)
                 : launch_bytes_t<uint32_t>(m, data, end_limit, offsets, nq, out, t, s);
}

template <typename F>
static hipError_t with_multi_kernel(int K, F &&f) {
    switch (K) {
    case 1: return f(query_multi<1>);
    case 2: return f(query_multi<2>);
    case 4: return f(query_multi<4>);
    case 8: return f(query_multi<8>);
    default: return hipErrorInvalidValue;
    }
}

int multi_blocks_per_cu(const MultiTuning &t) {
    int blocks = 0;
    const hipError_t e = with_multi_kernel(t.keys_per_lane, [&](auto kern) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, t.block, multi_lds_bytes(t));
    });
    return e == hipSuccess && blocks > 0 ? blocks : 1;
}

hipError_t launch_query_multi(const MultiTable *table, const MultiTuning &t, uint32_t grid, hipStream_t s) {
    const hipError_t e = with_multi_kernel(t.keys_per_lane, [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3((uint32_t)t.block), multi_lds_bytes(t), s, table);
        return hipSuccess;
    });
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_stage_in(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const uint64_t n16 = (bytes + 15) / 16;
    if (n16 == 0) return hipSuccess;
    const uint64_t blocks = (n16 + 255) / 256 < 1024 ? (n16 + 255) / 256 : 1024;
    hipLaunchKernelGGL(stage_in_k, dim3((uint32_t)blocks), dim3(256), 0, s, static_cast<const u32x4 *>(src),
                       static_cast<u32x4 *>(dst), n16);
    return hipGetLastError();
}

}  // namespace ptrhash
