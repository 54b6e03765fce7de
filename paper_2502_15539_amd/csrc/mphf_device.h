// Device-side evaluation of one PtrHash MPHF (gfx950).
//
// Everything here is 64-bit integer arithmetic: the key hash
// (Section 3.1, "Hash functions"), part/bucket (eq. partbucket, Section
// 3.3), the pilot hash and slot (eq. slot, "The reduce function") and the
// CacheLineEF lookup for slots >= n (Section 3.4, "Lookup"). No floating
// point and no matrix cores are involved.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptrhash {

// Global-memory views of pointers. Everything the queries read or write
// (keys, pilots, remap, outputs, batch tables) is device memory or mapped
// host memory, never LDS or scratch. Pointers that reach a kernel through a
// table in memory are otherwise generic, and a generic (flat) access counts
// against the LDS/scalar wait counter as well as the vector one, so that a
// wait for a scalar table read also waits for every pilot gather in flight.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gbl(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gbl(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// FxHash mixing constant (odd, so x -> C*x is a bijection of u64).
constexpr uint64_t kMix = 0x517cc1b727220a95ull;

enum : uint32_t { kGammaCubic = 0, kGammaLinear = 1 };
enum : uint32_t { kRemapClef = 0, kRemapU32 = 1, kRemapNone = 2 };
enum : uint32_t { kReducePow2 = 0, kReduceMod = 1 };

// One resident MPHF as the kernels see it (passed by value).
struct DevMphf {
    const uint8_t *pilots;  // P*B bytes, global bucket index
    const uint8_t *remap;   // CacheLineEF lines or u32 entries
    uint64_t n;
    uint64_t seed;
    uint32_t parts;         // P (< 2^32)
    uint32_t buckets;       // B (< 2^32)
    uint32_t log2_slots;    // S = 2^log2_slots
    uint32_t gamma;
    uint32_t remap_kind;
    uint32_t reduce_kind;
    uint32_t mod_slots;     // S for the mod reduce (one part)
    uint64_t mod_magic;     // floor(2^64 / S) for the mod reduce
    uint32_t hash128;       // byte keys: 128-bit hash (high half: part/bucket, low half: slot)
    uint32_t pad_;
};

// Seed of the low half of a 128-bit byte hash.
constexpr uint64_t kWideSalt = 0x9E3779B97F4A7C15ull;

// hi and lo 64-bit halves of a (32-bit) * b (64-bit): two 32x32->64
// multiplies instead of a full 64x64 product.
__device__ __forceinline__ void mul32x64(uint32_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
    const uint64_t p0 = (uint64_t)a * (uint32_t)b;
    const uint64_t p1 = (uint64_t)a * (uint32_t)(b >> 32);
    const uint64_t mid = p1 + (p0 >> 32);  // <= 2^64 - 2^32, no overflow
    hi = mid >> 32;
    lo = (mid << 32) | (uint32_t)p0;
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// Integer keys: h(k) = C*k mod 2^64.
__device__ __forceinline__ uint64_t hash_u64(uint64_t k) { return kMix * k; }

// gamma_1(x) = x; gamma_3(x) = (255/256)(x^2+x^3)/2 + x/256 in 64-bit fixed
// point, x^2 = hi(x*x), x^3 = hi(x^2*x) (Section 3.3, "Approximations").
__device__ __forceinline__ uint64_t gamma_fn(uint32_t kind, uint64_t x) {
    if (kind == kGammaLinear) return x;
    const uint64_t x2 = mulhi64(x, x);
    const uint64_t x3 = mulhi64(x2, x);
    const uint64_t y = (x2 >> 1) + (x3 >> 1);
    return y - (y >> 8) + (x >> 8);
}

// part = hi(P*h), x = lo(P*h), bucket = part*B + hi(B*gamma(x)).
__device__ __forceinline__ uint64_t bucket_of(const DevMphf &m, uint64_t h, uint32_t &part) {
    uint64_t phi, x;
    mul32x64(m.parts, h, phi, x);
    part = (uint32_t)phi;
    uint64_t b, unused;
    mul32x64(m.buckets, gamma_fn(m.gamma, x), b, unused);
    (void)unused;
    return (uint64_t)part * m.buckets + b;
}

// x mod S for S < 2^32, not a power of two: q = hi(x * floor(2^64/S)) is
// floor(x/S) or one less, so one conditional subtraction fixes the rest.
__device__ __forceinline__ uint64_t mod_reduce(uint64_t x, uint32_t S, uint64_t magic) {
    uint64_t r = x - mulhi64(x, magic) * S;
    return r >= S ? r - S : r;
}

// slot = part*S + reduce(h xor C*(pilot xor seed), S) with reduce(x, S) =
// hi(C*x) mod S (S a power of two) or x mod S (one part).
__device__ __forceinline__ uint64_t slot_of(const DevMphf &m, uint64_t h, uint32_t part, uint32_t pilot) {
    const uint64_t hp = kMix * ((uint64_t)pilot ^ m.seed);
    if (m.reduce_kind == kReduceMod) return mod_reduce(h ^ hp, m.mod_slots, m.mod_magic);
    const uint64_t local = mulhi64(kMix, h ^ hp) & ((1ull << m.log2_slots) - 1);
    return ((uint64_t)part << m.log2_slots) | local;
}

// Position of the r-th (from 0) set bit of w; w must hold more than r ones.
// Binary search on popcounts of halves (no PDEP on this target).
__device__ __forceinline__ uint32_t select64(uint64_t w, uint32_t r) {
    uint32_t pos = 0, c;
    c = __popc((uint32_t)w);
    if (r >= c) { r -= c; w >>= 32; pos += 32; }
    c = __popc((uint32_t)w & 0xffffu);
    if (r >= c) { r -= c; w >>= 16; pos += 16; }
    c = __popc((uint32_t)w & 0xffu);
    if (r >= c) { r -= c; w >>= 8; pos += 8; }
    c = __popc((uint32_t)w & 0xfu);
    if (r >= c) { r -= c; w >>= 4; pos += 4; }
    c = __popc((uint32_t)w & 0x3u);
    if (r >= c) { r -= c; w >>= 2; pos += 2; }
    c = (uint32_t)w & 1u;
    if (r >= c) pos += 1;
    return pos;
}

// One CacheLineEF line as held in registers: offset, the 128 high bits and
// the needed low byte.
struct ClefRead {
    uint32_t off, b0, b1, b2, b3, low;
};

__device__ __forceinline__ void clef_index(uint64_t j, uint64_t &line, uint32_t &i) {
    line = j / 44u;
    i = (uint32_t)(j - line * 44u);
}

__device__ __forceinline__ ClefRead clef_load(const uint8_t *remap, uint64_t line, uint32_t i) {
    const uint8_t *L = remap + line * 64u;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 a = *gbl(reinterpret_cast<const u32x4 *>(L));           // off, bits 0..95
    const uint32_t d4 = *gbl(reinterpret_cast<const uint32_t *>(L + 16));  // bits 96..127
    ClefRead r;
    r.off = a.x;
    r.b0 = a.y;
    r.b1 = a.z;
    r.b2 = a.w;
    r.b3 = d4;
    r.low = gbl(L)[20 + i];
    return r;
}

// v_i = 2^8*offset + 2^8*(select(i) - i) + low_i (Section 3.4, "Lookup").
__device__ __forceinline__ uint64_t clef_value(const ClefRead &r, uint32_t i) {
    const uint64_t lo = (uint64_t)r.b0 | ((uint64_t)r.b1 << 32);
    const uint64_t hi = (uint64_t)r.b2 | ((uint64_t)r.b3 << 32);
    const uint32_t c = (uint32_t)__popcll(lo);
    const uint32_t sel = i < c ? select64(lo, i) : 64u + select64(hi, i - c);
    return 256ull * r.off + 256ull * (sel - i) + r.low;
}

__device__ __forceinline__ uint64_t remap_lookup(const DevMphf &m, uint64_t slot) {
    const uint64_t j = slot - m.n;
    if (m.remap_kind == kRemapU32) return gbl(reinterpret_cast<const uint32_t *>(m.remap))[j];
    uint64_t line;
    uint32_t i;
    clef_index(j, line, i);
    return clef_value(clef_load(m.remap, line, i), i);
}

// MurmurHash3 fmix64 finalizer (Appleby).
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Byte-string hash (the library's stand-in for GxHash): st = seed ^ len*C;
// each little-endian 8-byte word w (last one zero padded): st = fmix64(st ^ w);
// h = fmix64(st). data must be 8-byte aligned with readable bytes up to the
// next 8-byte boundary after the string plus 8; words are read aligned and
// funnel shifted.
// With wide set, lo receives the same hash under seed ^ kWideSalt (the two
// chains share the word loads).
__device__ __forceinline__ uint64_t hash_bytes(uint64_t seed, const uint8_t *data, uint64_t o0, uint64_t len,
                                               bool wide, uint64_t &lo) {
    uint64_t st = seed ^ (len * kMix);
    uint64_t st2 = (seed ^ kWideSalt) ^ (len * kMix);
    const auto W = gbl(reinterpret_cast<const uint64_t *>(data + (o0 & ~7ull)));
    const uint32_t sh = (uint32_t)(o0 & 7u) * 8u;
    uint64_t cur = W[0];
    const uint64_t nw = (len + 7) >> 3;
    for (uint64_t w = 0; w < nw; ++w) {
        const uint64_t nxt = W[w + 1];
        uint64_t word = sh ? (cur >> sh) | (nxt << (64u - sh)) : cur;
        const uint64_t rem = len - 8 * w;
        if (rem < 8) word &= (1ull << (8 * rem)) - 1;
        st = fmix64(st ^ word);
        if (wide) st2 = fmix64(st2 ^ word);
        cur = nxt;
    }
    const uint64_t hi = fmix64(st);
    lo = wide ? fmix64(st2) : hi;
    return hi;
}

}  // namespace ptrhash
