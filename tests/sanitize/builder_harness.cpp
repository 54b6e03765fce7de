// The library's host construction (builder.cpp) on the CPU under
// AddressSanitizer and UBSan: u64 keys at several sizes with the Default,
// Fast, single-part mod and non-minimal settings, duplicate detection, and
// byte strings of lengths 8..78 with 64- and 128-bit hashes. The two
// functions builder.cpp takes from the rest of the library (the error
// message and the remap size) are restated here so that no GPU code is
// linked. Test infrastructure only.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>
#include "ptrhash.h"

namespace ptrhash {
int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap; va_start(ap, fmt); vsnprintf(buf, sizeof buf, fmt, ap); va_end(ap);
    return code;
}
}
extern "C" uint64_t ptrhash_remap_bytes(const ptrhash_params *p) {
    if (!p) return 0;
    if (p->remap_kind == PTRHASH_REMAP_CLEF) return (p->remap_len + 43) / 44 * 64;
    if (p->remap_kind == PTRHASH_REMAP_U32) return p->remap_len * 4;
    return 0;
}
static uint64_t next_pow2(uint64_t v) { uint64_t r = 1; while (r < v) r <<= 1; return r; }
static ptrhash_params params(uint64_t n, double lambda, uint32_t gamma, uint32_t remap, uint32_t key_kind, bool mod, uint32_t hb) {
    const double alpha = 0.99;
    double kpp = 80000.0 * std::log((double)n / 80000.0); if (kpp < 80000.0) kpp = 80000.0;
    uint64_t S = next_pow2((uint64_t)std::ceil(kpp / alpha));
    uint64_t P = (uint64_t)std::ceil((double)n / (alpha * (double)S)); if (P < 1) P = 1;
    if (P == 1) S = next_pow2((uint64_t)std::ceil((double)n / alpha));
    ptrhash_params p{}; p.n = n; p.num_parts = P; p.gamma = gamma; p.remap_kind = remap; p.key_kind = key_kind;
    p.index_bits = n <= (1ull << 32) ? 32 : 64; p.hash_bits = hb;
    if (mod && P == 1) {
        uint64_t Sm = (uint64_t)std::ceil((double)n / alpha); if (Sm < n + 16) Sm = n + 16; if ((Sm & (Sm - 1)) == 0) ++Sm;
        p.reduce_kind = PTRHASH_REDUCE_MOD; p.slots = Sm; p.log2_slots = 0;
        p.buckets_per_part = (uint32_t)std::ceil(alpha * (double)Sm / lambda); p.remap_len = Sm - n;
    } else {
        uint32_t l = 0; while ((1ull << l) < S) ++l; p.log2_slots = l;
        p.buckets_per_part = (uint32_t)std::ceil(alpha * (double)S / lambda); p.remap_len = P * S - n;
    }
    return p;
}
static uint64_t sm(uint64_t x) { x += 0x9e3779b97f4a7c15ull; x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull; x = (x ^ (x >> 27)) * 0x94d049bb133111ebull; return x ^ (x >> 31); }
int main() {
    int fails = 0;
    const uint64_t sizes[] = {1, 2, 3, 17, 100, 1000, 65537, 300000, 1000000};
    for (uint64_t n : sizes) {
        std::vector<uint64_t> keys(n); for (uint64_t i = 0; i < n; ++i) keys[i] = sm(i * 7 + 1);
        struct { double lam; uint32_t g, r; bool mod; } cfgs[] = {{3.5, 0, 0, false}, {3.0, 1, 1, false}, {3.5, 0, 0, true}, {3.5, 0, 2, false}};
        for (auto &c : cfgs) {
            if (c.lam == 3.0 && n > 300000) continue;
            ptrhash_params p = params(n, c.lam, c.g, c.r, PTRHASH_KEY_U64, c.mod, 64);
            std::vector<uint8_t> pil(p.num_parts * p.buckets_per_part), rem(ptrhash_remap_bytes(&p) + 1);
            ptrhash_build_info info{};
            int rc = ptrhash_build_u64(keys.data(), n, &p, pil.data(), rem.data(), 4, &info);
            if (rc) { std::printf("u64 n=%llu cfg lam=%.1f mod=%d rc=%d\n", (unsigned long long)n, c.lam, c.mod, rc); ++fails; }
        }
        // duplicates must be refused
        if (n >= 2) {
            std::vector<uint64_t> d = keys; d[n - 1] = d[0];
            ptrhash_params p = params(n, 3.5, 0, 0, PTRHASH_KEY_U64, false, 64);
            std::vector<uint8_t> pil(p.num_parts * p.buckets_per_part), rem(ptrhash_remap_bytes(&p) + 1);
            int rc = ptrhash_build_u64(d.data(), n, &p, pil.data(), rem.data(), 2, nullptr);
            if (rc != PTRHASH_E_DUPLICATE) { std::printf("dup n=%llu rc=%d\n", (unsigned long long)n, rc); ++fails; }
        }
    }
    // strings, 64- and 128-bit hashes, edge lengths 0..70
    for (uint64_t n : {1ull, 5ull, 1000ull, 50000ull}) {
        for (uint32_t hb : {64u, 128u}) {
            std::vector<uint64_t> off(n + 1); std::vector<uint8_t> data;
            for (uint64_t i = 0; i < n; ++i) {
                off[i] = data.size(); uint64_t r = sm(i + 99); uint64_t len = r % 71;
                for (uint64_t j = 0; j < len; ++j) data.push_back((uint8_t)(sm(r + j) & 0xff));
                uint64_t tag = i; for (int b = 0; b < 8; ++b) data.push_back((uint8_t)(tag >> (8 * b)));  // distinct
            }
            off[n] = data.size(); data.resize(data.size() + 72, 0);
            while (data.size() % 8) data.push_back(0);
            ptrhash_params p = params(n, 3.5, 0, 0, PTRHASH_KEY_BYTES, false, hb);
            std::vector<uint8_t> pil(p.num_parts * p.buckets_per_part), rem(ptrhash_remap_bytes(&p) + 1);
            int rc = ptrhash_build_bytes(data.data(), data.size(), off.data(), n, &p, pil.data(), rem.data(), 4, nullptr);
            if (rc) { std::printf("bytes n=%llu hb=%u rc=%d\n", (unsigned long long)n, hb, rc); ++fails; }
        }
    }
    std::printf("asan harness done, %d failures\n", fails);
    return fails != 0;
}
