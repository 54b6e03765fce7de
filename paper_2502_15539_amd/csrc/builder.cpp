// Host construction of a PtrHash MPHF (Section 3.2 "Construction",
// Section 3.4 "Remapping"), multi-threaded over parts.
//
// Parts are independent (Section 3.1: each part owns its own S slots), so
// worker threads take parts from a shared counter. Inside a part, buckets are
// placed largest first with hash-evict pilot search: the smallest pilot in
// [0, 256) whose slots are free and distinct; otherwise the pilot with the
// least sum over colliding keys of (size of the bucket owning the slot)^2,
// skipping pilots that would evict one of the 16 most recently placed
// buckets; the owners are evicted and requeued. A part fails after more than
// 10*S evictions and the whole construction restarts with seed + 1.
// Ties are resolved the deterministic way (largest bucket first, then the
// smaller bucket id; the smallest pilot among equal costs), so a build is a
// pure function of the keys and the parameters.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <queue>
#include <thread>
#include <vector>

#include "builder.h"
#include "errors.h"
#include "ptrhash.h"

namespace {

using u128 = unsigned __int128;
constexpr uint64_t kMix = 0x517cc1b727220a95ull;
constexpr int32_t kEmpty = -1;
constexpr int kRecent = 16;
constexpr int kEvictionFactor = 10;
constexpr int kMaxSeeds = 16;
constexpr uint64_t kWideSalt = 0x9E3779B97F4A7C15ull;  // seed of the low half of a 128-bit byte hash

inline uint64_t mul_hi(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) >> 64); }
inline uint64_t mul_lo(uint64_t a, uint64_t b) { return a * b; }

inline uint64_t fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Byte-string hash: st = seed ^ len*C; st = fmix64(st ^ w) for each
// little-endian 8-byte word (the last one zero padded); h = fmix64(st).
uint64_t hash_bytes(uint64_t seed, const uint8_t *s, uint64_t len) {
    uint64_t st = seed ^ (len * kMix);
    uint64_t i = 0;
    for (; i + 8 <= len; i += 8) {
        uint64_t w;
        std::memcpy(&w, s + i, 8);
        st = fmix64(st ^ w);
    }
    if (i < len) {
        uint64_t w = 0;
        std::memcpy(&w, s + i, len - i);
        st = fmix64(st ^ w);
    }
    return fmix64(st);
}

struct Geometry {
    uint64_t n, P, S, B, seed;
    uint32_t log2S, gamma;
    bool mod = false;  // reduce(x, S) = x mod S (one part) instead of hi(C*x) mod 2^log2S

    uint32_t part(uint64_t h) const { return (uint32_t)mul_hi(P, h); }
    uint32_t local_bucket(uint64_t h) const {
        const uint64_t x = mul_lo(P, h);
        uint64_t g = x;
        if (gamma == PTRHASH_GAMMA_CUBIC) {
            const uint64_t x2 = mul_hi(x, x);
            const uint64_t x3 = mul_hi(x2, x);
            const uint64_t y = (x2 >> 1) + (x3 >> 1);
            g = y - (y >> 8) + (x >> 8);
        }
        return (uint32_t)mul_hi(B, g);
    }
};

enum PartStatus { kPartOk = 0, kPartFailed = 1 };

// Scratch of one worker thread, reused across parts.
struct PartWorker {
    const Geometry *geo = nullptr;
    std::vector<int32_t> owner;      // local slot -> local bucket
    std::vector<uint64_t> taken;     // local slot bitmap (the paper's taken-slot bitvector)
    std::vector<uint32_t> stamp;     // local slot -> last trial that touched it (large buckets)
    uint32_t cur = 0;
    std::vector<uint32_t> bstart;    // local bucket -> offset into bh
    std::vector<uint64_t> bh;        // hashes grouped by local bucket (when regrouped)
    const uint64_t *bhp = nullptr;   // the part's hashes grouped by local bucket
    std::vector<uint64_t> bs;        // slot hashes grouped alike (128-bit byte keys)
    const uint64_t *bsp = nullptr;   // slot hashes grouped by local bucket (= bhp for 64-bit hashes)
    std::vector<int64_t> last;       // local bucket -> placement number
    std::vector<uint32_t> slots;     // slots of the bucket being placed
    uint64_t hp[256];
    uint64_t evictions = 0, max_bucket = 0;

    void init(const Geometry *g) {
        geo = g;
        owner.assign(g->S, kEmpty);
        taken.assign((g->S + 63) / 64, 0);
        stamp.assign(g->S, 0);
        cur = 0;
        bstart.assign(g->B + 1, 0);
        last.assign(g->B, 0);
        for (uint32_t p = 0; p < 256; ++p) hp[p] = kMix * ((uint64_t)p ^ g->seed);
    }

    uint32_t next_stamp() {
        if (++cur == 0) {  // wrapped: clear and restart
            std::fill(stamp.begin(), stamp.end(), 0u);
            cur = 1;
        }
        return cur;
    }

    bool is_taken(uint32_t q) const { return (taken[q >> 6] >> (q & 63)) & 1u; }
    void set_owner(uint32_t q, int32_t b) {
        owner[q] = b;
        if (b == kEmpty)
            taken[q >> 6] &= ~(1ull << (q & 63));
        else
            taken[q >> 6] |= 1ull << (q & 63);
    }

    // Slots of a bucket's keys under pilot p; true if they are distinct
    // (pairwise for small buckets, trial stamps for large ones).
    static constexpr uint32_t kPairwise = 16;
    bool distinct_slots(const uint64_t *kh, uint32_t s, uint32_t p, uint32_t *out) {
        if (s <= kPairwise) {
            for (uint32_t j = 0; j < s; ++j) {
                const uint32_t q = slot(kh[j], p);
                for (uint32_t i = 0; i < j; ++i)
                    if (out[i] == q) return false;
                out[j] = q;
            }
            return true;
        }
        const uint32_t st = next_stamp();
        for (uint32_t j = 0; j < s; ++j) {
            const uint32_t q = slot(kh[j], p);
            if (stamp[q] == st) return false;
            stamp[q] = st;
            out[j] = q;
        }
        return true;
    }

    uint32_t slot(uint64_t h, uint32_t p) const {
        return geo->mod ? (uint32_t)((h ^ hp[p]) % geo->S) : (uint32_t)(mul_hi(kMix, h ^ hp[p]) & (geo->S - 1));
    }

    // Group the part's hashes by local bucket (counting sort).
    void group(const uint64_t *h, const uint64_t *h2, uint64_t cnt) {
        std::fill(bstart.begin(), bstart.end(), 0u);
        for (uint64_t i = 0; i < cnt; ++i) bstart[geo->local_bucket(h[i]) + 1]++;
        for (uint64_t b = 0; b < geo->B; ++b) bstart[b + 1] += bstart[b];
        bh.resize(cnt);
        std::vector<uint32_t> fill(bstart.begin(), bstart.end() - 1);
        if (h2) {
            bs.resize(cnt);
            for (uint64_t i = 0; i < cnt; ++i) {
                const uint32_t d = fill[geo->local_bucket(h[i])]++;
                bh[d] = h[i];
                bs[d] = h2[i];
            }
            bhp = bh.data();
            bsp = bs.data();
            return;
        }
        for (uint64_t i = 0; i < cnt; ++i) bh[fill[geo->local_bucket(h[i])]++] = h[i];
        bhp = bsp = bh.data();
    }

    // Hashes sorted ascending are already grouped by bucket (the bucket index
    // is non-decreasing in the hash); only the bucket offsets are needed.
    void group_sorted(const uint64_t *h, uint64_t cnt) {
        std::fill(bstart.begin(), bstart.end(), 0u);
        for (uint64_t i = 0; i < cnt; ++i) bstart[geo->local_bucket(h[i]) + 1]++;
        for (uint64_t b = 0; b < geo->B; ++b) bstart[b + 1] += bstart[b];
        bhp = bsp = h;
    }

    // True if two keys of one bucket share their (bucket, slot) hashes.
    bool has_equal_hashes() {
        std::vector<std::pair<uint64_t, uint64_t>> tmp;
        for (uint64_t b = 0; b < geo->B; ++b) {
            const uint32_t s = bstart[b + 1] - bstart[b];
            if (s < 2) continue;
            tmp.clear();
            for (uint32_t j = bstart[b]; j < bstart[b + 1]; ++j) tmp.emplace_back(bhp[j], bsp[j]);
            std::sort(tmp.begin(), tmp.end());
            if (std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end()) return true;
        }
        return false;
    }

    PartStatus place(uint8_t *pilots /* this part's B pilots */, uint64_t max_evictions) {
        const uint32_t B = (uint32_t)geo->B;
        std::fill(owner.begin(), owner.end(), kEmpty);
        std::fill(taken.begin(), taken.end(), 0ull);
        std::priority_queue<uint64_t> heap;  // (size << 32) | (~id): big first, then small id
        uint64_t maxs = 0;
        for (uint32_t b = 0; b < B; ++b) {
            pilots[b] = 0;
            last[b] = INT64_MIN / 2;
            const uint64_t s = bstart[b + 1] - bstart[b];
            if (s) heap.push((s << 32) | (0xffffffffu - b));
            maxs = std::max(maxs, s);
        }
        max_bucket = std::max(max_bucket, maxs);
        slots.resize(std::max<uint64_t>(maxs, 1));
        uint32_t *sl = slots.data();
        int64_t placed = 0;
        uint64_t ev = 0;
        auto size_of = [&](uint32_t b) { return (uint64_t)(bstart[b + 1] - bstart[b]); };
        while (!heap.empty()) {
            const uint32_t b = 0xffffffffu - (uint32_t)(heap.top() & 0xffffffffu);
            heap.pop();
            const uint64_t *kh = bsp + bstart[b];
            const uint32_t s = (uint32_t)size_of(b);
            int chosen = -1;
            // 1) smallest pilot with distinct, free slots
            if (s == 1) {
                for (uint32_t p = 0; p < 256; ++p)
                    if (!is_taken(slot(kh[0], p))) { chosen = (int)p; break; }
            } else {
                for (uint32_t p = 0; p < 256 && chosen < 0; ++p) {
                    bool ok = true;
                    for (uint32_t j = 0; j < s; ++j)
                        if (is_taken(slot(kh[j], p))) { ok = false; break; }
                    if (ok && distinct_slots(kh, s, p, sl)) chosen = (int)p;
                }
            }
            if (chosen < 0) {
                // 2) least weighted collisions, never touching the recent ones
                uint64_t best = UINT64_MAX;
                for (uint32_t p = 0; p < 256; ++p) {
                    if (!distinct_slots(kh, s, p, sl)) continue;
                    uint64_t cost = 0;
                    bool ok = true;
                    for (uint32_t j = 0; j < s; ++j) {
                        const int32_t o = owner[sl[j]];
                        if (o == kEmpty) continue;
                        if (last[o] + kRecent > placed) { ok = false; break; }
                        const uint64_t so = size_of((uint32_t)o);
                        cost += so * so;
                    }
                    if (ok && cost < best) { best = cost; chosen = (int)p; }
                }
                if (chosen < 0) return kPartFailed;
                for (uint32_t j = 0; j < s; ++j) {
                    const int32_t o = owner[slot(kh[j], (uint32_t)chosen)];
                    if (o == kEmpty) continue;
                    const uint64_t *oh = bsp + bstart[o];
                    const uint32_t os = (uint32_t)size_of((uint32_t)o);
                    for (uint32_t t = 0; t < os; ++t) set_owner(slot(oh[t], pilots[o]), kEmpty);
                    heap.push(((uint64_t)os << 32) | (0xffffffffu - (uint32_t)o));
                    ++ev;
                }
            }
            for (uint32_t j = 0; j < s; ++j) set_owner(slot(kh[j], (uint32_t)chosen), (int32_t)b);
            pilots[b] = (uint8_t)chosen;
            last[b] = ++placed;
            if (ev > max_evictions) return kPartFailed;
        }
        evictions = ev;
        return kPartOk;
    }
};

struct Partitioned {
    std::vector<uint64_t> hashes;   // grouped by part
    std::vector<uint64_t> slot_hashes;  // 128-bit byte keys: low halves, same order
    bool sorted = false;            // hashes sorted ascending (grouped by bucket too)
    std::vector<uint64_t> ids;      // key ids in the same order (byte keys only)
    std::vector<uint64_t> start;    // part -> offset, P+1 entries
};

int pick_threads(int threads) {
    if (threads > 0) return threads;
    const unsigned hw = std::thread::hardware_concurrency();
    return hw ? (int)std::min(hw, 64u) : 1;
}

template <typename F>
void parallel_for(int threads, uint64_t count, F &&fn) {
    std::atomic<uint64_t> next{0};
    std::vector<std::thread> pool;
    const int T = (int)std::min<uint64_t>((uint64_t)threads, std::max<uint64_t>(count, 1));
    for (int t = 0; t < T; ++t)
        pool.emplace_back([&, t] {
            for (;;) {
                const uint64_t i = next.fetch_add(1);
                if (i >= count) break;
                fn(t, i);
            }
        });
    for (auto &th : pool) th.join();
}

// Stable partition of hashes (and key ids) by part.
void partition(const Geometry &g, const uint64_t *h, const uint64_t *h2, uint64_t n, bool keep_ids, int threads,
               Partitioned &out) {
    const uint64_t chunk = 1 << 20;
    const uint64_t nchunks = (n + chunk - 1) / chunk;
    std::vector<uint64_t> counts(nchunks * g.P, 0);
    parallel_for(threads, nchunks, [&](int, uint64_t c) {
        uint64_t *cnt = counts.data() + c * g.P;
        for (uint64_t i = c * chunk, e = std::min(n, i + chunk); i < e; ++i) cnt[g.part(h[i])]++;
    });
    out.start.assign(g.P + 1, 0);
    // offsets: part-major, chunk-minor keeps the input order inside a part
    uint64_t run = 0;
    for (uint64_t p = 0; p < g.P; ++p) {
        out.start[p] = run;
        for (uint64_t c = 0; c < nchunks; ++c) {
            const uint64_t v = counts[c * g.P + p];
            counts[c * g.P + p] = run;
            run += v;
        }
    }
    out.start[g.P] = run;
    out.hashes.resize(n);
    if (keep_ids) out.ids.resize(n);
    if (h2) out.slot_hashes.resize(n);
    parallel_for(threads, nchunks, [&](int, uint64_t c) {
        uint64_t *pos = counts.data() + c * g.P;
        for (uint64_t i = c * chunk, e = std::min(n, i + chunk); i < e; ++i) {
            const uint64_t d = pos[g.part(h[i])]++;
            out.hashes[d] = h[i];
            if (keep_ids) out.ids[d] = i;
            if (h2) out.slot_hashes[d] = h2[i];
        }
    });
}

// Remap (Section 3.4): F[q_i - n] = L_i for the taken slots q_i >= n and
// the free slots L_i < n, in increasing order; other entries repeat their
// predecessor (0 before the first).
int build_remap(const Geometry &g, const std::vector<uint64_t> &taken, std::vector<uint64_t> &F) {
    const uint64_t total = g.P * g.S, len = total - g.n;
    F.assign(len, 0);
    auto bit = [&](uint64_t q) { return (taken[q >> 6] >> (q & 63)) & 1u; };
    uint64_t free_pos = 0;  // next candidate free slot < n
    auto next_free = [&]() -> uint64_t {
        while (free_pos < g.n) {
            const uint64_t w = ~taken[free_pos >> 6] >> (free_pos & 63);
            if (w) {
                const uint64_t q = free_pos + (uint64_t)__builtin_ctzll(w);
                if (q >= g.n) { free_pos = g.n; break; }
                free_pos = q + 1;
                return q;
            }
            free_pos = (free_pos | 63) + 1;
        }
        return UINT64_MAX;
    };
    uint64_t prev = 0;
    for (uint64_t t = 0; t < len; ++t) {
        if (bit(g.n + t)) {
            const uint64_t L = next_free();
            if (L == UINT64_MAX) return ptrhash::set_error(PTRHASH_E_BUILD, "remap: fewer free slots than overflow");
            prev = L;
        }
        F[t] = prev;
    }
    if (next_free() != UINT64_MAX) return ptrhash::set_error(PTRHASH_E_BUILD, "remap: unmatched free slot");
    return PTRHASH_OK;
}

// CacheLineEF lines: offset v0>>8 (32 bits), 128-bit map with bit
// i + (v_i>>8) - (v_0>>8) set, 44 low bytes (Section 3.4, eq. clef).
int encode_clef(const std::vector<uint64_t> &F, uint8_t *out) {
    const uint64_t lines = (F.size() + 43) / 44;
    std::memset(out, 0, lines * 64);
    for (uint64_t c = 0; c < lines; ++c) {
        const uint64_t first = c * 44, cnt = std::min<uint64_t>(44, F.size() - first);
        const uint64_t off = F[first] >> 8;
        if (off > 0xffffffffull) return ptrhash::set_error(PTRHASH_E_REMAP_RANGE, "remap value beyond 40 bits");
        uint64_t bits[2] = {0, 0};
        uint8_t *line = out + c * 64;
        for (uint64_t i = 0; i < cnt; ++i) {
            const uint64_t b = i + (F[first + i] >> 8) - off;
            if (b > 127)
                return ptrhash::set_error(PTRHASH_E_REMAP_RANGE, "CacheLineEF line %llu spans too far",
                                          (unsigned long long)c);
            bits[b >> 6] |= 1ull << (b & 63);
            line[20 + i] = (uint8_t)F[first + i];
        }
        const uint32_t off32 = (uint32_t)off;
        std::memcpy(line, &off32, 4);  // little endian host
        std::memcpy(line + 4, &bits[0], 8);
        std::memcpy(line + 12, &bits[1], 8);
    }
    return PTRHASH_OK;
}

struct KeySource {
    const uint64_t *keys = nullptr;   // u64 keys, or
    const uint8_t *data = nullptr;    // byte keys, or
    const uint64_t *offsets = nullptr;
    std::vector<uint64_t> *sorted = nullptr;  // hashes C*k of u64 keys, sorted ascending (consumed)
};

// Part boundaries of hashes sorted ascending: part p starts at the first hash
// h with hi(P*h) >= p, i.e. h >= ceil(p*2^64/P).
void sorted_part_starts(const Geometry &g, const std::vector<uint64_t> &h, std::vector<uint64_t> &start) {
    start.assign(g.P + 1, 0);
    for (uint64_t p = 1; p < g.P; ++p) {
        const uint64_t first = (uint64_t)((((u128)p << 64) + g.P - 1) / g.P);
        start[p] = (uint64_t)(std::lower_bound(h.begin(), h.end(), first) - h.begin());
    }
    start[g.P] = h.size();
}

// Parameter checks shared by every construction path (params->n is already
// known to equal the key count).
int check_geometry(const ptrhash_params *params) {
    using ptrhash::set_error;
    if (params->num_parts == 0 || params->num_parts > 0xffffffffull || params->buckets_per_part == 0 ||
        params->log2_slots > 31 || params->gamma > PTRHASH_GAMMA_LINEAR || params->remap_kind > PTRHASH_REMAP_NONE ||
        params->reduce_kind > PTRHASH_REDUCE_MOD ||
        (params->hash_bits != 0 && params->hash_bits != 64 && params->hash_bits != 128) ||
        (params->hash_bits == 128 && params->key_kind != PTRHASH_KEY_BYTES))
        return set_error(PTRHASH_E_INVAL, "invalid params");
    const bool mod = params->reduce_kind == PTRHASH_REDUCE_MOD;
    if (mod && (params->num_parts != 1 || params->slots < 2 || params->slots >= (1ull << 31) ||
                (params->slots & (params->slots - 1)) == 0))
        return set_error(PTRHASH_E_INVAL, "mod reduce: one part, 2 <= S < 2^31, S not a power of two");
    const uint64_t S = mod ? params->slots : 1ull << params->log2_slots;
    if (params->num_parts * S < params->n || params->remap_len != params->num_parts * S - params->n)
        return set_error(PTRHASH_E_INVAL, "P*S/remap_len");
    if (params->buckets_per_part >= (1ull << 31)) return set_error(PTRHASH_E_RANGE, "too many buckets per part");
    return PTRHASH_OK;
}

// F from the taken-slot bitvector, then its encoding into remap.
int write_remap(const Geometry &g, const ptrhash_params *params, const std::vector<uint64_t> &taken, void *remap) {
    std::vector<uint64_t> F;
    int rc = build_remap(g, taken, F);
    if (rc) return rc;
    if (params->remap_kind == PTRHASH_REMAP_CLEF) return encode_clef(F, static_cast<uint8_t *>(remap));
    if (params->remap_kind == PTRHASH_REMAP_U32) {
        uint32_t *r = static_cast<uint32_t *>(remap);
        for (uint64_t i = 0; i < F.size(); ++i) r[i] = (uint32_t)F[i];
    }
    return PTRHASH_OK;
}

int build_impl(const KeySource &src, uint64_t n, ptrhash_params *params, uint8_t *pilots, void *remap,
               int threads, ptrhash_build_info *info) {
    using ptrhash::set_error;
    if (!params || !pilots) return set_error(PTRHASH_E_INVAL, "params/pilots is NULL");
    if (params->n != n || n == 0) return set_error(PTRHASH_E_INVAL, "params->n must equal n > 0");
    const bool bytes = src.data != nullptr;
    if (src.sorted && bytes) return set_error(PTRHASH_E_INVAL, "sorted hashes are for u64 keys");
    if (params->key_kind != (bytes ? PTRHASH_KEY_BYTES : PTRHASH_KEY_U64))
        return set_error(PTRHASH_E_INVAL, "params->key_kind does not match the keys");
    if (int rc = check_geometry(params)) return rc;
    const bool mod = params->reduce_kind == PTRHASH_REDUCE_MOD;
    Geometry g{n, params->num_parts, mod ? params->slots : 1ull << params->log2_slots, params->buckets_per_part,
               params->seed, params->log2_slots, params->gamma, mod};
    const uint64_t rbytes = ptrhash_remap_bytes(params);
    if (rbytes && !remap) return set_error(PTRHASH_E_INVAL, "remap is NULL");
    threads = pick_threads(threads);

    const bool wide = bytes && params->hash_bits == 128;
    std::vector<uint64_t> h(src.sorted ? 0 : n), h2(wide ? n : 0);
    Partitioned part;
    ptrhash_build_info local{};
    const bool timing = std::getenv("PTRHASH_BUILD_TIMING") != nullptr;
    auto tick = std::chrono::steady_clock::now();
    auto phase = [&](const char *name) {
        if (!timing) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[build] %-10s %8.3f s\n", name, std::chrono::duration<double>(now - tick).count());
        tick = now;
    };
    int rc = PTRHASH_E_BUILD;
    for (int attempt = 0; attempt < kMaxSeeds; ++attempt) {
        local.attempts = attempt + 1;
        g.seed = params->seed + attempt;
        if (src.sorted && attempt == 0) {
            if (src.sorted->size() != n) return set_error(PTRHASH_E_INVAL, "sorted hash count != n");
            part.hashes = std::move(*src.sorted);
            part.sorted = true;
            sorted_part_starts(g, part.hashes, part.start);
            for (uint64_t i = 1; i < n; ++i)
                if (part.hashes[i] == part.hashes[i - 1]) return set_error(PTRHASH_E_DUPLICATE, "two equal keys");
            phase("partstarts");
        } else if (!src.sorted && (bytes || attempt == 0)) {
            const uint64_t chunk = 1 << 16;
            parallel_for(threads, (n + chunk - 1) / chunk, [&](int, uint64_t c) {
                for (uint64_t i = c * chunk, e = std::min(n, i + chunk); i < e; ++i) {
                    if (!bytes) {
                        h[i] = kMix * src.keys[i];
                        continue;
                    }
                    const uint8_t *sp = src.data + src.offsets[i];
                    const uint64_t len = src.offsets[i + 1] - src.offsets[i];
                    h[i] = hash_bytes(g.seed, sp, len);
                    if (wide) h2[i] = hash_bytes(g.seed ^ kWideSalt, sp, len);
                }
            });
            phase("hash");
            partition(g, h.data(), wide ? h2.data() : nullptr, n, bytes, threads, part);
            phase("partition");
        }
        bool overflow = false;
        for (uint64_t p = 0; p < g.P; ++p) overflow |= part.start[p + 1] - part.start[p] > g.S;
        if (overflow && !bytes) return set_error(PTRHASH_E_BUILD, "a part holds more than S keys");

        // equal hashes inside a bucket (found while placing): 1 = distinct keys
        // (byte keys: reseed), 2 = duplicate keys (error)
        std::atomic<int> equal{0};
        if (overflow) continue;  // byte keys: reseed

        std::vector<uint64_t> taken((g.P * g.S + 63) / 64, 0);
        std::atomic<bool> failed{false};
        std::vector<PartWorker> workers(threads);
        std::vector<uint64_t> part_ev(g.P, 0), part_max(g.P, 0);
        parallel_for(threads, g.P, [&](int t, uint64_t p) {
            if (failed.load(std::memory_order_relaxed)) return;
            PartWorker &w = workers[t];
            if (w.geo == nullptr) w.init(&g);
            const uint64_t s0 = part.start[p], cnt = part.start[p + 1] - s0;
            if (part.sorted)
                w.group_sorted(part.hashes.data() + s0, cnt);
            else
                w.group(part.hashes.data() + s0, wide ? part.slot_hashes.data() + s0 : nullptr, cnt);
            if (w.has_equal_hashes()) {
                int kind = 2;
                if (bytes) {  // distinct strings with one hash only need a new seed
                    kind = 1;
                    struct E {
                        uint64_t h, h2, id;
                        bool operator<(const E &o) const { return h != o.h ? h < o.h : h2 != o.h2 ? h2 < o.h2 : id < o.id; }
                    };
                    std::vector<E> v(cnt);
                    for (uint64_t i = 0; i < cnt; ++i)
                        v[i] = {part.hashes[s0 + i], wide ? part.slot_hashes[s0 + i] : 0, part.ids[s0 + i]};
                    std::sort(v.begin(), v.end());
                    for (uint64_t i = 1; i < cnt && kind == 1; ++i) {
                        if (v[i].h != v[i - 1].h || v[i].h2 != v[i - 1].h2) continue;
                        const uint64_t a = v[i].id, c = v[i - 1].id;
                        const uint64_t la = src.offsets[a + 1] - src.offsets[a];
                        const uint64_t lc = src.offsets[c + 1] - src.offsets[c];
                        if (la == lc && std::memcmp(src.data + src.offsets[a], src.data + src.offsets[c], la) == 0)
                            kind = 2;
                    }
                }
                int prev = equal.load();
                while (prev < kind && !equal.compare_exchange_weak(prev, kind)) {
                }
                failed.store(true);
                return;
            }
            w.max_bucket = 0;
            if (w.place(pilots + p * g.B, (uint64_t)kEvictionFactor * g.S) != kPartOk) {
                failed.store(true);
                return;
            }
            part_ev[p] = w.evictions;
            part_max[p] = w.max_bucket;
            // taken slots of this part (parts may share a bitmap word when S < 64)
            for (uint64_t s = 0; s < g.S; ++s)
                if (w.owner[s] != kEmpty) {
                    const uint64_t q = p * g.S + s;
                    __atomic_fetch_or(&taken[q >> 6], 1ull << (q & 63), __ATOMIC_RELAXED);
                }
        });
        phase("place");
        if (equal.load() == 2) return set_error(PTRHASH_E_DUPLICATE, "two equal keys");
        if (failed.load()) continue;
        local.evictions = 0;
        local.max_part_evictions = 0;
        local.max_bucket_size = 0;
        for (uint64_t p = 0; p < g.P; ++p) {
            local.evictions += part_ev[p];
            local.max_part_evictions = std::max(local.max_part_evictions, part_ev[p]);
            local.max_bucket_size = std::max(local.max_bucket_size, part_max[p]);
        }
        rc = write_remap(g, params, taken, remap);
        if (rc) return rc;
        phase("remap");
        params->seed = g.seed;
        if (info) *info = local;
        return PTRHASH_OK;
    }
    if (info) *info = local;
    return set_error(PTRHASH_E_BUILD, "construction failed for %d seeds", kMaxSeeds);
}

}  // namespace

namespace ptrhash {
int check_build_params(uint64_t n, const ptrhash_params *params, uint32_t key_kind) {
    if (!params) return set_error(PTRHASH_E_INVAL, "params is NULL");
    if (params->n != n || n == 0) return set_error(PTRHASH_E_INVAL, "params->n must equal n > 0");
    if (params->key_kind != key_kind) return set_error(PTRHASH_E_INVAL, "params->key_kind does not match the keys");
    return check_geometry(params);
}

int build_from_sorted(std::vector<uint64_t> &&sorted, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                      void *remap, int threads, ptrhash_build_info *info) {
    KeySource src;
    src.sorted = &sorted;
    try {
        return build_impl(src, n, params, pilots, remap, threads, info);
    } catch (const std::bad_alloc &) {
        return set_error(PTRHASH_E_NOMEM, "host allocation failed during construction");
    }
}
}  // namespace ptrhash

extern "C" {

PTRHASH_API int ptrhash_build_u64(const uint64_t *keys, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                                  void *remap, int threads, ptrhash_build_info *info) {
    if (!keys) return ptrhash::set_error(PTRHASH_E_INVAL, "keys is NULL");
    KeySource src;
    src.keys = keys;
    try {
        return build_impl(src, n, params, pilots, remap, threads, info);
    } catch (const std::bad_alloc &) {
        return ptrhash::set_error(PTRHASH_E_NOMEM, "host allocation failed during construction");
    }
}

PTRHASH_API int ptrhash_build_bytes(const uint8_t *data, uint64_t data_len, const uint64_t *offsets, uint64_t n,
                                    ptrhash_params *params, uint8_t *pilots, void *remap, int threads,
                                    ptrhash_build_info *info) {
    if (!data || !offsets) return ptrhash::set_error(PTRHASH_E_INVAL, "data/offsets is NULL");
    for (uint64_t i = 0; i < n; ++i)
        if (offsets[i + 1] < offsets[i])
            return ptrhash::set_error(PTRHASH_E_INVAL, "offsets decrease at key %llu", (unsigned long long)i);
    if (offsets[n] > data_len)
        return ptrhash::set_error(PTRHASH_E_INVAL, "the strings end at %llu, past data_len %llu",
                                  (unsigned long long)offsets[n], (unsigned long long)data_len);
    KeySource src;
    src.data = data;
    src.offsets = offsets;
    try {
        return build_impl(src, n, params, pilots, remap, threads, info);
    } catch (const std::bad_alloc &) {
        return ptrhash::set_error(PTRHASH_E_NOMEM, "host allocation failed during construction");
    }
}

}  // extern "C"
