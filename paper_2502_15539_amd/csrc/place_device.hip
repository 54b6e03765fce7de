// Pilot search on the device (Section 3.2 "Construction"; the hash-evict
// search of Section 3.2 "Hash-evict", the 10*S eviction limit of Section 4).
//
// Parts are independent, so each part is searched by one workgroup that owns
// the part's taken-slot bitvector in LDS (S bits; 128 KiB at S = 2^20): one
// wavefront places the buckets, the others look ahead for it (look_ahead
// below). The rules are exactly those of the host builder, so the device
// reaches the same pilots: buckets in order of (size descending, bucket id
// ascending); the
// smallest pilot in [0, 256) whose slots are free and pairwise distinct;
// otherwise, among pilots with distinct slots that touch none of the 16 most
// recently placed buckets, the one with the least sum over colliding keys of
// (size of the owning bucket)^2, smallest pilot first on ties; its owners are
// evicted and requeued. Requeued buckets wait in a small max-heap in LDS;
// merging it with the pre-sorted bucket order pops buckets in the same order
// as one priority queue holding both.
//
// Inputs come from device passes over the sorted hashes (the part and the
// bucket of a key are non-decreasing in its hash): bucket start offsets, the
// per-part (size desc, id asc) order from a radix sort, and a copy of the
// hashes laid out in that order so the search streams them.
#include <hipcub/hipcub.hpp>

#include "internal.h"
#include "place_device.h"

namespace ptrhash {
namespace {

constexpr int kWave = 64;
constexpr int kRecent = 16;
constexpr uint32_t kHeapCap = 1024;       // requeued buckets waiting at once
constexpr uint32_t kMaxBucket = 2048;     // largest bucket searched (its slots fit the per-wave scratch)
constexpr uint32_t kShuffleDistinct = 1;  // buckets up to this size set their bits without the tentative step
constexpr int kMaxHelpers = 7;            // look-ahead wavefronts beside the leading one, at most
constexpr int kMaxBlock = kWave * (1 + kMaxHelpers);
constexpr uint32_t kRing = 42;            // look-ahead results held at once, entry e in ring[e % kRing];
                                          // a multiple of every helper count allowed (1, 2, 3, 6, 7), so
                                          // that each ring entry has a single writer
constexpr uint32_t kNoPilot = 256;        // no pilot in [0, 256) has free, pairwise distinct slots
constexpr uint64_t kTagBusy = ~0ull;      // a look-ahead result being written

// Slot record written when a bucket is placed: owner bucket (local id), its
// placement number, its size and its pilot.
struct SlotRec {
    uint32_t owner, last, size, pilot;
};

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, kWave);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t bcast64(uint64_t v, int lane) {  // lane is wave-uniform
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// v from another lane of its row of 16 by a DPP move (ctrl: the lane
// pattern); a lane whose source is inactive keeps its own v.
template <int Ctrl>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)v, (int)(uint32_t)v, Ctrl, 0xf, 0xf, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(v >> 32), (int)(uint32_t)(v >> 32), Ctrl, 0xf, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

// The least v of the wavefront (every lane active), in every lane: within
// each row of 16 lanes by DPP moves (lanes of a quad swapped in pairs, then
// in halves; then each half-row and each row mirrored), then the four rows'
// minima read into scalars. No LDS traffic.
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
    uint64_t o = dpp64<0xB1>(v);  // quad_perm 1,0,3,2
    v = o < v ? o : v;
    o = dpp64<0x4E>(v);           // quad_perm 2,3,0,1
    v = o < v ? o : v;
    o = dpp64<0x141>(v);          // row_half_mirror
    v = o < v ? o : v;
    o = dpp64<0x140>(v);          // row_mirror
    v = o < v ? o : v;
    uint64_t m = bcast64(v, 0);
    for (int r = 16; r < kWave; r += 16) {
        const uint64_t x = bcast64(v, r);
        m = x < m ? x : m;
    }
    return m;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
    for (int d = 32; d >= 1; d >>= 1) v += shfl64(v, __lane_id() ^ d);
    return v;
}

// Slot within the part: reduce(h xor hp, S), the reduce fixed at compile time.
template <bool Mod>
__device__ __forceinline__ uint32_t local_slot(const DevMphf &m, uint64_t h, uint64_t hp) {
    if (Mod) return (uint32_t)mod_reduce(h ^ hp, m.mod_slots, m.mod_magic);
    return (uint32_t)(mulhi64(kMix, h ^ hp) & ((1ull << m.log2_slots) - 1));
}

__device__ __forceinline__ uint64_t pilot_hash(const DevMphf &m, uint32_t p) { return kMix * ((uint64_t)p ^ m.seed); }

__device__ __forceinline__ bool is_taken(const uint32_t *bits, uint32_t q) { return (bits[q >> 5] >> (q & 31)) & 1u; }

// bst[g] = index of the first sorted hash whose global bucket is >= g, for
// g in [0, P*B]; flags[0] = 1 if two hashes are equal.
__global__ void bucket_starts_k(const uint64_t *__restrict__ H, uint64_t n, DevMphf m, uint64_t *__restrict__ bst,
                                uint32_t *__restrict__ flags) {
    const uint64_t total = (uint64_t)m.parts * m.buckets;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t part;
        const uint64_t g = bucket_of(m, H[i], part);
        uint64_t first = 0;
        if (i > 0) {
            const uint64_t hp = H[i - 1];
            if (hp == H[i]) flags[0] = 1u;
            first = bucket_of(m, hp, part) + 1;
        }
        for (uint64_t b = first; b <= g; ++b) bst[b] = i;
        if (i == n - 1)
            for (uint64_t b = g + 1; b <= total; ++b) bst[b] = n;
    }
}

// Largest bucket and largest part.
__global__ void size_max_k(const uint64_t *__restrict__ bst, DevMphf m, unsigned long long *__restrict__ out) {
    const uint64_t total = (uint64_t)m.parts * m.buckets;
    uint64_t mb = 0, mp = 0;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = bst[g + 1] - bst[g];
        mb = s > mb ? s : mb;
        if (g % m.buckets == 0) {
            const uint64_t ps = bst[g + m.buckets] - bst[g];
            mp = ps > mp ? ps : mp;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t ob = shfl64(mb, __lane_id() ^ d), op = shfl64(mp, __lane_id() ^ d);
        mb = ob > mb ? ob : mb;
        mp = op > mp ? op : mp;
    }
    if (__lane_id() == 0) {
        atomicMax(&out[0], (unsigned long long)mb);
        atomicMax(&out[1], (unsigned long long)mp);
    }
}

// Sort key of bucket g: part, then size descending, then local id.
__global__ void order_keys_k(const uint64_t *__restrict__ bst, DevMphf m, uint64_t max_size, uint32_t size_bits,
                             uint32_t id_bits, uint64_t *__restrict__ keys) {
    const uint64_t total = (uint64_t)m.parts * m.buckets;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t part = g / m.buckets, id = g - part * m.buckets;
        const uint64_t s = bst[g + 1] - bst[g];
        keys[g] = (part << (size_bits + id_bits)) | ((max_size - s) << id_bits) | id;
    }
}

__device__ __forceinline__ void decode_key(uint64_t key, uint64_t max_size, uint32_t size_bits, uint32_t id_bits,
                                           uint32_t &size, uint32_t &id) {
    id = (uint32_t)(key & ((1ull << id_bits) - 1));
    size = (uint32_t)(max_size - ((key >> id_bits) & ((1ull << size_bits) - 1)));
}

__global__ void ordered_sizes_k(const uint64_t *__restrict__ keys, uint64_t total, uint64_t max_size,
                                uint32_t size_bits, uint32_t id_bits, uint64_t *__restrict__ sizes) {
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t s, id;
        decode_key(keys[k], max_size, size_bits, id_bits, s, id);
        sizes[k] = s;
    }
}

// OH[ostart[k] + t] = hashes of the k-th bucket in search order.
__global__ void scatter_ordered_k(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ ostart,
                                  const uint64_t *__restrict__ bst, const uint64_t *__restrict__ H, DevMphf m,
                                  uint64_t max_size, uint32_t size_bits, uint32_t id_bits, uint64_t *__restrict__ OH) {
    const uint64_t total = (uint64_t)m.parts * m.buckets;
    const uint32_t part_shift = size_bits + id_bits;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[k];
        uint32_t s, id;
        decode_key(key, max_size, size_bits, id_bits, s, id);
        const uint64_t g = (key >> part_shift) * m.buckets + id;
        const uint64_t src = bst[g], dst = ostart[k];
        for (uint32_t t = 0; t < s; ++t) OH[dst + t] = H[src + t];
    }
}

struct PlaceArgs {
    DevMphf m;                  // geometry and seed
    const uint64_t *H;          // n sorted hashes
    const uint64_t *bst;        // P*B + 1 bucket starts into H
    const uint64_t *okeys;      // P*B sorted order keys
    const uint64_t *OH;         // hashes in search order (same part ranges as H)
    uint64_t n;
    uint64_t max_size;
    uint32_t size_bits, id_bits;
    uint64_t max_evictions;
    uint8_t *pilots;            // P*B, zeroed
    uint32_t *taken;            // P*S bits, zeroed
    SlotRec *recs;              // grid * S scratch
    uint32_t *big;              // grid * kMaxBucket scratch (slots of a large bucket)
    uint32_t *next_part;        // work counter, zeroed
    uint32_t *status;           // per part
    uint64_t *evictions;        // per part
    uint32_t *cancel;           // set by the host when this seed's result is no longer needed
    const uint64_t *ostart;     // P*B: offset in OH of each order entry's hashes
    uint32_t helpers;           // look-ahead wavefronts per workgroup (blockDim.x / 64 - 1)
};

// The cancel flag, in coherent pinned host memory that the host sets while
// the search runs; read at system scope so that the host's store is seen.
// Wave-uniform.
__device__ __forceinline__ bool cancel_requested(uint32_t *flag) {
    const uint32_t v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return __builtin_amdgcn_readfirstlane((int)v) != 0;
}

// Pairwise distinctness of up to 64 slots, key j in lane j (j < s). Up to
// eight keys, key j's slot is read into a scalar and compared by the lanes
// after j (no LDS traffic); beyond, lane a compares with lane a+d mod 64
// for d = 1..32, which covers every pair.
__device__ __forceinline__ bool distinct_lanes(uint32_t q, uint32_t s) {
    const int lane = __lane_id();
    bool dup = false;
    if (s <= 8) {
        for (uint32_t j = 0; j + 1 < s; ++j) {
            const uint32_t qj = (uint32_t)__builtin_amdgcn_readlane((int)q, (int)j);
            dup |= (uint32_t)lane > j && (uint32_t)lane < s && q == qj;
        }
        return __ballot(dup) == 0;
    }
    for (int d = 1; d <= kWave / 2; ++d) {
        if ((uint32_t)d >= s) break;
        const int src = (lane + d) & (kWave - 1);
        const uint32_t o = (uint32_t)__shfl((int)q, src, kWave);
        dup |= (uint32_t)lane < s && (uint32_t)src < s && o == q;
    }
    return __ballot(dup) == 0;
}

// What a look-ahead wavefront found for one order entry (a bucket of at most
// 64 keys): the bucket, the smallest pilot whose slots were free and
// pairwise distinct in the bitvector it read (or kNoPilot), and that
// pilot's slots. Written before the tag; once the leader has read its entry's
// tag with the current generation the entry no longer changes (its one writer
// moves on to later entries, and only the leader changes the generation).
struct LookAhead {
    uint64_t tag;            // (generation << 32) | entry; kTagBusy while written
    uint32_t pilot;
    uint32_t size, id;       // the bucket (size, local id) of the entry
    uint32_t pad;
    uint32_t slots[kWave];   // key j's slot in slots[j]
};

// The generation counts the leader's changes to the bitvector that clear
// bits (evictions, undone tentative placements, a new part): it is odd
// while one is under way. Between two changes bits are only added.
struct LdsState {
    uint64_t heap[kHeapCap];  // max-heap of (size << 32) | ~id; its size lives in a register
    LookAhead ring[kRing];
    uint64_t gb0;             // first order entry of the part being searched
    uint32_t gen;             // generation (written by the leader only)
    uint32_t front;           // order entries of the part the leader has taken
    uint32_t nb;              // order entries of the part
    uint32_t done;            // the leader has finished
};

// LDS words shared by the wavefronts of the workgroup, each read or written
// by one instruction. lds_fence orders this wavefront's LDS accesses before
// it against those after it (it waits for LDS operations only, not for
// global stores).
__device__ __forceinline__ uint32_t lds_ld(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t lds_ld(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }
// Keeps the compiler from moving memory accesses across it; no wait. A
// wavefront's LDS operations are carried out in the order they are issued,
// so a read issued after another also observes the LDS after it.
__device__ __forceinline__ void compiler_fence() { __asm__ __volatile__("" ::: "memory"); }
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint64_t uniform(uint64_t v) {
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// The leader's generation steps: open before it clears bits, close after.
__device__ __forceinline__ void open_gen(LdsState &st, uint32_t &gen) {
    gen |= 1u;
    if (__lane_id() == 0) lds_st(&st.gen, gen);
    lds_fence();
}
__device__ __forceinline__ void close_gen(LdsState &st, uint32_t &gen) {
    lds_fence();
    gen += 1u;
    if (__lane_id() == 0) lds_st(&st.gen, gen);
}

// Heap operations run in every lane on the same values (LDS reads
// broadcast); lane 0 writes. hn is the heap's size (wave-uniform).
__device__ void heap_push(LdsState &st, uint32_t &hn, uint64_t v) {
    uint32_t i = hn;
    while (i > 0) {
        const uint32_t p = (i - 1) >> 1;
        const uint64_t pv = st.heap[p];
        if (pv >= v) break;
        if (__lane_id() == 0) st.heap[i] = pv;
        __builtin_amdgcn_wave_barrier();
        i = p;
    }
    if (__lane_id() == 0) st.heap[i] = v;
    ++hn;
    __builtin_amdgcn_wave_barrier();
}

__device__ uint64_t heap_pop(LdsState &st, uint32_t &hn) {
    const uint64_t top = st.heap[0];
    const uint32_t n = hn - 1;
    const uint64_t v = st.heap[n];
    uint32_t i = 0;
    for (;;) {
        const uint32_t c = 2 * i + 1;
        if (c >= n) break;
        uint32_t best = c;
        if (c + 1 < n && st.heap[c + 1] > st.heap[c]) best = c + 1;
        const uint64_t cv = st.heap[best];
        if (cv <= v) break;
        if (__lane_id() == 0) st.heap[i] = cv;
        __builtin_amdgcn_wave_barrier();
        i = best;
    }
    if (__lane_id() == 0 && n) st.heap[i] = v;
    hn = n;
    __builtin_amdgcn_wave_barrier();
    return top;
}

// Wait for every vector memory operation of this wavefront (s_waitcnt with
// vmcnt = 0, expcnt and lgkmcnt left at their maxima). Placed where a load's
// result must be complete on that path only, so that the compiler's own wait
// is not put on the paths that merge after it.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// A window of a read-only u64 stream held one entry per lane in two
// registers (entries [start, start + 128)). It is refilled synchronously:
// a prefetched register would be read by the loop's phi copies on every
// iteration, and the wait for it would also wait for every store in flight.
struct Window {
    const uint64_t *base;
    uint64_t len, start;
    uint64_t w0, w1;

    __device__ void fill(uint64_t at) {
        start = at;
        const uint64_t i = at + (uint64_t)__lane_id();
        w0 = i < len ? base[i] : 0;
        w1 = i + kWave < len ? base[i + kWave] : 0;
        wait_vm();
    }
    // entries [at, at + 64) available: at - start <= 64
    __device__ void need(uint64_t at) {
        if (at > start + kWave) fill(at);
    }
    // entry at (wave-uniform), at - start < 128
    __device__ uint64_t get(uint64_t at) const {
        const uint32_t o = (uint32_t)(at - start);
        return o < (uint32_t)kWave ? bcast64(w0, (int)o) : bcast64(w1, (int)(o - kWave));
    }
    // entry at + lane for lane < 64, at - start <= 64
    __device__ uint64_t lanes(uint64_t at) const {
        const uint32_t o = (uint32_t)(at - start) + (uint32_t)__lane_id();
        const uint64_t x0 = shfl64(w0, (int)(o & 63)), x1 = shfl64(w1, (int)(o & 63));
        return o < (uint32_t)kWave ? x0 : x1;
    }
};

// Pilots p in [64 round, 64 round + 64) with p >= start, pilot p in lane
// p % 64 of the result: none of the bucket's s keys (key j's hash in lane j
// of h) lands on a taken slot with p. Four independent LDS reads per step.
template <bool Mod>
__device__ __forceinline__ uint64_t free_pilots(const DevMphf &m, const uint32_t *bits, uint64_t h, uint32_t s,
                                                int round, uint32_t start) {
    const uint32_t pl = (uint32_t)(round * kWave + __lane_id());
    const uint64_t hp = pilot_hash(m, pl);
    bool free = pl >= start;
    for (uint32_t j = 0; j < s; j += 4) {
        bool t = is_taken(bits, local_slot<Mod>(m, bcast64(h, (int)j), hp));
        if (j + 1 < s) t |= is_taken(bits, local_slot<Mod>(m, bcast64(h, (int)j + 1), hp));
        if (j + 2 < s) t |= is_taken(bits, local_slot<Mod>(m, bcast64(h, (int)j + 2), hp));
        if (j + 3 < s) t |= is_taken(bits, local_slot<Mod>(m, bcast64(h, (int)j + 3), hp));
        free = free && !t;
        if (__ballot(free) == 0) break;
    }
    return __ballot(free);
}

// A look-ahead wavefront (hid of nh). While the leader places buckets one by
// one, it takes the part's order entries e = hid, hid + nh, ... that lie
// less than kRing ahead of the leader and, for each bucket of at most 64
// keys, records in ring[e % kRing] the smallest pilot whose slots are free
// and pairwise distinct in the bitvector as it reads it, tagged with the
// generation it read under. Within a generation bits are only added, so the
// pilots below the recorded one stay blocked; the leader, finding its entry
// tagged with the current generation, only re-checks the recorded slots. The
// leader never waits for a look-ahead wavefront; these leave once it is done.
// The order keys and hash offsets of its next 64 entries are loaded at once
// (lane j: entry eb + j nh), and the hashes of the next bucket are loaded
// while the current one is searched.
template <bool Mod>
__device__ __forceinline__ void look_ahead(const PlaceArgs &a, const uint32_t *bits, LdsState &st, uint32_t hid,
                                           uint32_t nh) {
    const DevMphf &m = a.m;
    const int lane = __lane_id();
    uint32_t hgen = 1u, e = hid;
    uint64_t bgb = ~0ull, bk = 0, bo = 0;  // batch: part, order key and hash offset of entry eb + lane nh
    uint32_t eb = 0;
    uint64_t pgb = ~0ull, ph = 0;          // prefetched hashes of entry pe of part pgb
    uint32_t pe = 0;
    for (;;) {
        if (uniform(lds_ld(&st.done))) break;
        // generation, part and leader position, then the generation again,
        // read in this order (LDS carries them out in issue order)
        const uint32_t g1r = lds_ld(&st.gen);
        compiler_fence();
        const uint64_t gb0r = lds_ld(&st.gb0);
        const uint32_t nbr = lds_ld(&st.nb), frontr = lds_ld(&st.front);
        compiler_fence();
        const uint32_t g2 = uniform(lds_ld(&st.gen));
        const uint32_t g1 = uniform(g1r), nb = uniform(nbr), front = uniform(frontr);
        const uint64_t gb0 = uniform(gb0r);
        if ((g1 & 1u) || g1 != g2) {
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        if (g1 != hgen) {  // a new generation: earlier results no longer count
            hgen = g1;
            e = hid;
        }
        if (e < front) e += (front - e + nh - 1) / nh * nh;
        if (e >= nb || e >= front + kRing) {
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        if (bgb != gb0 || e < eb || e - eb >= (uint32_t)kWave * nh) {
            const uint64_t ej = (uint64_t)e + (uint64_t)lane * nh;
            bk = ej < nb ? a.okeys[gb0 + ej] : 0;
            bo = ej < nb ? a.ostart[gb0 + ej] : 0;
            bgb = gb0;
            eb = e;
        }
        uint32_t s, id;
        const int j = (int)((e - eb) / nh);
        decode_key(bcast64(bk, j), a.max_size, a.size_bits, a.id_bits, s, id);
        if (s == 0) {  // sizes only fall along the order: the rest are empty
            e = nb;
            continue;
        }
        if (s > (uint32_t)kWave) {
            e += nh;
            continue;
        }
        uint64_t h = ph;
        if (pgb != gb0 || pe != e) {
            const uint64_t c = bcast64(bo, j);
            h = (uint32_t)lane < s ? a.OH[c + lane] : 0;
        }
        // h complete before the next load is issued, so that the search below
        // does not wait for that load too (vmcnt cannot tell the two apart)
        wait_vm();
        // the next entry's hashes, in flight during this search
        pgb = ~0ull;
        if (j + 1 < kWave && e + nh < nb) {
            uint32_t sn, idn;
            decode_key(bcast64(bk, j + 1), a.max_size, a.size_bits, a.id_bits, sn, idn);
            if (sn > 0 && sn <= (uint32_t)kWave) {
                const uint64_t cn = bcast64(bo, j + 1);
                ph = (uint32_t)lane < sn ? a.OH[cn + lane] : 0;
                pgb = gb0;
                pe = e + nh;
            }
        }
        uint32_t pilot = kNoPilot, q = 0;
        for (int round = 0; round < 4 && pilot == kNoPilot; ++round) {
            uint64_t cand = free_pilots<Mod>(m, bits, h, s, round, 0);
            while (cand) {
                const int lbit = __builtin_ctzll(cand);
                cand &= cand - 1;
                const uint32_t pc = (uint32_t)(round * kWave + lbit);
                const uint32_t qc = (uint32_t)lane < s ? local_slot<Mod>(m, h, pilot_hash(m, pc)) : 0u;
                if (distinct_lanes(qc, s)) {
                    pilot = pc;
                    q = qc;
                    break;
                }
            }
        }
        // the entry marked busy, its contents, then its tag, written in this
        // order (LDS carries them out in issue order)
        LookAhead &r = st.ring[e % kRing];
        if (lane == 0) lds_st(&r.tag, kTagBusy);
        compiler_fence();
        if ((uint32_t)lane < s) r.slots[lane] = q;
        if (lane == 0) {
            r.pilot = pilot;
            r.size = s;
            r.id = id;
        }
        compiler_fence();
        if (lane == 0) lds_st(&r.tag, ((uint64_t)g1 << 32) | e);
        e += nh;
    }
}

// The eviction cost step for keys j .. j+N-1 of a small bucket (key j's hash
// in lane j of h0) under the pilots lane, 64 + lane, 128 + lane and
// 192 + lane: for each taken slot, the owner's size squared is added to
// cost[round], and ok[round] is cleared if the owner is among the recently
// placed buckets. The 4 N slot records are loaded unconditionally (a slot is
// below S; the record of a free slot is not used) and the 4 N taken bits read
// together, so that the loads of the group are in flight at once.
template <bool Mod, int N>
__device__ __forceinline__ void cost_group(const DevMphf &m, const uint32_t *bits, const SlotRec *recs, uint64_t h0,
                                           uint32_t j, uint64_t placed, uint64_t (&cost)[4], bool (&ok)[4]) {
    const int lane = __lane_id();
    uint32_t q[4][N];
    SlotRec rec[4][N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint64_t hj = bcast64(h0, (int)j + i);
#pragma unroll
        for (int round = 0; round < 4; ++round)
            q[round][i] = local_slot<Mod>(m, hj, pilot_hash(m, (uint32_t)(round * kWave + lane)));
    }
#pragma unroll
    for (int round = 0; round < 4; ++round)
#pragma unroll
        for (int i = 0; i < N; ++i) rec[round][i] = recs[q[round][i]];
    uint32_t tk = 0;  // bit N round + i: the slot of key j + i under the round's pilot is taken
#pragma unroll
    for (int round = 0; round < 4; ++round)
#pragma unroll
        for (int i = 0; i < N; ++i) tk |= (uint32_t)is_taken(bits, q[round][i]) << (N * round + i);
    __asm__ __volatile__("" : "+v"(tk));  // every read issued before any is used
#pragma unroll
    for (int round = 0; round < 4; ++round)
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (ok[round] && ((tk >> (N * round + i)) & 1u)) {
                if ((uint64_t)rec[round][i].last + kRecent > placed) ok[round] = false;
                cost[round] += (uint64_t)rec[round][i].size * rec[round][i].size;
            }
}

// One workgroup per part at a time, a persistent grid taking parts from a
// counter: wavefront 0 places the buckets, the others look ahead for it.
// Mod: the single-part x mod S reduce instead of the power-of-two one.
template <bool Mod>
__global__ void __launch_bounds__(kMaxBlock) place_k(PlaceArgs a) {
    extern __shared__ uint32_t bits[];  // S bits of the current part
    __shared__ LdsState st;
    for (uint32_t i = threadIdx.x; i < kRing; i += blockDim.x) st.ring[i].tag = kTagBusy;
    if (threadIdx.x == 0) {
        st.gb0 = 0;
        st.gen = 1u;
        st.front = 0u;
        st.nb = 0u;
        st.done = 0u;
    }
    __syncthreads();
    if (threadIdx.x >= (uint32_t)kWave) {
        look_ahead<Mod>(a, bits, st, threadIdx.x / kWave - 1, a.helpers);
        return;
    }
    const DevMphf &m = a.m;
    const int lane = __lane_id();
    uint32_t gen = 1u;  // the generation (odd: no part yet)
    const uint32_t S = m.reduce_kind == kReduceMod ? m.mod_slots : (1u << m.log2_slots);
    const uint32_t words = (S + 31) / 32;
    const uint32_t B = m.buckets;
    SlotRec *recs = a.recs + (uint64_t)blockIdx.x * S;
    uint32_t *big = a.big + (uint64_t)blockIdx.x * kMaxBucket;

    for (;;) {
        if (cancel_requested(a.cancel)) break;
        uint32_t p = 0;
        if (lane == 0) p = atomicAdd(a.next_part, 1u);
        p = (uint32_t)__builtin_amdgcn_readfirstlane((int)p);
        if (p >= m.parts) break;

        const uint64_t gb0 = (uint64_t)p * B;
        open_gen(st, gen);
        if (lane == 0) {
            lds_st(&st.gb0, gb0);
            lds_st(&st.nb, B);
            lds_st(&st.front, 0u);
        }
        for (uint32_t w = lane; w < words; w += kWave) bits[w] = 0u;
        uint32_t hn = 0;  // requeued buckets in the heap
        close_gen(st, gen);
        uint64_t k = gb0;                    // next entry of the search order
        const uint64_t kend = gb0 + B;
        uint64_t c = a.bst[gb0];             // its first hash in OH
        Window ow{a.okeys, kend, 0, 0, 0};
        ow.fill(k);
        Window hw{a.OH, a.n, 0, 0, 0};  // hashes in search order
        hw.fill(c);
        uint64_t placed = 0, ev = 0;
        uint32_t status = kPlaceOk;
        const uint64_t max_iter = (uint64_t)B + a.max_evictions + 2;

        for (uint64_t iter = 0;; ++iter) {
            if (iter > max_iter) { status = kPlaceFailed; break; }
            if ((iter & 8191u) == 8191u && cancel_requested(a.cancel)) { status = kPlaceCancelled; break; }
            // next bucket: the larger of the order's head and the heap's top
            uint32_t s = 0, id = 0;
            bool from_order = false;
            bool have = false;       // the look-ahead result for entry k, read under the current generation
            uint32_t rp = 0, rq = 0; // its pilot and key `lane`'s slot
            if (k < kend) {
                const uint32_t e = (uint32_t)(k - gb0);
                LookAhead &r = st.ring[e % kRing];
                if (uniform(lds_ld(&r.tag)) == (((uint64_t)gen << 32) | e)) {
                    lds_fence();
                    s = uniform(r.size);
                    id = uniform(r.id);
                    rp = uniform(r.pilot);
                    rq = (uint32_t)lane < s ? r.slots[lane] : 0u;
                    have = true;
                } else {
                    ow.need(k);
                    decode_key(ow.get(k), a.max_size, a.size_bits, a.id_bits, s, id);
                }
                from_order = s > 0;
            }
            if (hn > 0) {
                const uint64_t head = from_order ? (((uint64_t)s << 32) | (0xffffffffu - id)) : 0;
                if (st.heap[0] > head) {
                    const uint64_t v = heap_pop(st, hn);
                    s = (uint32_t)(v >> 32);
                    id = 0xffffffffu - (uint32_t)v;
                    from_order = false;
                }
            } else if (!from_order) {
                break;  // every bucket placed
            }
            const bool small = s <= kWave;
            const uint64_t *src;
            uint64_t h0 = 0;     // key `lane` of a small bucket
            int chosen = -1;
            uint32_t myq = 0;    // key `lane`'s slot with the chosen pilot (small buckets)
            uint32_t start = 0;  // the pilots below it are known to be blocked
            if (from_order) {
                src = a.OH + c;
                if (small) {
                    if (have) {
                        start = rp;
                        if (rp < kNoPilot) {
                            if (__ballot((uint32_t)lane < s && is_taken(bits, rq)) == 0) {
                                // still free, and distinct (checked by the look-ahead)
                                if ((uint32_t)lane < s) atomicOr(&bits[rq >> 5], 1u << (rq & 31));
                                chosen = (int)rp;
                                myq = rq;
                            } else {
                                start = rp + 1;
                            }
                        }
                    }
                    if (chosen < 0) {
                        hw.need(c);
                        h0 = hw.lanes(c);
                    }
                }
                c += s;
                ++k;
                if (lane == 0) lds_st(&st.front, (uint32_t)(k - gb0));
            } else {
                src = a.H + a.bst[gb0 + id];
                if (small && (uint32_t)lane < s) h0 = src[lane];
                wait_vm();
            }
            if (!small && s > kMaxBucket) { status = kPlaceTooLarge; break; }

            // 1) smallest pilot with free, distinct slots
            if (small) {
                for (int round = (int)(start >> 6); round < 4 && chosen < 0; ++round) {
                    uint64_t cand = free_pilots<Mod>(m, bits, h0, s, round, start);
                    while (cand) {
                        const int lbit = __builtin_ctzll(cand);
                        cand &= cand - 1;
                        const uint32_t pc = (uint32_t)(round * kWave + lbit);
                        if (s <= kShuffleDistinct) {
                            // the slots are free: distinct among the bucket's own
                            // keys (lane shuffles) is all that is left to check
                            myq = (uint32_t)lane < s ? local_slot<Mod>(m, h0, pilot_hash(m, pc)) : 0u;
                            if (!distinct_lanes(myq, s)) continue;
                            if ((uint32_t)lane < s) atomicOr(&bits[myq >> 5], 1u << (myq & 31));
                            chosen = (int)pc;
                            break;
                        }
                        // larger buckets: set the bits tentatively; a key that finds
                        // its bit already set collides with a sibling (all were free)
                        bool mine = false, dup = false;
                        if ((uint32_t)lane < s) {
                            myq = local_slot<Mod>(m, h0, pilot_hash(m, pc));
                            const uint32_t old = atomicOr(&bits[myq >> 5], 1u << (myq & 31));
                            if (old & (1u << (myq & 31))) dup = true; else mine = true;
                        }
                        if (__ballot(dup) == 0) { chosen = (int)pc; break; }
                        open_gen(st, gen);  // bits are cleared
                        if (mine) atomicAnd(&bits[myq >> 5], ~(1u << (myq & 31)));
                        close_gen(st, gen);
                    }
                }
                if (chosen >= 0) {
                    // placed without evictions: one record store per key, no waits
                    ++placed;
                    const SlotRec rec{id, (uint32_t)placed, s, (uint32_t)chosen};
                    if ((uint32_t)lane < s) recs[myq] = rec;
                    if (lane == 0) a.pilots[gb0 + id] = (uint8_t)chosen;
                    // The entries that follow, as long as each is a look-ahead result
                    // of the current generation whose slots are still free and no
                    // requeued bucket waits: the same steps as above, in a loop of
                    // their own. Only stores are in flight at its back edge, so the
                    // compiler puts no wait for memory operations in it (at the
                    // general loop's head it may, for loads of the slower paths, and
                    // vmcnt counts the record stores too). The next entry is read
                    // while this one's slots are checked. Anything else goes back to
                    // the general loop, which takes the same entry again.
                    if (have && hn == 0 && k < kend) {
                        uint32_t e = (uint32_t)(k - gb0), ri = e % kRing;
                        uint64_t t2 = lds_ld(&st.ring[ri].tag);
                        compiler_fence();
                        uint32_t s2 = st.ring[ri].size, id2 = st.ring[ri].id, p2 = st.ring[ri].pilot;
                        uint32_t q2 = st.ring[ri].slots[lane];
                        while (((iter + 1) & 8191u) != 8191u && iter + 1 <= max_iter) {
                            if (uniform(t2) != (((uint64_t)gen << 32) | e)) break;
                            s2 = uniform(s2);
                            id2 = uniform(id2);
                            p2 = uniform(p2);
                            if (p2 >= kNoPilot) break;
                            // the bitvector words of this entry's slots (every lane reads:
                            // no branch around the read, so the reads of the next entry,
                            // its tag first, are issued before it is waited for)
                            const uint32_t qa = (uint32_t)lane < s2 ? q2 : 0u;
                            uint32_t w = bits[qa >> 5];
                            const uint32_t r1 = ri + 1 == kRing ? 0u : ri + 1;
                            compiler_fence();
                            const uint64_t t3 = lds_ld(&st.ring[r1].tag);
                            compiler_fence();
                            const uint32_t s3 = st.ring[r1].size, id3 = st.ring[r1].id, p3 = st.ring[r1].pilot;
                            const uint32_t q3 = st.ring[r1].slots[lane];
                            compiler_fence();
                            __asm__ __volatile__("" : "+v"(w));  // w is used only from here on
                            if (__ballot((uint32_t)lane < s2 && ((w >> (qa & 31)) & 1u))) break;
                            if ((uint32_t)lane < s2) atomicOr(&bits[q2 >> 5], 1u << (q2 & 31));
                            ++iter;
                            ++placed;
                            const SlotRec rec2{id2, (uint32_t)placed, s2, p2};
                            if ((uint32_t)lane < s2) recs[q2] = rec2;
                            if (lane == 0) a.pilots[gb0 + id2] = (uint8_t)p2;
                            c += s2;
                            ++k;
                            if (lane == 0) lds_st(&st.front, (uint32_t)(k - gb0));
                            if (k >= kend) break;
                            e += 1;
                            ri = r1;
                            t2 = t3;
                            s2 = s3;
                            id2 = id3;
                            p2 = p3;
                            q2 = q3;
                        }
                    }
                    continue;
                }
            } else {
                for (uint32_t pc = 0; pc < 256 && chosen < 0; ++pc) {
                    const uint64_t hpc = pilot_hash(m, pc);
                    bool any_taken = false;
                    for (uint32_t t = lane; t < s; t += kWave) any_taken |= is_taken(bits, local_slot<Mod>(m, src[t], hpc));
                    if (__ballot(any_taken)) continue;
                    bool dup = false;
                    uint32_t mine = 0;
                    for (uint32_t t = lane, r = 0; t < s; t += kWave, ++r) {
                        const uint32_t qq = local_slot<Mod>(m, src[t], hpc);
                        const uint32_t old = atomicOr(&bits[qq >> 5], 1u << (qq & 31));
                        if (old & (1u << (qq & 31))) dup = true; else mine |= 1u << r;
                    }
                    if (__ballot(dup) == 0) { chosen = (int)pc; break; }
                    open_gen(st, gen);  // bits are cleared
                    for (uint32_t t = lane, r = 0; t < s; t += kWave, ++r)
                        if (mine & (1u << r)) {
                            const uint32_t qq = local_slot<Mod>(m, src[t], hpc);
                            atomicAnd(&bits[qq >> 5], ~(1u << (qq & 31)));
                        }
                    close_gen(st, gen);
                }
            }

            if (chosen < 0) {
                // 2) least weighted collisions, never touching the recent ones.
                // The slot records read below were written by earlier
                // placements of this wavefront: wait for those stores.
                __threadfence_block();
                if (small) {
                    // Per lane, pilots lane, 64 + lane, 128 + lane and 192 + lane: the
                    // sum over the keys on taken slots of the owner's size squared,
                    // unless a slot belongs to a recently placed bucket; up to four keys
                    // at a time (cost_group).
                    uint64_t keyr[4], cost[4] = {0, 0, 0, 0};
                    bool ok[4] = {true, true, true, true};
                    for (uint32_t j = 0; j < s; j += 4) {
                        const uint32_t left = s - j;
                        if (left >= 4)
                            cost_group<Mod, 4>(m, bits, recs, h0, j, placed, cost, ok);
                        else if (left == 3)
                            cost_group<Mod, 3>(m, bits, recs, h0, j, placed, cost, ok);
                        else if (left == 2)
                            cost_group<Mod, 2>(m, bits, recs, h0, j, placed, cost, ok);
                        else
                            cost_group<Mod, 1>(m, bits, recs, h0, j, placed, cost, ok);
                    }
#pragma unroll
                    for (int round = 0; round < 4; ++round)
                        keyr[round] = ok[round] ? ((cost[round] << 8) | (uint32_t)(round * kWave + lane)) : ~0ull;
                    // the least (cost, pilot) whose slots are distinct
                    for (int tries = 0; tries < 256; ++tries) {
                        uint64_t mn = keyr[0];
                        for (int r = 1; r < 4; ++r) mn = keyr[r] < mn ? keyr[r] : mn;
                        mn = wave_min64(mn);
                        if (mn == ~0ull) break;
                        const uint32_t pc = (uint32_t)(mn & 255);
                        const uint32_t qq = (uint32_t)lane < s ? local_slot<Mod>(m, h0, pilot_hash(m, pc)) : 0u;
                        if (distinct_lanes(qq, s)) { chosen = (int)pc; break; }
                        if ((uint32_t)lane == (pc & 63)) keyr[pc >> 6] = ~0ull;
                    }
                } else {
                    uint64_t best = ~0ull;
                    for (uint32_t pc = 0; pc < 256; ++pc) {
                        const uint64_t hpc = pilot_hash(m, pc);
                        uint64_t cost = 0;
                        bool ok = true;
                        for (uint32_t t = lane; t < s; t += kWave) {
                            const uint32_t qq = local_slot<Mod>(m, src[t], hpc);
                            if (is_taken(bits, qq)) {
                                const SlotRec rec = recs[qq];
                                if ((uint64_t)rec.last + kRecent > placed) ok = false;
                                cost += (uint64_t)rec.size * rec.size;
                            }
                        }
                        if (__ballot(!ok)) continue;
                        cost = wave_sum64(cost);
                        if (cost >= best) continue;
                        // distinct: write the slots to scratch, compare all pairs
                        for (uint32_t t = lane; t < s; t += kWave) big[t] = local_slot<Mod>(m, src[t], hpc);
                        __threadfence_block();
                        bool dup = false;
                        for (uint32_t t = lane; t < s && !dup; t += kWave) {
                            const uint32_t qt = big[t];
                            for (uint32_t u = t + 1; u < s; ++u)
                                if (big[u] == qt) { dup = true; break; }
                        }
                        if (__ballot(dup) == 0) {
                            best = cost;
                            chosen = (int)pc;
                        }
                    }
                }
                if (chosen < 0) { status = kPlaceFailed; break; }
                // evict every owner the chosen slots hit, key by key
                open_gen(st, gen);  // bits are cleared
                const uint64_t hpc = pilot_hash(m, (uint32_t)chosen);
                for (uint32_t j = 0; j < s; ++j) {
                    const uint64_t hj = small ? bcast64(h0, (int)j) : src[j];
                    const uint32_t qq = local_slot<Mod>(m, hj, hpc);
                    if (!is_taken(bits, qq)) continue;
                    const SlotRec rec = recs[qq];
                    if (rec.owner >= B || rec.size == 0 || rec.size > kMaxBucket || rec.pilot > 255) {
                        status = kPlaceCorrupt;  // never expected: a record that no placement wrote
                        break;
                    }
                    const uint64_t *oh = a.H + a.bst[gb0 + rec.owner];
                    const uint64_t hpo = pilot_hash(m, rec.pilot);
                    for (uint32_t t = lane; t < rec.size; t += kWave) {
                        const uint32_t qo = local_slot<Mod>(m, oh[t], hpo);
                        atomicAnd(&bits[qo >> 5], ~(1u << (qo & 31)));
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (hn >= kHeapCap) { status = kPlaceHeapFull; break; }
                    heap_push(st, hn, ((uint64_t)rec.size << 32) | (0xffffffffu - rec.owner));
                    ++ev;
                }
                if (status != kPlaceOk) break;
                // the bucket's bits (phase 1 set them already)
                for (uint32_t t = lane; t < s; t += kWave) {
                    const uint32_t qq = local_slot<Mod>(m, small ? h0 : src[t], hpc);
                    atomicOr(&bits[qq >> 5], 1u << (qq & 31));
                }
                close_gen(st, gen);
            }

            // slot records and pilot of the placed bucket
            ++placed;
            const uint64_t hpc = pilot_hash(m, (uint32_t)chosen);
            const SlotRec rec{id, (uint32_t)placed, s, (uint32_t)chosen};
            for (uint32_t t = lane; t < s; t += kWave) recs[local_slot<Mod>(m, small ? h0 : src[t], hpc)] = rec;
            if (lane == 0) a.pilots[gb0 + id] = (uint8_t)chosen;
            if (ev > a.max_evictions) { status = kPlaceFailed; break; }
        }

        // the part's taken slots into the global bitvector (P*S bits; parts
        // start on a word boundary: S is a multiple of 32 or there is one part)
        __builtin_amdgcn_wave_barrier();
        if (status == kPlaceOk) {
            const uint64_t wbase = (uint64_t)p * S / 32;
            for (uint32_t w = lane; w < words; w += kWave) {
                uint32_t v = bits[w];
                if (w == words - 1 && (S & 31)) v &= (1u << (S & 31)) - 1;
                a.taken[wbase + w] = v;
            }
        }
        if (lane == 0) {
            a.status[p] = status;
            a.evictions[p] = ev;
        }
    }
    if (lane == 0) lds_st(&st.done, 1u);
}

}  // namespace
}  // namespace ptrhash

// ---------------------------------------------------------------------------
// Host side: buffers, passes, reseeding.

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "builder.h"
#include "errors.h"

namespace {

using ptrhash::set_error;

__global__ void hash_keys_gpu_k(const uint64_t *__restrict__ keys, uint64_t n, uint64_t *__restrict__ out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = ptrhash::hash_u64(keys[i]);
}

struct DevBufs {
    std::vector<void *> p;
    ~DevBufs() {
        for (void *x : p)
            if (x) (void)hipFree(x);
    }
    template <typename T>
    hipError_t get(T **out, uint64_t count) {
        void *x = nullptr;
        const hipError_t e = hipMalloc(&x, count ? count * sizeof(T) : 1);
        if (e == hipSuccess) p.push_back(x);
        *out = static_cast<T *>(x);
        return e;
    }
};

uint32_t bit_width(uint64_t v) { return v ? 64u - (uint32_t)__builtin_clzll(v) : 0u; }

#define HIP_OR_FAIL(expr, what)                                                                      \
    do {                                                                                             \
        const hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                        \
            return set_error(e_ == hipErrorOutOfMemory ? PTRHASH_E_NOMEM : PTRHASH_E_HIP, "%s: %s", \
                             what, hipGetErrorString(e_));                                           \
    } while (0)

constexpr int kMaxSeeds = 16;
constexpr uint64_t kEvictionFactor = 10;
constexpr uint32_t kMaxPairs = 64;  // equal-hash pairs of string keys examined per attempt

// String keys: h[i] = the byte-string hash of key i under seed, ids[i] = i.
__global__ void hash_strings_gpu_k(const uint8_t *__restrict__ data, const uint64_t *__restrict__ offsets, uint64_t n,
                                   uint64_t seed, uint64_t *__restrict__ h, uint64_t *__restrict__ ids) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t o0 = offsets[i], o1 = offsets[i + 1];
        uint64_t unused;
        h[i] = ptrhash::hash_bytes(seed, data, o0, o1 - o0, false, unused);
        ids[i] = i;
    }
}

// 128-bit string hashes: hi (part and bucket) and lo (slot) of key i under
// seed, ids[i] = i.
__global__ void hash_strings128_gpu_k(const uint8_t *__restrict__ data, const uint64_t *__restrict__ offsets,
                                      uint64_t n, uint64_t seed, uint64_t *__restrict__ hi, uint64_t *__restrict__ lo,
                                      uint64_t *__restrict__ ids) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t o0 = offsets[i], o1 = offsets[i + 1];
        hi[i] = ptrhash::hash_bytes(seed, data, o0, o1 - o0, true, lo[i]);
        ids[i] = i;
    }
}

// flag[0] = 1 if some key's offsets decrease or its end passes end_limit.
__global__ void check_offsets_k(const uint64_t *__restrict__ offsets, uint64_t n, uint64_t end_limit,
                                uint32_t *__restrict__ flag) {
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t o0 = offsets[i], o1 = offsets[i + 1];
        bad |= o1 < o0 || o1 > end_limit;
    }
    if (bad) atomicOr(flag, 1u);
}

// out[i] = src[idx[i]]
__global__ void gather_k(const uint64_t *__restrict__ src, const uint64_t *__restrict__ idx, uint64_t n,
                         uint64_t *__restrict__ out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = src[idx[i]];
}

// 128-bit hashes sorted by the high half: adjacent keys whose two halves
// are both equal (count, and the first kMaxPairs as ids), and whether three
// keys in a row share the high half (then not every equal pair is adjacent).
__global__ void equal_pairs128_k(const uint64_t *__restrict__ hi, const uint64_t *__restrict__ lo,
                                 const uint64_t *__restrict__ ids, uint64_t n, uint32_t *__restrict__ count,
                                 uint64_t *__restrict__ pairs) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (hi[i] != hi[i - 1]) continue;
        if (i >= 2 && hi[i - 2] == hi[i]) atomicOr(&count[1], 1u);
        if (lo[i] == lo[i - 1]) {
            const uint32_t k = atomicAdd(&count[0], 1u);
            if (k < kMaxPairs) {
                pairs[2 * k] = ids[i - 1];
                pairs[2 * k + 1] = ids[i];
            }
        }
    }
}

// Pairs of keys with equal hashes (adjacent after the sort): count them and
// keep the first kMaxPairs (ids) for the host to compare.
__global__ void equal_pairs_k(const uint64_t *__restrict__ H, const uint64_t *__restrict__ ids, uint64_t n,
                              uint32_t *__restrict__ count, uint64_t *__restrict__ pairs) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        if (H[i] == H[i - 1]) {
            const uint32_t k = atomicAdd(count, 1u);
            if (k < kMaxPairs) {
                pairs[2 * k] = ids[i - 1];
                pairs[2 * k + 1] = ids[i];
            }
        }
}

// ---------------------------------------------------------------------------
// The remap table (Section 3.4) from the taken-slot bitvector (slot q is bit
// q & 63 of u64 word q >> 6): F[q - n] for the slots q in [n, P*S) is, where
// q is taken, the next free slot below n, both taken in increasing order;
// elsewhere it repeats its predecessor (0 before the first). Then F is
// encoded into CacheLineEF lines (or written as u32). The same table as the
// host builder's, byte for byte.

// Bits of the word whose first slot is base that lie below slot lim.
__device__ __forceinline__ uint64_t bits_below(uint64_t base, uint64_t lim) {
    if (lim <= base) return 0;
    return lim - base >= 64 ? ~0ull : (1ull << (lim - base)) - 1;
}

// Per word: free slots below n, taken slots in [n, total).
__global__ void remap_counts_k(const uint64_t *__restrict__ taken, uint64_t words, uint64_t n, uint64_t total,
                               uint64_t *__restrict__ cfree, uint64_t *__restrict__ ctaken) {
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = w * 64, v = taken[w], below = bits_below(base, n);
        cfree[w] = (uint64_t)__popcll(~v & below);
        ctaken[w] = (uint64_t)__popcll(v & bits_below(base, total) & ~below);
    }
}

// The free slots below n in increasing order (ofree: exclusive prefix sums of cfree).
__global__ void remap_free_list_k(const uint64_t *__restrict__ taken, uint64_t words, uint64_t n,
                                  const uint64_t *__restrict__ ofree, uint64_t *__restrict__ fl) {
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = w * 64;
        uint64_t f = ~taken[w] & bits_below(base, n), o = ofree[w];
        while (f) {
            fl[o++] = base + (uint64_t)__builtin_ctzll(f);
            f &= f - 1;
        }
    }
}

// F[t], t < len: the free slot matched with the last taken slot in
// [n, n + t], or 0 if there is none (otaken: exclusive prefix sums of ctaken).
__global__ void remap_values_k(const uint64_t *__restrict__ taken, uint64_t n, uint64_t len,
                               const uint64_t *__restrict__ otaken, const uint64_t *__restrict__ fl,
                               uint64_t *__restrict__ F) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t q = n + t, w = q >> 6, b = q & 63, base = w * 64;
        const uint64_t upto = b == 63 ? ~0ull : (2ull << b) - 1;
        const uint64_t r = otaken[w] + (uint64_t)__popcll(taken[w] & ~bits_below(base, n) & upto);
        F[t] = r ? fl[r - 1] : 0;
    }
}

// One CacheLineEF line per thread: the offset F[first] >> 8 (32 bits), a
// 128-bit map with bit i + (F[first + i] >> 8) - offset set for each of
// the line's values, and their low bytes (eq. clef). err: 1 = an offset
// beyond 32 bits, 2 = a line whose values span too far.
__global__ void remap_clef_k(const uint64_t *__restrict__ F, uint64_t len, uint32_t *__restrict__ out,
                             uint32_t *__restrict__ err) {
    const uint64_t lines = (len + 43) / 44;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < lines; c += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t first = c * 44, cnt = len - first < 44 ? len - first : 44;
        const uint64_t off = F[first] >> 8;
        uint32_t e = off > 0xffffffffull ? 1u : 0u;
        uint64_t m0 = 0, m1 = 0;
        uint32_t low[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (uint64_t i = 0; i < cnt; ++i) {
            const uint64_t v = F[first + i], b = i + (v >> 8) - off;
            if (b > 127) {
                e |= 2u;
                continue;
            }
            if (b < 64) m0 |= 1ull << b; else m1 |= 1ull << (b - 64);
            low[i >> 2] |= (uint32_t)(v & 255) << (8 * (i & 3));
        }
        uint32_t *line = out + c * 16;
        line[0] = (uint32_t)off;
        line[1] = (uint32_t)m0;
        line[2] = (uint32_t)(m0 >> 32);
        line[3] = (uint32_t)m1;
        line[4] = (uint32_t)(m1 >> 32);
        for (int i = 0; i < 11; ++i) line[5 + i] = low[i];
        if (e) atomicOr(err, e);
    }
}

__global__ void remap_u32_k(const uint64_t *__restrict__ F, uint64_t len, uint32_t *__restrict__ out) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (uint64_t)gridDim.x * blockDim.x)
        out[t] = (uint32_t)F[t];
}

// The buffers of one seed's search. Slot 0 runs on the caller's stream; the
// others, used when seeds run side by side, on streams of their own.
struct Attempt {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t done = nullptr;
    uint8_t *pil = nullptr;
    uint32_t *taken = nullptr, *big = nullptr, *next = nullptr, *status = nullptr;
    uint32_t *cancel = nullptr;    // coherent pinned host memory: set by the host, read by the search
    ptrhash::SlotRec *recs = nullptr;
    uint64_t *ev = nullptr;
    uint32_t *status_h = nullptr;  // pinned host copies, filled by the search's stream
    uint64_t *ev_h = nullptr;
    uint64_t seed = 0;
    bool busy = false;
    std::chrono::steady_clock::time_point started{};
};

constexpr int kSpecSlots = 4;  // seeds searched side by side at most

// Device pilot search over one set of sorted 64-bit hashes: bucket starts,
// the (size desc, id asc) order, the hashes in that order, then one search
// kernel per seed. A seed whose search runs far longer than a normal one
// (a part caught in an eviction cycle) has the following seeds started on
// the CUs its finished parts left idle; the result is still the first seed
// that succeeds, and later seeds still running then are cancelled.
class GpuSearch {
  public:
    GpuSearch(const ptrhash_params *params, uint64_t n, hipStream_t stream) : n_(n), stream_(stream) {
        using namespace ptrhash;
        mod_ = params->reduce_kind == PTRHASH_REDUCE_MOD;
        S_ = mod_ ? params->slots : 1ull << params->log2_slots;
        P_ = params->num_parts;
        B_ = params->buckets_per_part;
        total_ = P_ * B_;
        m_.n = n;
        m_.parts = (uint32_t)P_;
        m_.buckets = (uint32_t)B_;
        m_.log2_slots = mod_ ? 0 : params->log2_slots;
        m_.gamma = params->gamma;
        m_.reduce_kind = params->reduce_kind;
        m_.mod_slots = mod_ ? (uint32_t)S_ : 0;
        m_.mod_magic = mod_ ? ~0ull / S_ : 0;  // floor((2^64 - 1) / S) = floor(2^64 / S): S is not a power of two
        timing_ = std::getenv("PTRHASH_BUILD_TIMING") != nullptr;
        // look-ahead wavefronts per part (0, 1, 2, 3, 6 or 7)
        if (const char *la = std::getenv("PTRHASH_SEARCH_HELPERS")) {
            const int h = std::atoi(la);
            if (h == 0 || (h > 0 && h <= ptrhash::kMaxHelpers && ptrhash::kRing % h == 0)) helpers_ = (uint32_t)h;
        }
        tick_ = std::chrono::steady_clock::now();
    }

    void phase(const char *name) {
        if (!timing_) return;
        (void)hipStreamSynchronize(stream_);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[build] %-10s %8.3f s\n", name, std::chrono::duration<double>(now - tick_).count());
        tick_ = now;
    }

    // Threads per search workgroup: the leading wavefront and its helpers.
    int block() const { return ptrhash::kWave * (1 + (int)helpers_); }

    // Limits of the device search and the buffers that do not depend on the
    // hash set.
    int init() {
        using namespace ptrhash;
        words_ = (S_ + 31) / 32;
        if (P_ > 1 && S_ % 32) return set_error(PTRHASH_E_RANGE, "device placement: S must be a multiple of 32");
        int dev = 0, cus = 0, lds_max = 0;
        HIP_OR_FAIL(hipGetDevice(&dev), "device query");
        HIP_OR_FAIL(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device query");
        HIP_OR_FAIL(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "device query");
        lds_ = words_ * sizeof(uint32_t);
        if (lds_ + sizeof(LdsState) > (size_t)lds_max)
            return set_error(PTRHASH_E_RANGE, "device placement: %llu slots per part exceed the LDS of one CU",
                             (unsigned long long)S_);
        const void *kern = mod_ ? reinterpret_cast<const void *>(&place_k<true>)
                                : reinterpret_cast<const void *>(&place_k<false>);
        (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_);
        int per_cu = 0;
        if (mod_)
            HIP_OR_FAIL(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, place_k<true>, block(), lds_),
                        "occupancy query");
        else
            HIP_OR_FAIL(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, place_k<false>, block(), lds_),
                        "occupancy query");
        if (per_cu < 1) return set_error(PTRHASH_E_RANGE, "device placement does not fit one CU");
        grid_ = std::min<uint64_t>(P_, (uint64_t)cus * (uint64_t)per_cu);
        taken_words_ = (P_ * S_ + 63) / 64 * 2;  // u32 words, whole u64 words
        HIP_OR_FAIL(buf_.get(&bst_, total_ + 1), "bucket starts");
        HIP_OR_FAIL(buf_.get(&maxes_, 2), "device scalars");
        HIP_OR_FAIL(buf_.get(&flags_, 1), "device scalars");
        HIP_OR_FAIL(buf_.get(&ka_, total_), "order keys");
        HIP_OR_FAIL(buf_.get(&kb_, total_), "order keys");
        HIP_OR_FAIL(buf_.get(&ostart_, total_), "order offsets");
        att_.resize(kSpecSlots);
        return alloc_attempt(att_[0], false);
    }

    ~GpuSearch() {
        for (Attempt &t : att_) {
            if (t.busy && t.done) (void)hipEventSynchronize(t.done);
            if (t.done) (void)hipEventDestroy(t.done);
            if (t.own_stream && t.stream) (void)hipStreamDestroy(t.stream);
            if (t.status_h) (void)hipHostFree(t.status_h);
            if (t.ev_h) (void)hipHostFree(t.ev_h);
            if (t.cancel) (void)hipHostFree(t.cancel);
        }
        if (prepared_) (void)hipEventDestroy(prepared_);
    }

    // Device bytes of one seed's search buffers.
    uint64_t attempt_bytes() const {
        return total_ + taken_words_ * 4 + grid_ * S_ * sizeof(ptrhash::SlotRec) + grid_ * (uint64_t)ptrhash::kMaxBucket * 4 +
               P_ * 12 + 64;
    }

    // Buffers (and, for a side-by-side seed, a stream that first waits for
    // the prepared order) of one search slot.
    int alloc_attempt(Attempt &t, bool own_stream) {
        using namespace ptrhash;
        HIP_OR_FAIL(buf_.get(&t.pil, total_), "pilots");
        HIP_OR_FAIL(buf_.get(&t.taken, taken_words_), "taken bits");
        HIP_OR_FAIL(buf_.get(&t.recs, grid_ * S_), "slot records");
        HIP_OR_FAIL(buf_.get(&t.big, grid_ * (uint64_t)kMaxBucket), "bucket scratch");
        HIP_OR_FAIL(buf_.get(&t.next, 1), "work counter");
        HIP_OR_FAIL(buf_.get(&t.status, P_), "part status");
        HIP_OR_FAIL(buf_.get(&t.ev, P_), "part evictions");
        HIP_OR_FAIL(hipHostMalloc(&t.status_h, P_ * sizeof(uint32_t), hipHostMallocDefault), "pinned status");
        HIP_OR_FAIL(hipHostMalloc(&t.ev_h, P_ * sizeof(uint64_t), hipHostMallocDefault), "pinned evictions");
        HIP_OR_FAIL(hipHostMalloc(&t.cancel, sizeof(uint32_t), hipHostMallocCoherent), "cancel flag");
        __atomic_store_n(t.cancel, 0u, __ATOMIC_SEQ_CST);
        HIP_OR_FAIL(hipEventCreateWithFlags(&t.done, hipEventDisableTiming), "event");
        if (own_stream) {
            HIP_OR_FAIL(hipStreamCreateWithFlags(&t.stream, hipStreamNonBlocking), "stream");
            t.own_stream = true;
            HIP_OR_FAIL(hipStreamWaitEvent(t.stream, prepared_, 0), "stream wait");
        } else {
            t.stream = stream_;
        }
        return PTRHASH_OK;
    }

    // Radix-sort n keys (with values if vals) in place through a second
    // buffer; returns the sorted keys (and values) via the double buffers.
    int sort(hipcub::DoubleBuffer<uint64_t> &keys, hipcub::DoubleBuffer<uint64_t> *vals) {
        size_t temp = 0;
        if (vals)
            HIP_OR_FAIL(hipcub::DeviceRadixSort::SortPairs(nullptr, temp, keys, *vals, (size_t)n_, 0, 64, stream_),
                        "sort sizing");
        else
            HIP_OR_FAIL(hipcub::DeviceRadixSort::SortKeys(nullptr, temp, keys, (size_t)n_, 0, 64, stream_),
                        "sort sizing");
        if (temp > sort_temp_bytes_) {
            HIP_OR_FAIL(buf_.get(&sort_temp_, temp), "sort scratch");
            sort_temp_bytes_ = temp;
        }
        if (vals)
            HIP_OR_FAIL(hipcub::DeviceRadixSort::SortPairs(sort_temp_, temp, keys, *vals, (size_t)n_, 0, 64, stream_),
                        "sort");
        else
            HIP_OR_FAIL(hipcub::DeviceRadixSort::SortKeys(sort_temp_, temp, keys, (size_t)n_, 0, 64, stream_), "sort");
        return PTRHASH_OK;
    }

    // Bucket starts, order and ordered hashes for the sorted hashes H (OH: n
    // entries of scratch). *dup: two equal hashes; *overflow: a part with
    // more than S keys (then nothing else is prepared).
    // Hs: the hashes the slots are computed from, in the order of H, when
    // they differ from H (128-bit string hashes: H is the high half, which
    // picks part and bucket, Hs the low half).
    int prepare(const uint64_t *H, uint64_t *OH, bool *dup, bool *overflow, const uint64_t *Hs = nullptr) {
        using namespace ptrhash;
        H_ = Hs ? Hs : H;
        OH_ = OH;
        HIP_OR_FAIL(hipMemsetAsync(flags_, 0, sizeof(uint32_t), stream_), "memset");
        HIP_OR_FAIL(hipMemsetAsync(maxes_, 0, 2 * sizeof(unsigned long long), stream_), "memset");
        hipLaunchKernelGGL(bucket_starts_k, dim3(8192), dim3(256), 0, stream_, H, n_, m_, bst_, flags_);
        HIP_OR_FAIL(hipGetLastError(), "bucket starts launch");
        hipLaunchKernelGGL(size_max_k, dim3(4096), dim3(256), 0, stream_, bst_, m_, maxes_);
        HIP_OR_FAIL(hipGetLastError(), "size launch");
        uint32_t d = 0;
        unsigned long long mx[2] = {0, 0};
        HIP_OR_FAIL(hipMemcpyAsync(&d, flags_, sizeof d, hipMemcpyDeviceToHost, stream_), "copy out");
        HIP_OR_FAIL(hipMemcpyAsync(mx, maxes_, sizeof mx, hipMemcpyDeviceToHost, stream_), "copy out");
        HIP_OR_FAIL(hipStreamSynchronize(stream_), "sync");
        *dup = d != 0;
        *overflow = mx[1] > S_;
        if (*dup || *overflow) return PTRHASH_OK;
        max_size_ = mx[0];
        if (max_size_ > kMaxBucket)
            return set_error(PTRHASH_E_RANGE, "device placement: a bucket of %llu keys (at most %u)",
                             (unsigned long long)max_size_, kMaxBucket);
        size_bits_ = bit_width(max_size_);
        id_bits_ = bit_width(B_ - 1);
        const uint32_t part_bits = bit_width(P_ - 1);
        if (size_bits_ + id_bits_ + part_bits > 64)
            return set_error(PTRHASH_E_RANGE, "device placement: sort key width");
        phase("starts");
        hipLaunchKernelGGL(order_keys_k, dim3(8192), dim3(256), 0, stream_, bst_, m_, max_size_, size_bits_, id_bits_,
                           ka_);
        HIP_OR_FAIL(hipGetLastError(), "order launch");
        hipcub::DoubleBuffer<uint64_t> kdb(ka_, kb_);
        const int end_bit = (int)(size_bits_ + id_bits_ + part_bits);
        size_t temp = 0;
        HIP_OR_FAIL(hipcub::DeviceRadixSort::SortKeys(nullptr, temp, kdb, (size_t)total_, 0, end_bit, stream_),
                    "order sort sizing");
        if (temp > sort_temp_bytes_) {
            HIP_OR_FAIL(buf_.get(&sort_temp_, temp), "order sort scratch");
            sort_temp_bytes_ = temp;
        }
        HIP_OR_FAIL(hipcub::DeviceRadixSort::SortKeys(sort_temp_, temp, kdb, (size_t)total_, 0, end_bit, stream_),
                    "order sort");
        okeys_ = kdb.Current();
        uint64_t *osize = kdb.Alternate();
        hipLaunchKernelGGL(ordered_sizes_k, dim3(8192), dim3(256), 0, stream_, okeys_, total_, max_size_, size_bits_,
                           id_bits_, osize);
        HIP_OR_FAIL(hipGetLastError(), "sizes launch");
        temp = 0;
        HIP_OR_FAIL(hipcub::DeviceScan::ExclusiveSum(nullptr, temp, osize, ostart_, (int64_t)total_, stream_),
                    "scan sizing");
        if (temp > sort_temp_bytes_) {
            HIP_OR_FAIL(buf_.get(&sort_temp_, temp), "scan scratch");
            sort_temp_bytes_ = temp;
        }
        HIP_OR_FAIL(hipcub::DeviceScan::ExclusiveSum(sort_temp_, temp, osize, ostart_, (int64_t)total_, stream_),
                    "scan");
        hipLaunchKernelGGL(scatter_ordered_k, dim3(8192), dim3(256), 0, stream_, okeys_, ostart_, bst_, H_, m_,
                           max_size_, size_bits_, id_bits_, OH);
        HIP_OR_FAIL(hipGetLastError(), "scatter launch");
        if (!prepared_) HIP_OR_FAIL(hipEventCreateWithFlags(&prepared_, hipEventDisableTiming), "event");
        HIP_OR_FAIL(hipEventRecord(prepared_, stream_), "event record");
        phase("order");
        return PTRHASH_OK;
    }

    // Start the search of one seed on a slot (asynchronous).
    int launch(Attempt &t, uint64_t seed) {
        using namespace ptrhash;
        HIP_OR_FAIL(hipMemsetAsync(t.pil, 0, total_, t.stream), "memset");
        HIP_OR_FAIL(hipMemsetAsync(t.taken, 0, taken_words_ * sizeof(uint32_t), t.stream), "memset");
        HIP_OR_FAIL(hipMemsetAsync(t.next, 0, sizeof(uint32_t), t.stream), "memset");
        __atomic_store_n(t.cancel, 0u, __ATOMIC_SEQ_CST);  // the slot's previous search has finished
        PlaceArgs a{};
        a.m = m_;
        a.m.seed = seed;
        a.H = H_;
        a.bst = bst_;
        a.okeys = okeys_;
        a.OH = OH_;
        a.n = n_;
        a.max_size = max_size_;
        a.size_bits = size_bits_;
        a.id_bits = id_bits_;
        a.max_evictions = kEvictionFactor * S_;
        a.pilots = t.pil;
        a.taken = t.taken;
        a.recs = t.recs;
        a.big = t.big;
        a.next_part = t.next;
        a.status = t.status;
        a.evictions = t.ev;
        a.cancel = t.cancel;
        a.ostart = ostart_;
        a.helpers = helpers_;
        if (mod_)
            hipLaunchKernelGGL(place_k<true>, dim3((uint32_t)grid_), dim3(block()), lds_, t.stream, a);
        else
            hipLaunchKernelGGL(place_k<false>, dim3((uint32_t)grid_), dim3(block()), lds_, t.stream, a);
        HIP_OR_FAIL(hipGetLastError(), "search launch");
        HIP_OR_FAIL(hipMemcpyAsync(t.status_h, t.status, P_ * sizeof(uint32_t), hipMemcpyDeviceToHost, t.stream),
                    "copy out");
        HIP_OR_FAIL(hipMemcpyAsync(t.ev_h, t.ev, P_ * sizeof(uint64_t), hipMemcpyDeviceToHost, t.stream), "copy out");
        HIP_OR_FAIL(hipEventRecord(t.done, t.stream), "event record");
        t.seed = seed;
        t.busy = true;
        t.started = std::chrono::steady_clock::now();
        return PTRHASH_OK;
    }

    // The outcome of a finished search; *failed: some part failed (reseed).
    int check(Attempt &t, bool *failed) {
        using namespace ptrhash;
        t.busy = false;
        *failed = false;
        for (uint64_t p = 0; p < P_; ++p) {
            const uint32_t st = t.status_h[p];
            if (st == kPlaceHeapFull || st == kPlaceTooLarge)
                return set_error(PTRHASH_E_RANGE, "device placement: part %llu outside the search's limits (%u)",
                                 (unsigned long long)p, st);
            if (st != kPlaceOk && st != kPlaceFailed)
                return set_error(PTRHASH_E_HIP, "device placement: part %llu ended with status %u",
                                 (unsigned long long)p, st);
            *failed |= st != kPlaceOk;
        }
        return PTRHASH_OK;
    }

    // One search with the given seed on slot 0, waited for.
    int search(uint64_t seed, bool *failed) {
        using namespace ptrhash;
        if (int rc = launch(att_[0], seed)) return rc;
        HIP_OR_FAIL(hipEventSynchronize(att_[0].done), "search");
        if (int rc = check(att_[0], failed)) return rc;
        phase("search");
        return PTRHASH_OK;
    }

    // Seconds after which a seed's search counts as stuck: three times a
    // generous estimate of a normal search (rounds of parts x buckets x
    // 1.5 us per placement) plus 2 s; PTRHASH_SPECULATE_MS overrides it.
    double stuck_after() const {
        if (const char *e = std::getenv("PTRHASH_SPECULATE_MS")) return std::atof(e) / 1e3;
        const double rounds = (double)((P_ + grid_ - 1) / grid_);
        return 2.0 + 3.0 * rounds * (double)B_ * 1.5e-6;
    }

    // Extra search slots that fit in free device memory (keeping 2 GiB and
    // a tenth of it spare), allocated now; returns the slots in use.
    int add_slots() {
        size_t freeb = 0, totalb = 0;
        if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return 1;
        const uint64_t spare = std::max<uint64_t>(2ull << 30, freeb / 10);
        int slots = 1;
        uint64_t avail = freeb > spare ? freeb - spare : 0;
        while (slots < kSpecSlots && avail >= attempt_bytes()) {
            if (alloc_attempt(att_[slots], true) != PTRHASH_OK) {
                (void)hipGetLastError();
                break;
            }
            avail -= attempt_bytes();
            ++slots;
        }
        return slots;
    }

    // Cancel every running search but `keep` and wait for them to stop. The
    // flag is a host store into coherent memory, so it does not queue behind
    // any device work.
    void cancel_others(const Attempt *keep) {
        for (Attempt &t : att_)
            if (t.busy && &t != keep) __atomic_store_n(t.cancel, 1u, __ATOMIC_SEQ_CST);
        for (Attempt &t : att_)
            if (t.busy && &t != keep) {
                (void)hipEventSynchronize(t.done);
                t.busy = false;
            }
    }

    // Seeds params->seed, +1, ... until one succeeds (at most kMaxSeeds).
    int run_seeds(ptrhash_params *params, uint8_t *pilots, void *remap, ptrhash_build_info *info) {
        using namespace ptrhash;
        const uint64_t base = params->seed;
        const double stuck = stuck_after();
        int slot_of[kMaxSeeds];
        for (int &x : slot_of) x = -1;
        int slots = 1, next_seed = 1;
        bool tried = false;  // side-by-side seeds tried (once)
        if (int rc = launch(att_[0], base)) return rc;
        slot_of[0] = 0;
        for (int cur = 0; cur < kMaxSeeds; ++cur) {
            Attempt &t = att_[slot_of[cur]];
            for (;;) {
                const hipError_t q = hipEventQuery(t.done);
                if (q == hipSuccess) break;
                if (q != hipErrorNotReady) {
                    cancel_others(&t);
                    return set_error(PTRHASH_E_HIP, "search: %s", hipGetErrorString(q));
                }
                const double ran = std::chrono::duration<double>(std::chrono::steady_clock::now() - t.started).count();
                if (!tried && ran > stuck && next_seed < kMaxSeeds) {
                    tried = true;
                    slots = add_slots();
                    for (int sl = 0; sl < slots && next_seed < kMaxSeeds; ++sl) {
                        if (att_[sl].busy) continue;
                        if (int rc = launch(att_[sl], base + (uint64_t)next_seed)) {
                            cancel_others(nullptr);
                            return rc;
                        }
                        slot_of[next_seed++] = sl;
                    }
                    if (timing_)
                        std::fprintf(stderr, "[build] seed %d still searching after %.1f s: %d seeds side by side\n",
                                     cur, ran, slots);
                }
                std::this_thread::sleep_for(std::chrono::milliseconds(1));
            }
            bool failed = false;
            const int rc = check(t, &failed);
            if (timing_)
                std::fprintf(stderr, "[build] search seed %d %s after %.3f s\n", cur, rc ? "error" : failed ? "failed" : "ok",
                             std::chrono::duration<double>(std::chrono::steady_clock::now() - t.started).count());
            if (rc) {
                cancel_others(nullptr);
                return rc;
            }
            if (!failed) {
                cancel_others(&t);
                phase("search");
                return finish(params, base + (uint64_t)cur, pilots, remap, info, (uint64_t)cur + 1, t);
            }
            // this slot is free again: the next seed not yet started goes there
            const int want = slots == 1 ? cur + 1 : next_seed;
            if (want < kMaxSeeds && slot_of[want] < 0) {
                if (int rc2 = launch(t, base + (uint64_t)want)) {
                    cancel_others(nullptr);
                    return rc2;
                }
                slot_of[want] = (int)(&t - att_.data());
                next_seed = want + 1;
            }
        }
        cancel_others(nullptr);
        if (info) *info = ptrhash_build_info{(uint64_t)kMaxSeeds, 0, 0, 0};
        return set_error(PTRHASH_E_BUILD, "construction failed for %d seeds", kMaxSeeds);
    }

    // The remap table from a finished search's taken-slot bitvector, built on
    // the device and copied to remap (host memory; none for REMAP_NONE).
    int device_remap(const ptrhash_params &p, Attempt &t, void *remap) {
        using namespace ptrhash;
        const uint64_t total = P_ * S_, len = total - n_, words = (total + 63) / 64;
        const uint64_t *taken = reinterpret_cast<const uint64_t *>(t.taken);
        hipStream_t s = t.stream;
        if (!rm_cfree_) {
            HIP_OR_FAIL(buf_.get(&rm_cfree_, words), "remap counts");
            HIP_OR_FAIL(buf_.get(&rm_ctaken_, words), "remap counts");
            HIP_OR_FAIL(buf_.get(&rm_ofree_, words), "remap offsets");
            HIP_OR_FAIL(buf_.get(&rm_otaken_, words), "remap offsets");
            HIP_OR_FAIL(buf_.get(&rm_err_, 1), "remap flags");
        }
        const dim3 grid(4096), block(256);
        hipLaunchKernelGGL(remap_counts_k, grid, block, 0, s, taken, words, n_, total, rm_cfree_, rm_ctaken_);
        HIP_OR_FAIL(hipGetLastError(), "remap counts launch");
        for (int i = 0; i < 2; ++i) {
            const uint64_t *in = i ? rm_ctaken_ : rm_cfree_;
            uint64_t *out = i ? rm_otaken_ : rm_ofree_;
            size_t temp = 0;
            HIP_OR_FAIL(hipcub::DeviceScan::ExclusiveSum(nullptr, temp, in, out, (int64_t)words, s), "scan sizing");
            if (temp > sort_temp_bytes_) {
                HIP_OR_FAIL(buf_.get(&sort_temp_, temp), "scan scratch");
                sort_temp_bytes_ = temp;
            }
            HIP_OR_FAIL(hipcub::DeviceScan::ExclusiveSum(sort_temp_, temp, in, out, (int64_t)words, s), "scan");
        }
        // the numbers of free slots below n and of taken slots at or above n must agree
        uint64_t last[4] = {0, 0, 0, 0};
        HIP_OR_FAIL(hipMemcpyAsync(&last[0], rm_ofree_ + words - 1, 8, hipMemcpyDeviceToHost, s), "copy out");
        HIP_OR_FAIL(hipMemcpyAsync(&last[1], rm_cfree_ + words - 1, 8, hipMemcpyDeviceToHost, s), "copy out");
        HIP_OR_FAIL(hipMemcpyAsync(&last[2], rm_otaken_ + words - 1, 8, hipMemcpyDeviceToHost, s), "copy out");
        HIP_OR_FAIL(hipMemcpyAsync(&last[3], rm_ctaken_ + words - 1, 8, hipMemcpyDeviceToHost, s), "copy out");
        HIP_OR_FAIL(hipStreamSynchronize(s), "copy out");
        const uint64_t nfree = last[0] + last[1], ntaken = last[2] + last[3];
        if (ntaken > nfree) return set_error(PTRHASH_E_BUILD, "remap: fewer free slots than overflow");
        if (ntaken < nfree) return set_error(PTRHASH_E_BUILD, "remap: unmatched free slot");
        const uint64_t rbytes = ptrhash_remap_bytes(&p);
        if (!rbytes || !len) return PTRHASH_OK;
        uint64_t *fl = nullptr, *F = nullptr;
        uint32_t *enc = nullptr;
        HIP_OR_FAIL(buf_.get(&fl, nfree), "remap free list");
        HIP_OR_FAIL(buf_.get(&F, len), "remap values");
        HIP_OR_FAIL(buf_.get(&enc, (rbytes + 3) / 4), "remap table");
        HIP_OR_FAIL(hipMemsetAsync(rm_err_, 0, sizeof(uint32_t), s), "memset");
        hipLaunchKernelGGL(remap_free_list_k, grid, block, 0, s, taken, words, n_, rm_ofree_, fl);
        HIP_OR_FAIL(hipGetLastError(), "remap free list launch");
        hipLaunchKernelGGL(remap_values_k, grid, block, 0, s, taken, n_, len, rm_otaken_, fl, F);
        HIP_OR_FAIL(hipGetLastError(), "remap values launch");
        if (p.remap_kind == PTRHASH_REMAP_CLEF)
            hipLaunchKernelGGL(remap_clef_k, grid, block, 0, s, F, len, enc, rm_err_);
        else
            hipLaunchKernelGGL(remap_u32_k, grid, block, 0, s, F, len, enc);
        HIP_OR_FAIL(hipGetLastError(), "remap encode launch");
        uint32_t err = 0;
        HIP_OR_FAIL(hipMemcpyAsync(&err, rm_err_, sizeof err, hipMemcpyDeviceToHost, s), "copy out");
        HIP_OR_FAIL(hipMemcpyAsync(remap, enc, rbytes, hipMemcpyDeviceToHost, s), "remap to host");
        HIP_OR_FAIL(hipStreamSynchronize(s), "copy out");
        if (err & 1u) return set_error(PTRHASH_E_REMAP_RANGE, "remap value beyond 40 bits");
        if (err & 2u) return set_error(PTRHASH_E_REMAP_RANGE, "a CacheLineEF line spans too far");
        return PTRHASH_OK;
    }

    // After a successful search: pilots and remap to the host, statistics.
    int finish(ptrhash_params *params, uint64_t seed, uint8_t *pilots, void *remap, ptrhash_build_info *info,
               uint64_t attempts) {
        return finish(params, seed, pilots, remap, info, attempts, att_[0]);
    }
    int finish(ptrhash_params *params, uint64_t seed, uint8_t *pilots, void *remap, ptrhash_build_info *info,
               uint64_t attempts, Attempt &t) {
        using namespace ptrhash;
        ptrhash_build_info local{};
        local.attempts = attempts;
        local.max_bucket_size = max_size_;
        for (uint64_t p = 0; p < P_; ++p) {
            local.evictions += t.ev_h[p];
            local.max_part_evictions = std::max(local.max_part_evictions, t.ev_h[p]);
        }
        HIP_OR_FAIL(hipMemcpyAsync(pilots, t.pil, total_, hipMemcpyDeviceToHost, t.stream), "pilots to host");
        if (int rc = device_remap(*params, t, remap)) return rc;
        phase("remap");
        params->seed = seed;
        if (info) *info = local;
        return PTRHASH_OK;
    }

    DevBufs &buffers() { return buf_; }

  private:
    DevBufs buf_;
    uint64_t n_;
    hipStream_t stream_;
    bool mod_ = false, timing_ = false;
    uint32_t helpers_ = 7;
    std::chrono::steady_clock::time_point tick_;
    uint64_t S_ = 0, P_ = 0, B_ = 0, total_ = 0, words_ = 0, grid_ = 0, taken_words_ = 0;
    size_t lds_ = 0, sort_temp_bytes_ = 0;
    ptrhash::DevMphf m_{};
    uint64_t *bst_ = nullptr, *ka_ = nullptr, *kb_ = nullptr, *ostart_ = nullptr;
    unsigned long long *maxes_ = nullptr;
    uint32_t *flags_ = nullptr;
    uint8_t *sort_temp_ = nullptr;
    std::vector<Attempt> att_;
    hipEvent_t prepared_ = nullptr;  // the search order is ready
    const uint64_t *H_ = nullptr, *okeys_ = nullptr;
    uint64_t *OH_ = nullptr;
    uint64_t max_size_ = 0;
    uint32_t size_bits_ = 0, id_bits_ = 0;
    uint64_t *rm_cfree_ = nullptr, *rm_ctaken_ = nullptr, *rm_ofree_ = nullptr, *rm_otaken_ = nullptr;
    uint32_t *rm_err_ = nullptr;
};

int build_gpu(const uint64_t *keys, uint64_t n, ptrhash_params *params, uint8_t *pilots, void *remap,
              ptrhash_build_info *info, hipStream_t stream) {
    using namespace ptrhash;
    if (!keys || !params || !pilots) return set_error(PTRHASH_E_INVAL, "NULL argument");
    if (int rc = check_build_params(n, params, PTRHASH_KEY_U64)) return rc;
    if (ptrhash_remap_bytes(params) && !remap) return set_error(PTRHASH_E_INVAL, "remap is NULL");
    GpuSearch g(params, n, stream);
    if (int rc = g.init()) return rc;
    uint64_t *ha = nullptr, *hb = nullptr;
    HIP_OR_FAIL(g.buffers().get(&ha, n), "device hashes");
    HIP_OR_FAIL(g.buffers().get(&hb, n), "device hashes");
    // the hash of a u64 key has no seed: hash, sort and order once
    hipLaunchKernelGGL(hash_keys_gpu_k, dim3(8192), dim3(256), 0, stream, keys, n, ha);
    HIP_OR_FAIL(hipGetLastError(), "hash launch");
    hipcub::DoubleBuffer<uint64_t> hdb(ha, hb);
    if (int rc = g.sort(hdb, nullptr)) return rc;
    g.phase("hash+sort");
    bool dup = false, overflow = false;
    if (int rc = g.prepare(hdb.Current(), hdb.Alternate(), &dup, &overflow)) return rc;
    if (dup) return set_error(PTRHASH_E_DUPLICATE, "two equal keys");
    if (overflow) return set_error(PTRHASH_E_BUILD, "a part holds more than S keys");
    // the order does not depend on the seed: seeds may be searched side by side
    return g.run_seeds(params, pilots, remap, info);
}

// Do two of the equal-hash pairs name the same string? (Then the keys are
// not distinct; otherwise a new seed separates them.)
int equal_strings(const uint8_t *data, const uint64_t *offsets, const std::vector<uint64_t> &pairs, uint32_t count,
                  hipStream_t stream, bool *same) {
    *same = false;
    for (uint32_t k = 0; k < count && k < kMaxPairs; ++k) {
        uint64_t o[2][2];
        for (int j = 0; j < 2; ++j)
            HIP_OR_FAIL(hipMemcpyAsync(o[j], offsets + pairs[2 * k + j], 2 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                       stream),
                        "offsets to host");
        HIP_OR_FAIL(hipStreamSynchronize(stream), "sync");
        const uint64_t la = o[0][1] - o[0][0], lb = o[1][1] - o[1][0];
        if (la != lb) continue;
        std::vector<uint8_t> a(la), b(lb);
        if (la) {
            HIP_OR_FAIL(hipMemcpyAsync(a.data(), data + o[0][0], la, hipMemcpyDeviceToHost, stream), "key to host");
            HIP_OR_FAIL(hipMemcpyAsync(b.data(), data + o[1][0], lb, hipMemcpyDeviceToHost, stream), "key to host");
            HIP_OR_FAIL(hipStreamSynchronize(stream), "sync");
        }
        if (a == b) {
            *same = true;
            return PTRHASH_OK;
        }
    }
    return PTRHASH_OK;
}

int build_bytes_gpu(const uint8_t *data, uint64_t data_len, const uint64_t *offsets, uint64_t n,
                    ptrhash_params *params, uint8_t *pilots, void *remap, ptrhash_build_info *info,
                    hipStream_t stream) {
    using namespace ptrhash;
    if (!data || !offsets || !params || !pilots) return set_error(PTRHASH_E_INVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(data) & 7u) return set_error(PTRHASH_E_INVAL, "data must be 8-byte aligned");
    if (data_len < kBytesPadding)
        return set_error(PTRHASH_E_INVAL, "data_len %llu is below the %llu bytes of padding",
                         (unsigned long long)data_len, (unsigned long long)kBytesPadding);
    if (int rc = check_build_params(n, params, PTRHASH_KEY_BYTES)) return rc;
    if (ptrhash_remap_bytes(params) && !remap) return set_error(PTRHASH_E_INVAL, "remap is NULL");
    // 128-bit hashes: the high half picks part and bucket, the low half the
    // slot; two keys collide only when both halves are equal
    const bool wide = params->hash_bits == 128;
    GpuSearch g(params, n, stream);
    if (int rc = g.init()) return rc;
    uint64_t *ha = nullptr, *hb = nullptr, *ia = nullptr, *ib = nullptr, *pairs = nullptr;
    uint64_t *lo_raw = nullptr, *lo = nullptr;
    uint32_t *npairs = nullptr;
    HIP_OR_FAIL(g.buffers().get(&ha, n), "device hashes");
    HIP_OR_FAIL(g.buffers().get(&hb, n), "device hashes");
    HIP_OR_FAIL(g.buffers().get(&ia, n), "key ids");
    HIP_OR_FAIL(g.buffers().get(&ib, n), "key ids");
    if (wide) {
        HIP_OR_FAIL(g.buffers().get(&lo_raw, n), "device hashes");
        HIP_OR_FAIL(g.buffers().get(&lo, n), "device hashes");
    }
    HIP_OR_FAIL(g.buffers().get(&pairs, 2 * kMaxPairs), "pairs");
    HIP_OR_FAIL(g.buffers().get(&npairs, 2), "pairs");
    // the offsets are on the device: check them there before any string is read
    {
        HIP_OR_FAIL(hipMemsetAsync(npairs, 0, sizeof(uint32_t), stream), "memset");
        hipLaunchKernelGGL(check_offsets_k, dim3(4096), dim3(256), 0, stream, offsets, n, bytes_end_limit(data_len),
                           npairs);
        HIP_OR_FAIL(hipGetLastError(), "offsets check launch");
        uint32_t bad = 0;
        HIP_OR_FAIL(hipMemcpyAsync(&bad, npairs, sizeof bad, hipMemcpyDeviceToHost, stream), "copy out");
        HIP_OR_FAIL(hipStreamSynchronize(stream), "sync");
        if (bad)
            return set_error(PTRHASH_E_INVAL, "offsets decrease, or a string ends later than data_len - %llu",
                             (unsigned long long)kBytesReadSlack);
    }
    std::vector<uint64_t> hpairs(2 * kMaxPairs);
    for (int attempt = 0; attempt < kMaxSeeds; ++attempt) {
        // the string hash depends on the seed: hash, sort and order per attempt
        const uint64_t seed = params->seed + (uint64_t)attempt;
        if (wide)
            hipLaunchKernelGGL(hash_strings128_gpu_k, dim3(8192), dim3(256), 0, stream, data, offsets, n, seed, ha,
                               lo_raw, ia);
        else
            hipLaunchKernelGGL(hash_strings_gpu_k, dim3(8192), dim3(256), 0, stream, data, offsets, n, seed, ha, ia);
        HIP_OR_FAIL(hipGetLastError(), "hash launch");
        hipcub::DoubleBuffer<uint64_t> hdb(ha, hb), idb(ia, ib);
        if (int rc = g.sort(hdb, &idb)) return rc;
        if (wide) {
            hipLaunchKernelGGL(gather_k, dim3(8192), dim3(256), 0, stream, lo_raw, idb.Current(), n, lo);
            HIP_OR_FAIL(hipGetLastError(), "gather launch");
        }
        g.phase("hash+sort");
        bool dup = false, overflow = false;
        // the ids' second buffer serves as the ordered-hash scratch
        if (int rc = g.prepare(hdb.Current(), idb.Alternate(), &dup, &overflow, wide ? lo : nullptr)) return rc;
        if (overflow) continue;  // a part with more than S keys: a new seed
        if (dup) {  // equal (high halves of the) hashes
            HIP_OR_FAIL(hipMemsetAsync(npairs, 0, 2 * sizeof(uint32_t), stream), "memset");
            if (wide)
                hipLaunchKernelGGL(equal_pairs128_k, dim3(4096), dim3(256), 0, stream, hdb.Current(), lo,
                                   idb.Current(), n, npairs, pairs);
            else
                hipLaunchKernelGGL(equal_pairs_k, dim3(4096), dim3(256), 0, stream, hdb.Current(), idb.Current(), n,
                                   npairs, pairs);
            HIP_OR_FAIL(hipGetLastError(), "pairs launch");
            uint32_t np[2] = {0, 0};
            HIP_OR_FAIL(hipMemcpyAsync(np, npairs, sizeof np, hipMemcpyDeviceToHost, stream), "copy out");
            HIP_OR_FAIL(hipMemcpyAsync(hpairs.data(), pairs, hpairs.size() * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                       stream),
                        "copy out");
            HIP_OR_FAIL(hipStreamSynchronize(stream), "sync");
            if (np[1])  // three equal high halves in a row: not every equal pair is adjacent
                return set_error(PTRHASH_E_RANGE, "device construction: three keys share a 64-bit hash half");
            if (np[0]) {
                bool same = false;
                if (int rc = equal_strings(data, offsets, hpairs, np[0], stream, &same)) return rc;
                if (same) return set_error(PTRHASH_E_DUPLICATE, "two equal keys");
                if (np[0] > kMaxPairs)  // more pairs than examined: the host construction checks them all
                    return set_error(PTRHASH_E_RANGE, "device construction: %u equal string hashes", np[0]);
                continue;  // distinct strings with one hash: a new seed
            }
            // 128-bit: equal high halves only; such keys share a bucket but not a slot hash
        }
        bool failed = false;
        if (int rc = g.search(seed, &failed)) return rc;
        if (!failed) return g.finish(params, seed, pilots, remap, info, (uint64_t)attempt + 1);
    }
    if (info) *info = ptrhash_build_info{(uint64_t)kMaxSeeds, 0, 0, 0};
    return set_error(PTRHASH_E_BUILD, "construction failed for %d seeds", kMaxSeeds);
}

}  // namespace

extern "C" {

PTRHASH_API int ptrhash_build_u64_gpu(const uint64_t *keys, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                                      void *remap, ptrhash_build_info *info, hipStream_t stream) {
    try {
        return build_gpu(keys, n, params, pilots, remap, info, stream);
    } catch (const std::bad_alloc &) {
        return ptrhash::set_error(PTRHASH_E_NOMEM, "host allocation failed during construction");
    }
}

PTRHASH_API int ptrhash_build_bytes_gpu(const uint8_t *data, uint64_t data_len, const uint64_t *offsets, uint64_t n,
                                        ptrhash_params *params, uint8_t *pilots, void *remap,
                                        ptrhash_build_info *info, hipStream_t stream) {
    try {
        return build_bytes_gpu(data, data_len, offsets, n, params, pilots, remap, info, stream);
    } catch (const std::bad_alloc &) {
        return ptrhash::set_error(PTRHASH_E_NOMEM, "host allocation failed during construction");
    }
}

}  // extern "C"
