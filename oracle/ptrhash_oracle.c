/*
 * PtrHash CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain single-threaded C. Every function names the passage of the PtrHash
 * paper (arXiv 2502.15539) that it follows. No blocking, no fusion, no
 * reordering beyond what those definitions state. The readings taken where
 * the paper is silent are marked "reading:" in the comments.
 *
 * Parity unpinned by the paper: orc_hash_bytes (project-defined stand-in
 * for GxHash, whose steps the paper does not give).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---- 128-bit products: hi(a*b), lo(a*b) (Section 3.1, Overview) ---- */
uint64_t orc_hi(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * (u128)b) >> 64); }
uint64_t orc_lo(uint64_t a, uint64_t b) { return (uint64_t)((u128)a * (u128)b); }

static uint64_t next_pow2(uint64_t v)
{
    uint64_t r = 1;
    while (r < v) r <<= 1;
    return r;
}

static uint32_t log2_exact(uint64_t v)
{
    uint32_t l = 0;
    while ((1ULL << l) < v) l++;
    return l;
}

/*
 * Parameter rule (Section 3.1, "Parameter values"): the keys per part
 * alpha*S >= 80000*ln(n/80000), with a minimum of 80000; S a power of two
 * (so that reduce is a multiply and a mask, "The reduce function");
 * P = ceil(n/(alpha*S)); B = ceil(alpha*S/lambda).
 * reading: when this gives a single part, S shrinks to the smallest power of
 * two >= n/alpha, so that small inputs do not leave most slots empty (the
 * paper notes that a power-of-two S can leave up to half the slots empty).
 */
int orc_params_for(uint64_t n, double alpha, double lambda, int32_t gamma,
                   uint32_t log2_slots_override, uint64_t seed, orc_params *out)
{
    if (!out || n == 0 || !(alpha > 0.0 && alpha <= 1.0) || !(lambda > 0.0)) return ORC_EINVAL;
    if (gamma != ORC_GAMMA_CUBIC && gamma != ORC_GAMMA_LINEAR) return ORC_EINVAL;
    uint64_t S;
    if (log2_slots_override) {
        if (log2_slots_override > 40) return ORC_EINVAL;
        S = 1ULL << log2_slots_override;
    } else {
        double K = 80000.0 * log((double)n / 80000.0);
        if (K < 80000.0) K = 80000.0;
        S = next_pow2((uint64_t)ceil(K / alpha));
    }
    uint64_t P = (uint64_t)ceil((double)n / (alpha * (double)S));
    if (P < 1) P = 1;
    if (P == 1 && !log2_slots_override) S = next_pow2((uint64_t)ceil((double)n / alpha));
    uint64_t B = (uint64_t)ceil(alpha * (double)S / lambda);
    if (B < 1) B = 1;
    if (B > 0xFFFFFFFFULL) return ORC_EINVAL;
    return orc_params_explicit(n, P, log2_exact(S), (uint32_t)B, gamma, seed, out);
}

int orc_params_explicit(uint64_t n, uint64_t P, uint32_t log2_slots, uint32_t B,
                        int32_t gamma, uint64_t seed, orc_params *out)
{
    if (!out || n == 0 || P == 0 || B == 0 || log2_slots > 40) return ORC_EINVAL;
    if (gamma != ORC_GAMMA_CUBIC && gamma != ORC_GAMMA_LINEAR) return ORC_EINVAL;
    uint64_t S = 1ULL << log2_slots;
    if (P > (1ULL << 40) / S) return ORC_EINVAL;
    if (P * S < n) return ORC_EINVAL;
    memset(out, 0, sizeof *out);
    out->n = n;
    out->num_parts = P;
    out->slots_per_part = S;
    out->log2_slots = log2_slots;
    out->buckets_per_part = B;
    out->seed = seed;
    out->gamma = gamma;
    out->remap_len = P * S - n;
    return ORC_OK;
}

/*
 * reading: the fast-mod variant ("The reduce function"): a single part whose
 * S is not a power of two, so that x mod S depends on every bit of x.
 */
int orc_params_single_mod(uint64_t n, uint64_t S, uint32_t B, int32_t gamma, uint64_t seed, orc_params *out)
{
    if (!out || n == 0 || B == 0 || S < n || S < 2 || (S & (S - 1)) == 0 || S > (1ULL << 40)) return ORC_EINVAL;
    if (gamma != ORC_GAMMA_CUBIC && gamma != ORC_GAMMA_LINEAR) return ORC_EINVAL;
    memset(out, 0, sizeof *out);
    out->n = n;
    out->num_parts = 1;
    out->slots_per_part = S;
    out->log2_slots = 0;
    out->buckets_per_part = B;
    out->seed = seed;
    out->gamma = gamma;
    out->reduce_kind = ORC_REDUCE_MOD;
    out->remap_len = S - n;
    return ORC_OK;
}

int orc_params_for_single_mod(uint64_t n, double alpha, double lambda, int32_t gamma, uint64_t seed,
                              orc_params *out)
{
    if (!out || n == 0 || !(alpha > 0.0 && alpha <= 1.0) || !(lambda > 0.0)) return ORC_EINVAL;
    /* reading: at least 16 free slots, so that tiny inputs still build */
    uint64_t S = (uint64_t)ceil((double)n / alpha);
    if (S < n + 16) S = n + 16;
    if ((S & (S - 1)) == 0) S++;
    uint64_t B = (uint64_t)ceil(alpha * (double)S / lambda);
    if (B < 1) B = 1;
    if (B > 0xFFFFFFFFULL) return ORC_EINVAL;
    return orc_params_single_mod(n, S, (uint32_t)B, gamma, seed, out);
}

/* ---- Key hashes (Section 3.1, "Hash functions") ---- */

/* Integer keys: h(k) = C*k, invertible modulo 2^64 because C is odd. */
uint64_t orc_hash_u64(uint64_t key) { return ORC_C * key; }

/* MurmurHash3's 64-bit finalizer (Appleby): xor-shift, multiply, xor-shift,
 * multiply, xor-shift; every step is invertible. */
uint64_t orc_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

/*
 * reading: byte-string keys. The paper hashes strings with 64-bit GxHash
 * (AES based, steps not given). This project hash is used instead: the
 * state starts at seed xor (len*C), absorbs each little-endian 8-byte word
 * of the string (the last one zero-padded) as st = fmix64(st xor w), and
 * the hash is fmix64(st).
 */
uint64_t orc_hash_bytes(uint64_t seed, const uint8_t *s, uint64_t len)
{
    uint64_t st = seed ^ (len * ORC_C);
    for (uint64_t i = 0; i < len; i += 8) {
        uint64_t w = 0;
        for (uint64_t j = 0; j < 8 && i + j < len; j++) w |= (uint64_t)s[i + j] << (8 * j);
        st = orc_fmix64(st ^ w);
    }
    return orc_fmix64(st);
}

/*
 * reading: beyond 2^32 keys the paper switches to a 128-bit hash whose high
 * 64 bits choose part and bucket and whose low 64 bits choose the slot
 * ("Hash functions"). The 128-bit project hash is the 64-bit one twice, the
 * second time with the seed xor-ed with 0x9E3779B97F4A7C15.
 */
void orc_hash_bytes128(uint64_t seed, const uint8_t *s, uint64_t len, uint64_t *hi, uint64_t *lo)
{
    *hi = orc_hash_bytes(seed, s, len);
    *lo = orc_hash_bytes(seed ^ 0x9E3779B97F4A7C15ULL, s, len);
}

/* ---- Part and bucket (eq. partbucket; Section 3.3) ---- */

/* part(k) = hi(P*h(k)) = floor(P*h/2^64). */
uint64_t orc_part(const orc_params *p, uint64_t h) { return orc_hi(p->num_parts, h); }

/* relative position x = lo(P*h(k)), a fraction of 2^64. */
uint64_t orc_rel(const orc_params *p, uint64_t h) { return orc_lo(p->num_parts, h); }

/*
 * Bucket assignment functions on 64-bit fixed point (Section 3.3,
 * "Approximations"): gamma_1(x) = x; gamma_3(x) = (255/256)(x^2+x^3)/2 + x/256
 * with x^2 = hi(x*x) and x^3 = hi(x^2 * x).
 * reading: (x^2+x^3)/2 is taken as (x^2>>1)+(x^3>>1) and the 255/256 factor
 * as y - (y>>8); the result never exceeds x, so it stays below 2^64.
 */
uint64_t orc_gamma(int32_t kind, uint64_t x)
{
    if (kind == ORC_GAMMA_LINEAR) return x;
    uint64_t x2 = orc_hi(x, x);
    uint64_t x3 = orc_hi(x2, x);
    uint64_t y = (x2 >> 1) + (x3 >> 1);
    return y - (y >> 8) + (x >> 8);
}

/*
 * bucket(k) = hi(B * gamma(x)) is the bucket inside the part (eq.
 * partbucket). reading: the pilot array p_0..p_{P*B-1} is indexed by the
 * global bucket part*B + bucket (Section 3.1, "Slots and pilots"; Fig. 1).
 */
uint64_t orc_bucket(const orc_params *p, uint64_t h)
{
    uint64_t part = orc_part(p, h);
    uint64_t x = orc_rel(p, h);
    uint64_t g = orc_gamma(p->gamma, x);
    return part * (uint64_t)p->buckets_per_part + orc_hi((uint64_t)p->buckets_per_part, g);
}

/* ---- Pilot hash, reduce and slot (eq. slot; Section 3.1) ---- */

/* h_p(p) = C * (p xor seed). */
uint64_t orc_hp(uint64_t seed, uint32_t pilot) { return ORC_C * ((uint64_t)pilot ^ seed); }

/* reduce(x, S) = hi(C*x) mod S for S a power of two. */
uint64_t orc_reduce(uint64_t x, uint64_t S) { return orc_hi(ORC_C, x) & (S - 1); }

/* reduce(x, S) = x mod S (S not a power of two, single part). */
uint64_t orc_reduce_mod(uint64_t x, uint64_t S) { return x % S; }

static uint64_t reduce_of(const orc_params *p, uint64_t x)
{
    return p->reduce_kind == ORC_REDUCE_MOD ? orc_reduce_mod(x, p->slots_per_part)
                                            : orc_reduce(x, p->slots_per_part);
}

/* slot(k) = part(k)*S + reduce(h(k) xor h_p(p_bucket(k)), S). */
uint64_t orc_slot(const orc_params *p, uint64_t h, uint32_t pilot)
{
    return orc_part(p, h) * p->slots_per_part + reduce_of(p, h ^ orc_hp(p->seed, pilot));
}

uint64_t orc_slot2(const orc_params *p, uint64_t h_part, uint64_t h_slot, uint32_t pilot)
{
    return orc_part(p, h_part) * p->slots_per_part + reduce_of(p, h_slot ^ orc_hp(p->seed, pilot));
}

/* ---- CacheLineEF (Section 3.4, eq. clef) ---- */

#define CLEF_VALUES 44
#define CLEF_LINE 64

uint64_t orc_clef_bytes(uint64_t len) { return (len + CLEF_VALUES - 1) / CLEF_VALUES * CLEF_LINE; }

static uint64_t load_le64(const uint8_t *b)
{
    uint64_t v = 0;
    for (int i = 0; i < 8; i++) v |= (uint64_t)b[i] << (8 * i);
    return v;
}

static void store_le64(uint8_t *b, uint64_t v)
{
    for (int i = 0; i < 8; i++) b[i] = (uint8_t)(v >> (8 * i));
}

/*
 * Encode a non-decreasing list in chunks of 44 values, one 64-byte line
 * each: a 32-bit offset floor(v_0/2^8), 128 bits where bit
 * i + floor(v_i/2^8) - floor(v_0/2^8) is set for each i, and the 44 low
 * bytes v_i mod 2^8. reading (the figure is not in the text): the fields are
 * laid out in that order, little endian: bytes [0,4) offset, [4,12) bits
 * 0..63, [12,20) bits 64..127, [20,64) low bytes. A chunk whose bits do not
 * fit in 128, or whose offset needs more than 32 bits, is an error.
 */
int orc_clef_encode(const uint64_t *F, uint64_t len, uint8_t *out)
{
    if (len && (!F || !out)) return ORC_EINVAL;
    uint64_t lines = (len + CLEF_VALUES - 1) / CLEF_VALUES;
    memset(out, 0, lines * CLEF_LINE);
    for (uint64_t c = 0; c < lines; c++) {
        uint64_t first = c * CLEF_VALUES;
        uint64_t cnt = len - first < CLEF_VALUES ? len - first : CLEF_VALUES;
        uint64_t off = F[first] >> 8;
        if (off > 0xFFFFFFFFULL) return ORC_ECLEF_RANGE;
        uint64_t bits[2] = {0, 0};
        uint8_t *line = out + c * CLEF_LINE;
        for (uint64_t i = 0; i < cnt; i++) {
            uint64_t v = F[first + i];
            if (i > 0 && v < F[first + i - 1]) return ORC_EINVAL;
            uint64_t bit = i + (v >> 8) - off;
            if (bit > 127) return ORC_ECLEF_RANGE;
            bits[bit / 64] |= 1ULL << (bit % 64);
            line[20 + i] = (uint8_t)(v & 0xFF);
        }
        line[0] = (uint8_t)off;
        line[1] = (uint8_t)(off >> 8);
        line[2] = (uint8_t)(off >> 16);
        line[3] = (uint8_t)(off >> 24);
        store_le64(line + 4, bits[0]);
        store_le64(line + 12, bits[1]);
    }
    return ORC_OK;
}

/* select(r): position of the r-th (from 0) set bit of the 128-bit word,
 * by scanning the bits in order. Returns 128 if there are not r+1 bits. */
uint32_t orc_select128(uint64_t lo, uint64_t hi, uint32_t r)
{
    uint32_t seen = 0;
    for (uint32_t b = 0; b < 128; b++) {
        uint64_t w = b < 64 ? lo : hi;
        if ((w >> (b % 64)) & 1) {
            if (seen == r) return b;
            seen++;
        }
    }
    return 128;
}

/* Lookup (Section 3.4, "Lookup"): v_i = 2^8*offset + 2^8*(select(i)-i) + low_i. */
uint64_t orc_clef_get(const uint8_t *clef, uint64_t i)
{
    const uint8_t *line = clef + (i / CLEF_VALUES) * CLEF_LINE;
    uint32_t j = (uint32_t)(i % CLEF_VALUES);
    uint64_t off = (uint64_t)line[0] | ((uint64_t)line[1] << 8) | ((uint64_t)line[2] << 16) |
                   ((uint64_t)line[3] << 24);
    uint32_t sel = orc_select128(load_le64(line + 4), load_le64(line + 12), j);
    return 256 * off + 256 * (uint64_t)(sel - j) + line[20 + j];
}

/* ---- Query (eq. partbucket, eq. slot, Section 3.4 "Remapping") ---- */

uint64_t orc_query_hash(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                        const void *remap, uint64_t h)
{
    return orc_query_hash2(p, pilots, remap_kind, remap, h, h);
}

uint64_t orc_query_hash2(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                         const void *remap, uint64_t h_bucket, uint64_t h_slot)
{
    uint64_t b = orc_bucket(p, h_bucket);
    uint64_t slot = orc_slot2(p, h_bucket, h_slot, pilots[b]);
    if (remap_kind == ORC_REMAP_NONE || slot < p->n) return slot;
    if (remap_kind == ORC_REMAP_PLAIN) return ((const uint64_t *)remap)[slot - p->n];
    return orc_clef_get((const uint8_t *)remap, slot - p->n);
}

int orc_query_u64(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                  const void *remap, const uint64_t *keys, uint64_t nq, uint64_t *out)
{
    if (!p || !pilots || (nq && (!keys || !out))) return ORC_EINVAL;
    if (remap_kind != ORC_REMAP_NONE && p->remap_len && !remap) return ORC_EINVAL;
    for (uint64_t i = 0; i < nq; i++)
        out[i] = orc_query_hash(p, pilots, remap_kind, remap, orc_hash_u64(keys[i]));
    return ORC_OK;
}

int orc_query_bytes(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                    const void *remap, const uint8_t *data, const uint64_t *offsets,
                    uint64_t nq, uint64_t *out)
{
    if (!p || !pilots || (nq && (!data || !offsets || !out))) return ORC_EINVAL;
    if (remap_kind != ORC_REMAP_NONE && p->remap_len && !remap) return ORC_EINVAL;
    for (uint64_t i = 0; i < nq; i++) {
        uint64_t hb, hs;
        if (p->hash_bits == 128) {
            orc_hash_bytes128(p->seed, data + offsets[i], offsets[i + 1] - offsets[i], &hb, &hs);
        } else {
            hb = orc_hash_bytes(p->seed, data + offsets[i], offsets[i + 1] - offsets[i]);
            hs = hb;
        }
        out[i] = orc_query_hash2(p, pilots, remap_kind, remap, hb, hs);
    }
    return ORC_OK;
}

/* ---- Construction (Section 3.1 "Construction", Section 3.2) ---- */

/* Max-heap of a part's buckets ordered by (size descending, id ascending):
 * larger buckets are placed first ("sorts the buckets from large to small");
 * reading: ties go to the smaller bucket id. */
typedef struct {
    uint32_t *a;
    uint64_t len;
    const uint64_t *size; /* local bucket -> size */
} heap_t;

static int heap_before(const heap_t *h, uint32_t x, uint32_t y)
{
    if (h->size[x] != h->size[y]) return h->size[x] > h->size[y];
    return x < y;
}

static void heap_push(heap_t *h, uint32_t v)
{
    uint64_t i = h->len++;
    h->a[i] = v;
    while (i > 0) {
        uint64_t parent = (i - 1) / 2;
        if (!heap_before(h, h->a[i], h->a[parent])) break;
        uint32_t t = h->a[i];
        h->a[i] = h->a[parent];
        h->a[parent] = t;
        i = parent;
    }
}

static uint32_t heap_pop(heap_t *h)
{
    uint32_t top = h->a[0];
    h->a[0] = h->a[--h->len];
    uint64_t i = 0;
    for (;;) {
        uint64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->len && heap_before(h, h->a[l], h->a[m])) m = l;
        if (r < h->len && heap_before(h, h->a[r], h->a[m])) m = r;
        if (m == i) break;
        uint32_t t = h->a[i];
        h->a[i] = h->a[m];
        h->a[m] = t;
        i = m;
    }
    return top;
}

#define RECENT 16
#define EMPTY (-1)

typedef struct {
    const orc_params *p;
    const uint64_t *h;      /* key hashes (part and bucket) */
    const uint64_t *hs;     /* key hashes for the slot (= h unless 128-bit) */
    const uint64_t *order;  /* key ids grouped by global bucket */
    const uint64_t *start;  /* global bucket -> first position in order */
    uint8_t *pilots;
    int64_t *owner;         /* local slot -> local bucket or EMPTY */
    uint64_t *size;         /* local bucket -> size */
    uint32_t *heap_buf;
    uint64_t *slots;        /* scratch, one entry per key of the largest bucket */
    uint64_t *victim_slots; /* same size */
    orc_trace *trace;       /* optional record of every placement */
    uint32_t attempt;
} part_ctx;

/* Local slot of every key of local bucket b under pilot p; returns the
 * bucket size. */
static uint64_t bucket_slots(part_ctx *c, uint64_t part, uint32_t b, uint32_t pilot, uint64_t *slots)
{
    uint64_t g = part * c->p->buckets_per_part + b;
    uint64_t s = c->start[g + 1] - c->start[g];
    for (uint64_t j = 0; j < s; j++)
        slots[j] = reduce_of(c->p, c->hs[c->order[c->start[g] + j]] ^ orc_hp(c->p->seed, pilot));
    return s;
}

static int distinct(const uint64_t *slots, uint64_t s)
{
    for (uint64_t i = 0; i < s; i++)
        for (uint64_t j = i + 1; j < s; j++)
            if (slots[i] == slots[j]) return 0;
    return 1;
}

static int in_recent(const int64_t *recent, int64_t b)
{
    for (int i = 0; i < RECENT; i++)
        if (recent[i] == b) return 1;
    return 0;
}

/*
 * Hash-evict placement of one part (Section 3.2, "Hash-evict"):
 * buckets are taken largest first from a priority queue; a bucket gets the
 * smallest pilot in [0, 256) whose slots are free (and distinct). If there
 * is none, the pilot with the least weighted collisions is used, where a
 * collision with a key of a bucket of size s weighs s^2; buckets among the
 * 16 most recently placed are never evicted; the colliding buckets are
 * evicted (their slots emptied, pushed back on the queue) and the bucket is
 * placed. A part fails after more than factor*S evictions (Section 4.1.2).
 * reading: pilots whose own keys collide among themselves are never used;
 * collision costs add up per colliding key; ties go to the smallest pilot.
 */
static int place_part(part_ctx *c, uint64_t part, uint64_t max_evictions, orc_build_stats *st)
{
    const orc_params *p = c->p;
    uint64_t S = p->slots_per_part, B = p->buckets_per_part;
    for (uint64_t s = 0; s < S; s++) c->owner[s] = EMPTY;
    heap_t heap = {c->heap_buf, 0, c->size};
    for (uint32_t b = 0; b < B; b++) {
        uint64_t g = part * B + b;
        c->size[b] = c->start[g + 1] - c->start[g];
        c->pilots[g] = 0; /* empty buckets keep pilot 0 */
        if (c->size[b] > st->max_bucket_size) st->max_bucket_size = c->size[b];
    }
    for (uint32_t b = 0; b < B; b++)
        if (c->size[b]) heap_push(&heap, b);

    int64_t recent[RECENT];
    for (int i = 0; i < RECENT; i++) recent[i] = EMPTY;
    int recent_pos = 0;
    uint64_t evictions = 0;
    uint64_t *slots = c->slots;

    while (heap.len) {
        uint32_t b = heap_pop(&heap);
        int chosen = -1;
        uint64_t evicted = 0;
        for (uint32_t pl = 0; pl < 256 && chosen < 0; pl++) {
            uint64_t s = bucket_slots(c, part, b, pl, slots);
            if (!distinct(slots, s)) continue;
            int free_all = 1;
            for (uint64_t j = 0; j < s; j++)
                if (c->owner[slots[j]] != EMPTY) { free_all = 0; break; }
            if (free_all) chosen = (int)pl;
        }
        if (chosen < 0) {
            uint64_t best_cost = UINT64_MAX;
            for (uint32_t pl = 0; pl < 256; pl++) {
                uint64_t s = bucket_slots(c, part, b, pl, slots);
                if (!distinct(slots, s)) continue;
                uint64_t cost = 0;
                int ok = 1;
                for (uint64_t j = 0; j < s; j++) {
                    int64_t o = c->owner[slots[j]];
                    if (o == EMPTY) continue;
                    if (in_recent(recent, o)) { ok = 0; break; }
                    cost += c->size[o] * c->size[o];
                }
                if (ok && cost < best_cost) { best_cost = cost; chosen = (int)pl; }
            }
            if (chosen < 0) return ORC_EPART_FAIL;
            uint64_t s = bucket_slots(c, part, b, (uint32_t)chosen, slots);
            uint64_t before = evictions;
            uint64_t *victim_slots = c->victim_slots;
            for (uint64_t j = 0; j < s; j++) {
                int64_t o = c->owner[slots[j]];
                if (o == EMPTY) continue;
                uint64_t vs = bucket_slots(c, part, (uint32_t)o, c->pilots[part * B + o], victim_slots);
                for (uint64_t t = 0; t < vs; t++) c->owner[victim_slots[t]] = EMPTY;
                heap_push(&heap, (uint32_t)o);
                evictions++;
            }
            evicted = evictions - before;
        }
        uint64_t s = bucket_slots(c, part, b, (uint32_t)chosen, slots);
        for (uint64_t j = 0; j < s; j++) c->owner[slots[j]] = b;
        c->pilots[part * B + b] = (uint8_t)chosen;
        st->placements++;
        if (c->trace) {
            orc_trace *tr = c->trace;
            if (tr->len < tr->cap) {
                orc_trace_rec *r = &tr->rec[tr->len++];
                r->part = part;
                r->bucket = b;
                r->pilot = (uint32_t)chosen;
                r->evicted = (uint32_t)evicted;
                r->attempt = c->attempt;
                r->part_evictions = evictions;
            }
            tr->total++;
        }
        recent[recent_pos] = b;
        recent_pos = (recent_pos + 1) % RECENT;
        if (evictions > max_evictions) return ORC_EPART_FAIL;
    }
    st->evictions += evictions;
    if (evictions > st->max_part_evictions) st->max_part_evictions = evictions;
    return ORC_OK;
}

/* Key equality hook: 1 if keys a and b (same hash) are the same key. */
typedef int (*same_key_fn)(const void *ctx, uint64_t a, uint64_t b);

/*
 * One construction attempt over given hashes: group keys by global bucket,
 * reject parts with more than S keys, detect equal hashes inside a bucket,
 * place every part, then build the remap table F (Section 3.4
 * "Remapping"): with q_0 < ... < q_{R-1} the taken slots >= n and
 * L_0 < ... < L_{R-1} the free slots < n, F[q_i - n] = L_i, and every other
 * entry repeats its predecessor (reading: the entries before the first
 * defined one are 0).
 */
static int build_attempt(const orc_params *p, const uint64_t *h, const uint64_t *hs, same_key_fn same,
                         const void *sctx, uint8_t *pilots, uint64_t *F, orc_build_stats *st,
                         uint64_t max_evictions, orc_trace *trace, uint32_t attempt)
{
    uint64_t n = p->n, P = p->num_parts, S = p->slots_per_part, B = p->buckets_per_part;
    uint64_t nb = P * B;
    int rc = ORC_OK;
    uint64_t *bucket = malloc(n * sizeof *bucket);
    uint64_t *start = calloc(nb + 1, sizeof *start);
    uint64_t *fill = malloc((nb + 1) * sizeof *fill);
    uint64_t *order = malloc(n * sizeof *order);
    int64_t *owner = malloc(S * sizeof *owner);
    uint64_t *size = malloc(B * sizeof *size);
    uint32_t *heap_buf = malloc(B * sizeof *heap_buf);
    uint8_t *taken = calloc(P * S, 1);
    uint64_t *slots = NULL, *victim_slots = NULL, max_size = 1;
    part_ctx c;
    if (!bucket || !start || !fill || !order || !owner || !size || !heap_buf || !taken) {
        rc = ORC_ENOMEM;
        goto out;
    }
    for (uint64_t i = 0; i < n; i++) {
        bucket[i] = orc_bucket(p, h[i]);
        start[bucket[i] + 1]++;
    }
    for (uint64_t g = 0; g < nb; g++) start[g + 1] += start[g];
    memcpy(fill, start, (nb + 1) * sizeof *fill);
    for (uint64_t i = 0; i < n; i++) order[fill[bucket[i]]++] = i;

    for (uint64_t part = 0; part < P; part++)
        if (start[(part + 1) * B] - start[part * B] > S) { rc = ORC_EPART_OVERFLOW; goto out; }
    for (uint64_t g = 0; g < nb; g++)
        if (start[g + 1] - start[g] > max_size) max_size = start[g + 1] - start[g];
    slots = malloc(max_size * sizeof *slots);
    victim_slots = malloc(max_size * sizeof *victim_slots);
    if (!slots || !victim_slots) { rc = ORC_ENOMEM; goto out; }

    for (uint64_t g = 0; g < nb; g++)
        for (uint64_t a = start[g]; a < start[g + 1]; a++)
            for (uint64_t b = a + 1; b < start[g + 1]; b++)
                if (h[order[a]] == h[order[b]] && hs[order[a]] == hs[order[b]]) {
                    rc = same(sctx, order[a], order[b]) ? ORC_EDUPLICATE : ORC_EPART_FAIL;
                    goto out;
                }

    c.p = p;
    c.h = h;
    c.hs = hs;
    c.order = order;
    c.start = start;
    c.pilots = pilots;
    c.owner = owner;
    c.size = size;
    c.heap_buf = heap_buf;
    c.slots = slots;
    c.victim_slots = victim_slots;
    c.trace = trace;
    c.attempt = attempt;
    for (uint64_t part = 0; part < P; part++) {
        rc = place_part(&c, part, max_evictions, st);
        if (rc) goto out;
        for (uint64_t s = 0; s < S; s++)
            if (owner[s] != EMPTY) taken[part * S + s] = 1;
    }

    /* remap */
    {
        uint64_t len = P * S - n, li = 0, prev = 0;
        for (uint64_t t = 0; t < len; t++) {
            if (taken[n + t]) {
                while (li < n && taken[li]) li++;
                if (li >= n) { rc = ORC_EINVAL; goto out; }
                F[t] = li++;
            } else {
                F[t] = prev;
            }
            prev = F[t];
        }
        while (li < n && taken[li]) li++;
        if (li != n) rc = ORC_EINVAL; /* as many gaps as taken slots >= n */
    }
out:
    free(bucket);
    free(start);
    free(fill);
    free(order);
    free(owner);
    free(size);
    free(heap_buf);
    free(taken);
    free(slots);
    free(victim_slots);
    return rc;
}

static int same_u64(const void *ctx, uint64_t a, uint64_t b)
{
    const uint64_t *keys = ctx;
    return keys[a] == keys[b];
}

typedef struct {
    const uint8_t *data;
    const uint64_t *offsets;
} bytes_ctx;

static int same_bytes(const void *ctx, uint64_t a, uint64_t b)
{
    const bytes_ctx *k = ctx;
    uint64_t la = k->offsets[a + 1] - k->offsets[a], lb = k->offsets[b + 1] - k->offsets[b];
    return la == lb && memcmp(k->data + k->offsets[a], k->data + k->offsets[b], la) == 0;
}

static void default_cfg(const orc_build_cfg *cfg, uint64_t *factor, uint64_t *attempts)
{
    *factor = cfg ? cfg->eviction_factor : 10;
    *attempts = cfg && cfg->max_attempts ? cfg->max_attempts : 16;
}

/*
 * reading: on a failed part the whole construction restarts with seed+1
 * (the seed changes every pilot hash), up to max_attempts times. Integer
 * keys cannot fix an overfull part this way (h does not depend on the seed).
 */
int orc_build_u64(orc_params *p, const uint64_t *keys, const orc_build_cfg *cfg,
                  uint8_t *pilots, uint64_t *F, orc_build_stats *st)
{
    return orc_build_u64_traced(p, keys, cfg, pilots, F, st, NULL);
}

int orc_build_u64_traced(orc_params *p, const uint64_t *keys, const orc_build_cfg *cfg,
                         uint8_t *pilots, uint64_t *F, orc_build_stats *st, orc_trace *trace)
{
    if (!p || !keys || !pilots || (p->remap_len && !F)) return ORC_EINVAL;
    orc_build_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof *st);
    uint64_t factor, attempts;
    default_cfg(cfg, &factor, &attempts);
    uint64_t *h = malloc(p->n * sizeof *h);
    if (!h) return ORC_ENOMEM;
    for (uint64_t i = 0; i < p->n; i++) h[i] = orc_hash_u64(keys[i]);
    int rc = ORC_EBUILD_FAILED;
    for (uint64_t a = 0; a < attempts; a++) {
        orc_build_stats s1;
        memset(&s1, 0, sizeof s1);
        st->attempts = a + 1;
        rc = build_attempt(p, h, h, same_u64, keys, pilots, F, &s1, factor * p->slots_per_part, trace,
                           (uint32_t)a);
        st->placements += s1.placements;
        st->max_bucket_size = s1.max_bucket_size;
        if (rc != ORC_EPART_FAIL) {
            st->evictions = s1.evictions;
            st->max_part_evictions = s1.max_part_evictions;
            break;
        }
        rc = ORC_EBUILD_FAILED;
        p->seed++;
    }
    free(h);
    return rc;
}

int orc_build_bytes(orc_params *p, const uint8_t *data, const uint64_t *offsets,
                    const orc_build_cfg *cfg, uint8_t *pilots, uint64_t *F,
                    orc_build_stats *st)
{
    if (!p || !data || !offsets || !pilots || (p->remap_len && !F)) return ORC_EINVAL;
    orc_build_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof *st);
    uint64_t factor, attempts;
    default_cfg(cfg, &factor, &attempts);
    uint64_t *h = malloc(p->n * sizeof *h);
    uint64_t *hs = p->hash_bits == 128 ? malloc(p->n * sizeof *hs) : h;
    if (!h || !hs) {
        free(h);
        if (hs != h) free(hs);
        return ORC_ENOMEM;
    }
    bytes_ctx bc = {data, offsets};
    int rc = ORC_EBUILD_FAILED;
    for (uint64_t a = 0; a < attempts; a++) {
        for (uint64_t i = 0; i < p->n; i++) {
            if (p->hash_bits == 128)
                orc_hash_bytes128(p->seed, data + offsets[i], offsets[i + 1] - offsets[i], &h[i], &hs[i]);
            else
                h[i] = orc_hash_bytes(p->seed, data + offsets[i], offsets[i + 1] - offsets[i]);
        }
        orc_build_stats s1;
        memset(&s1, 0, sizeof s1);
        st->attempts = a + 1;
        rc = build_attempt(p, h, hs, same_bytes, &bc, pilots, F, &s1, factor * p->slots_per_part, NULL,
                           (uint32_t)a);
        st->placements += s1.placements;
        st->max_bucket_size = s1.max_bucket_size;
        if (rc != ORC_EPART_FAIL && rc != ORC_EPART_OVERFLOW) {
            st->evictions = s1.evictions;
            st->max_part_evictions = s1.max_part_evictions;
            break;
        }
        rc = ORC_EBUILD_FAILED;
        p->seed++;
    }
    if (hs != h) free(hs);
    free(h);
    return rc;
}
