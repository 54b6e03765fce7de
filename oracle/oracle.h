/*
 * PtrHash CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of what the PtrHash paper
 * (Groot Koerkamp, "PtrHash: Minimal Perfect Hashing at RAM Throughput",
 * SEA 2025, arXiv 2502.15539) defines: parameters, key hash, part/bucket,
 * pilots, slot, hash-evict construction, remap and CacheLineEF. It exists to
 * check the HIP library; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it. It shares no code with the HIP library.
 *
 * Parity pins are in tests/test_oracle_*.py. One function is "parity
 * unpinned" by the paper: orc_hash_bytes (the paper uses GxHash, whose steps
 * it does not give; this oracle defines its own byte-string hash, pinned only
 * by invertibility of its mixer, collision freedom and uniformity tests).
 */
#ifndef PTRHASH_ORACLE_H
#define PTRHASH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* FxHash mixing constant C (Section 3.1, "Hash functions"); any odd value
 * is valid, the paper does not print its value. */
#define ORC_C 0x517cc1b727220a95ULL

enum { ORC_GAMMA_CUBIC = 0, ORC_GAMMA_LINEAR = 1 };
enum { ORC_REMAP_CLEF = 0, ORC_REMAP_PLAIN = 1, ORC_REMAP_NONE = 2 };
/* reduce(x, S): hi(C*x) mod S with S a power of two, or x mod S with S not a
 * power of two and a single part ("The reduce function", Section 3.1). */
enum { ORC_REDUCE_POW2 = 0, ORC_REDUCE_MOD = 1 };

enum {
    ORC_OK = 0,
    ORC_EINVAL = 1,          /* bad arguments */
    ORC_EDUPLICATE = 2,      /* two equal keys */
    ORC_EPART_OVERFLOW = 3,  /* a part holds more than S keys */
    ORC_EBUILD_FAILED = 4,   /* every attempt failed (eviction cap) */
    ORC_ECLEF_RANGE = 5,     /* a CacheLineEF chunk spans too much */
    ORC_ENOMEM = 6,
    ORC_EPART_FAIL = 7       /* internal: one part failed, reseed */
};

typedef struct {
    uint64_t n;                /* number of keys */
    uint64_t num_parts;        /* P */
    uint64_t slots_per_part;   /* S (2^log2_slots unless reduce_kind is MOD) */
    uint32_t log2_slots;
    uint32_t buckets_per_part; /* B */
    uint64_t seed;             /* pilot-hash seed (and byte-hash seed) */
    int32_t gamma;             /* ORC_GAMMA_* */
    int32_t reduce_kind;       /* ORC_REDUCE_* */
    uint64_t remap_len;        /* P*S - n, entries of the remap table F */
    int32_t hash_bits;         /* byte keys: 64, or 128 (high half -> part/bucket, low half -> slot) */
    int32_t pad_;
} orc_params;

typedef struct {
    uint32_t eviction_factor;  /* a part fails after > factor*S evictions (paper: 10) */
    uint32_t max_attempts;     /* reseed attempts before giving up */
} orc_build_cfg;

typedef struct {
    uint64_t attempts;
    uint64_t evictions;        /* total over parts, successful attempt */
    uint64_t max_part_evictions;
    uint64_t placements;       /* bucket placements incl. re-placements */
    uint64_t max_bucket_size;
} orc_build_stats;

/* 128-bit product halves: hi(a*b), lo(a*b) (Section 3.1). */
uint64_t orc_hi(uint64_t a, uint64_t b);
uint64_t orc_lo(uint64_t a, uint64_t b);

/* Parameter rule (Section 3.1, "Parameter values"). */
int orc_params_for(uint64_t n, double alpha, double lambda, int32_t gamma,
                   uint32_t log2_slots_override, uint64_t seed, orc_params *out);
int orc_params_explicit(uint64_t n, uint64_t P, uint32_t log2_slots, uint32_t B,
                        int32_t gamma, uint64_t seed, orc_params *out);
/* One part of S slots (S not a power of two) with reduce(x, S) = x mod S. */
int orc_params_single_mod(uint64_t n, uint64_t S, uint32_t B, int32_t gamma, uint64_t seed, orc_params *out);
/* The rule for a single part with the mod reduce: S = max(ceil(n/alpha), n+16),
 * plus one if that is a power of two; B = ceil(alpha*S/lambda). */
int orc_params_for_single_mod(uint64_t n, double alpha, double lambda, int32_t gamma, uint64_t seed,
                              orc_params *out);

uint64_t orc_hash_u64(uint64_t key);
uint64_t orc_fmix64(uint64_t k);
uint64_t orc_hash_bytes(uint64_t seed, const uint8_t *s, uint64_t len);
/* 128-bit byte-string hash: hi = H(seed), lo = H(seed ^ 0x9E3779B97F4A7C15). */
void orc_hash_bytes128(uint64_t seed, const uint8_t *s, uint64_t len, uint64_t *hi, uint64_t *lo);

uint64_t orc_part(const orc_params *p, uint64_t h);
uint64_t orc_rel(const orc_params *p, uint64_t h);
uint64_t orc_gamma(int32_t kind, uint64_t x);
uint64_t orc_bucket(const orc_params *p, uint64_t h);
uint64_t orc_hp(uint64_t seed, uint32_t pilot);
uint64_t orc_reduce(uint64_t x, uint64_t S);
uint64_t orc_reduce_mod(uint64_t x, uint64_t S);
uint64_t orc_slot(const orc_params *p, uint64_t h, uint32_t pilot);
/* slot with separate hashes for the part and for the reduce (128-bit keys) */
uint64_t orc_slot2(const orc_params *p, uint64_t h_part, uint64_t h_slot, uint32_t pilot);

/* Construction (Section 3.2). pilots: P*B bytes; F: remap_len u64 entries.
 * On success *p may carry a new seed (reseeded after failed attempts). */
int orc_build_u64(orc_params *p, const uint64_t *keys, const orc_build_cfg *cfg,
                  uint8_t *pilots, uint64_t *F, orc_build_stats *st);

/* One record per bucket placement, in the order the search makes them, so
 * that tests can check each decision of the hash-evict search against the
 * rule of Section 3.2 on instances built by hand. Recording only observes:
 * the construction is the same with or without it. */
typedef struct {
    uint64_t part;
    uint32_t bucket;          /* local bucket id within the part */
    uint32_t pilot;           /* pilot chosen */
    uint32_t evicted;         /* buckets this placement evicted */
    uint32_t attempt;         /* seed attempt, from 0 */
    uint64_t part_evictions;  /* evictions in this part so far, this one included */
} orc_trace_rec;

typedef struct {
    orc_trace_rec *rec;
    uint64_t cap;    /* records rec can hold */
    uint64_t len;    /* records written (at most cap) */
    uint64_t total;  /* placements made */
} orc_trace;

int orc_build_u64_traced(orc_params *p, const uint64_t *keys, const orc_build_cfg *cfg,
                         uint8_t *pilots, uint64_t *F, orc_build_stats *st, orc_trace *trace);
int orc_build_bytes(orc_params *p, const uint8_t *data, const uint64_t *offsets,
                    const orc_build_cfg *cfg, uint8_t *pilots, uint64_t *F,
                    orc_build_stats *st);

/* CacheLineEF (Section 3.4). out: ceil(len/44)*64 bytes. */
uint64_t orc_clef_bytes(uint64_t len);
int orc_clef_encode(const uint64_t *F, uint64_t len, uint8_t *out);
uint64_t orc_clef_get(const uint8_t *clef, uint64_t i);
uint32_t orc_select128(uint64_t lo, uint64_t hi, uint32_t r);

/* Queries (eq. partbucket, eq. slot, Section 3.4). remap: CLEF bytes,
 * plain u64 F, or ignored for ORC_REMAP_NONE (non-minimal, returns slot). */
uint64_t orc_query_hash(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                        const void *remap, uint64_t h);
uint64_t orc_query_hash2(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                         const void *remap, uint64_t h_bucket, uint64_t h_slot);
int orc_query_u64(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                  const void *remap, const uint64_t *keys, uint64_t nq, uint64_t *out);
int orc_query_bytes(const orc_params *p, const uint8_t *pilots, int32_t remap_kind,
                    const void *remap, const uint8_t *data, const uint64_t *offsets,
                    uint64_t nq, uint64_t *out);

#ifdef __cplusplus
}
#endif
#endif
