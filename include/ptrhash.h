/*
 * ptrhash.h -- C ABI of the MI355X (gfx950) PtrHash query library.
 *
 * PtrHash (R. Groot Koerkamp, "PtrHash: Minimal Perfect Hashing at RAM
 * Throughput", SEA 2025, arXiv 2502.15539) maps a set of n keys bijectively
 * onto [0, n). A key is hashed (Section 3.1, "Hash functions"), sent to a
 * part and a bucket (eq. partbucket, Section 3.3), the bucket's 8-bit pilot
 * picks a slot (eq. slot), and slots >= n are remapped into the free slots
 * below n through one CacheLineEF table (Section 3.4). This library evaluates
 * that function on large batches of keys with HIP kernels; it also holds a
 * host-side construction (Section 3.2) so that a caller can build the
 * pilots and the remap table it loads.
 *
 * Conventions of every entry point:
 *  - Return value: PTRHASH_OK (0) or a ptrhash_status code; nothing throws
 *    across the ABI. ptrhash_last_error() gives a message for the calling
 *    thread's last failure.
 *  - Pointers documented as "device" are HIP device allocations (for
 *    example torch CUDA tensors); "host" pointers are ordinary memory.
 *    The caller owns every buffer it passes; the library owns only the
 *    device copies it makes in ptrhash_load.
 *  - Queries are asynchronous on the caller's stream: arguments are checked
 *    on the host before the launch; a fault inside a kernel surfaces at the
 *    caller's next synchronisation of that stream.
 *  - Threads: a loaded handle may be queried from several host threads and
 *    streams at once (queries only read it). ptrhash_load, ptrhash_set_kernel,
 *    ptrhash_set_occupancy and ptrhash_destroy change a handle and must not
 *    overlap any other call on it. A multi plan is used by one thread at a
 *    time; ptrhash_query_multi and the server calls other than
 *    ptrhash_server_destroy may be made from any thread.
 */
#ifndef PTRHASH_H
#define PTRHASH_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PTRHASH_API __attribute__((visibility("default")))

typedef enum ptrhash_status {
    PTRHASH_OK = 0,
    PTRHASH_E_INVAL = 1,       /* null pointer, bad size, inconsistent params */
    PTRHASH_E_STATE = 2,       /* handle not loaded, or wrong key kind */
    PTRHASH_E_RANGE = 3,       /* 32-bit output with n > 2^32, size limits */
    PTRHASH_E_NOMEM = 4,       /* device or host allocation failed */
    PTRHASH_E_HIP = 5,         /* a HIP runtime call failed */
    PTRHASH_E_DUPLICATE = 6,   /* construction: two equal keys */
    PTRHASH_E_BUILD = 7,       /* construction: every seed attempt failed */
    PTRHASH_E_REMAP_RANGE = 8  /* construction: a CacheLineEF line overflows */
} ptrhash_status;

/* Bucket assignment function (Section 3.3). */
enum { PTRHASH_GAMMA_CUBIC = 0, PTRHASH_GAMMA_LINEAR = 1 };
/* Remap encoding for slots >= n (Section 3.4): CacheLineEF lines, a plain
 * u32 array, or none (a non-minimal perfect hash that returns the slot). */
enum { PTRHASH_REMAP_CLEF = 0, PTRHASH_REMAP_U32 = 1, PTRHASH_REMAP_NONE = 2 };
/* reduce(x, S) (Section 3.1, "The reduce function"): hi(C*x) mod S with S a
 * power of two, or x mod S with one part whose S is not a power of two. */
enum { PTRHASH_REDUCE_POW2 = 0, PTRHASH_REDUCE_MOD = 1 };
/* Key type: 64-bit integers or byte strings (Section 3.1). */
enum { PTRHASH_KEY_U64 = 0, PTRHASH_KEY_BYTES = 1 };
/* Parameter presets (Section 4.1.2, "Recommended parameters"). Or-ing in
 * PTRHASH_PRESET_SINGLE_MOD switches inputs for which the rule gives a single
 * part to the mod reduce with S = max(ceil(n/alpha), n+16) (plus one if that is
 * a power of two), so small inputs keep a load near alpha. */
enum { PTRHASH_PRESET_DEFAULT = 0, PTRHASH_PRESET_FAST = 1, PTRHASH_PRESET_COMPACT = 2 };
enum { PTRHASH_PRESET_SINGLE_MOD = 0x100 };

/*
 * Parameters of one MPHF. num_parts = P, slots per part S = 2^log2_slots,
 * buckets_per_part = B (Section 3.1). seed enters the pilot hash
 * h_p(p) = C*(p xor seed) and, for byte keys, the string hash.
 * remap_len must equal P*S - n. index_bits (32 or 64) is the width of each
 * output index. With reduce_kind PTRHASH_REDUCE_MOD there is one part of
 * S = slots slots (not a power of two, below 2^32) and log2_slots is unused.
 * Passed by pointer and copied.
 */
typedef struct ptrhash_params {
    uint64_t n;
    uint64_t num_parts;
    uint32_t log2_slots;
    uint32_t buckets_per_part;
    uint64_t seed;
    uint32_t gamma;       /* PTRHASH_GAMMA_* */
    uint32_t remap_kind;  /* PTRHASH_REMAP_* */
    uint64_t remap_len;   /* P*S - n */
    uint32_t key_kind;    /* PTRHASH_KEY_* */
    uint32_t index_bits;  /* 32 or 64 */
    uint32_t reduce_kind; /* PTRHASH_REDUCE_* */
    uint32_t hash_bits;   /* byte keys: 64 (0 means 64) or 128 -- the high half picks part and
                             bucket, the low half the slot; u64 keys: 64 */
    uint64_t slots;       /* S when reduce_kind is PTRHASH_REDUCE_MOD */
} ptrhash_params;

typedef struct ptrhash_handle ptrhash_handle;

/* Create an empty handle (*out). Host only; no device memory yet. */
PTRHASH_API int ptrhash_create(ptrhash_handle **out);

/* Free the handle and its device buffers. NULL is a no-op. The caller must
 * not destroy a handle while queries on it are still running. */
PTRHASH_API int ptrhash_destroy(ptrhash_handle *h);

/*
 * Parameters by the paper's rule (Section 3.1, "Parameter values"):
 * alpha*S >= 80000*ln(n/80000) keys per part (at least 80000), S a power of
 * two, P = ceil(n/(alpha*S)), B = ceil(alpha*S/lambda); a single part
 * shrinks S to the smallest power of two >= n/alpha. Presets: Default
 * (cubic, lambda 3.5, CacheLineEF), Fast (linear, lambda 3.0, u32 remap),
 * Compact (cubic, lambda 4.0, CacheLineEF), alpha = 0.99 for all.
 * index_bits 0 picks 32 when n <= 2^32, else 64. Byte keys get 128-bit
 * hashing when n > 2^32 (Section 3.1, "Hash functions"), else 64-bit.
 */
PTRHASH_API int ptrhash_params_default(uint64_t n, int preset, uint32_t key_kind, uint32_t index_bits,
                                       uint64_t seed, ptrhash_params *out);

/* Bytes of the remap table for these params: CacheLineEF
 * ceil(remap_len/44)*64, u32 4*remap_len, none 0. */
PTRHASH_API uint64_t ptrhash_remap_bytes(const ptrhash_params *params);

/*
 * Copy an MPHF into handle-owned device memory: pilots (host, P*B bytes,
 * indexed by global bucket part*B + bucket) and remap (host,
 * ptrhash_remap_bytes(params) bytes; may be NULL when that is 0). Remap
 * layout, CacheLineEF: one 64-byte line per 44 entries; bytes [0,4) the
 * 32-bit offset, [4,20) the 128-bit high-part bitmap as two little-endian
 * u64 words, [20,64) the 44 low bytes (Section 3.4, eq. clef). Synchronous.
 * A reload replaces the previous MPHF. Errors: E_INVAL (null pointer, S not
 * a power of two, P*S < n, B == 0, remap_len != P*S - n, bad enum),
 * E_RANGE (index_bits 32 with n > 2^32, P*B or P*S >= 2^40), E_NOMEM, E_HIP.
 */
PTRHASH_API int ptrhash_load(ptrhash_handle *h, const uint8_t *pilots, const void *remap,
                             const ptrhash_params *params);

/* The parameters of the loaded MPHF (E_STATE if none). */
PTRHASH_API int ptrhash_get_params(const ptrhash_handle *h, ptrhash_params *out);

/*
 * Evaluate the MPHF on n_q u64 keys: out[i] = H(keys[i]) (eq. partbucket,
 * eq. slot, remap of Section 3.4). keys: device, n_q u64. out: device, n_q
 * elements of index_bits. Members map bijectively onto [0, n); any other key
 * gets a deterministic value in [0, n) (minimal remaps) or [0, P*S) (no
 * remap). Asynchronous on stream; keys/out must stay valid until it
 * completes. n_q == 0 launches nothing. Any n_q is taken: batches beyond
 * 2^31 work-items are split into several launches on the same stream.
 * Errors: E_STATE (not loaded, or a byte-key MPHF), E_INVAL (null, or the
 * byte ranges of keys and out overlap), E_HIP.
 */
PTRHASH_API int ptrhash_query(ptrhash_handle *h, const uint64_t *keys, uint64_t n_q, void *out,
                              hipStream_t stream);

/*
 * As ptrhash_query for byte-string keys (Section 3.1, "Hash functions"):
 * key i is data[offsets[i] .. offsets[i+1]). data: device, 8-byte aligned,
 * data_len bytes, which must include at least 64 readable bytes after
 * offsets[n_q]; offsets: device, n_q+1 u64, non-decreasing. The offsets
 * live on the device, so they are checked by the kernel: a key whose end
 * precedes its start, or which ends later than data_len - 16, is not read
 * and gets an index of all ones (no valid index, unless n = 2^index_bits).
 * Errors: E_STATE (not loaded, or a u64-key MPHF), E_INVAL (null, data not
 * aligned, data_len < 64, or out overlapping data or offsets), E_HIP.
 */
PTRHASH_API int ptrhash_query_bytes(ptrhash_handle *h, const uint8_t *data, uint64_t data_len,
                                    const uint64_t *offsets, uint64_t n_q, void *out, hipStream_t stream);

/* ---- Many MPHFs in one launch (row A8) ---- */

/* One query batch against one loaded MPHF. For a u64-key handle set keys;
 * for a byte-key handle set data (8-byte aligned, data_len bytes with 64
 * bytes of readable padding after the last string, as in
 * ptrhash_query_bytes) and offsets (n_q+1 entries). out holds n_q indices of
 * the handle's index_bits. All pointers are device pointers. No batch's out
 * may overlap its own or another batch's out, keys, data or offsets. */
typedef struct ptrhash_query_desc {
    ptrhash_handle *handle;
    const uint64_t *keys;
    const uint8_t *data;
    uint64_t data_len;
    const uint64_t *offsets;
    uint64_t n_q;
    void *out;
} ptrhash_query_desc;

/*
 * A reusable launch plan: a device table of up to max_descs batches and a
 * pinned, mapped host staging copy of it. plan_set validates the batches
 * and writes the staging copy (host only). plan_launch enqueues on stream
 * a small kernel that copies the staging table into the device table (on
 * the stream itself, with no copy-engine hand-off), followed by one
 * persistent kernel that strides over the tiles of every batch; the
 * result of each batch equals a separate ptrhash_query/ptrhash_query_bytes
 * call. plan_launch may be captured into a HIP graph: when the stream is
 * capturing it copies the whole table, so each replay runs the batches the
 * latest plan_set wrote. The caller must not call plan_set while an
 * earlier launch of the same plan may still be copying its staging table
 * (synchronise the stream, or an event recorded after the launch, first).
 * Errors: E_INVAL (bad descriptor or count), E_STATE (handle not loaded or
 * wrong key kind), E_RANGE (k > max_descs), E_NOMEM, E_HIP.
 */
typedef struct ptrhash_multi_plan ptrhash_multi_plan;
PTRHASH_API int ptrhash_multi_plan_create(int max_descs, ptrhash_multi_plan **out);
PTRHASH_API int ptrhash_multi_plan_destroy(ptrhash_multi_plan *plan);
PTRHASH_API int ptrhash_multi_plan_set(ptrhash_multi_plan *plan, const ptrhash_query_desc *descs, int k);
PTRHASH_API int ptrhash_multi_plan_launch(ptrhash_multi_plan *plan, hipStream_t stream);

/*
 * Launch shape of a plan's persistent kernel: keys_per_lane (loads in
 * flight per lane: 1, 2, 4 or 8), block (threads per workgroup, 64..1024,
 * a multiple of 64) and blocks_per_cu (resident workgroups per compute
 * unit; 0 = as many as the kernel allows), so that the autotuner can pick
 * them. A batch is cut into tiles of keys_per_lane * block keys, so the
 * batches must be set again (ptrhash_multi_plan_set) after a change before
 * the next launch (E_STATE otherwise); a captured graph keeps the shape it
 * was captured with. New plans take the process default
 * (ptrhash_set_multi_kernel; initially 4, 256, 0), which ptrhash_query_multi
 * also uses. Errors: E_INVAL.
 */
PTRHASH_API int ptrhash_multi_plan_set_kernel(ptrhash_multi_plan *plan, int keys_per_lane, int block,
                                              int blocks_per_cu);
PTRHASH_API int ptrhash_set_multi_kernel(int keys_per_lane, int block, int blocks_per_cu);

/*
 * Evaluate k batches (descs: host array, copied before return) in one
 * persistent launch on stream, through an internal ring of plans whose
 * reuse waits for the launch that last used the slot. Not for use while
 * the stream is being captured (E_STATE): capture a plan instead.
 * k == 0 launches nothing. k is limited to ptrhash_multi_max().
 */
PTRHASH_API int ptrhash_query_multi(const ptrhash_query_desc *descs, int k, hipStream_t stream);
PTRHASH_API int ptrhash_multi_max(void);

/*
 * For callers that cannot allocate (tight serving loops, harnesses that
 * forbid hipMalloc): as ptrhash_query_multi, with results identical to it,
 * but nothing is allocated on the device or the host. The batch table goes
 * into a fixed device array of the library (about 35 KB on each GPU it runs
 * on, held until the process ends) through a fixed host array, copied on
 * stream ahead of the launch (a copy from pageable memory, which returns
 * once the table has left the host array). At most 256 batches per call
 * (E_RANGE beyond). Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU, on different streams or from different threads,
 * race; calls one after the other on one stream do not. Not for use while
 * the stream is being captured (E_STATE). Other errors as
 * ptrhash_query_multi.
 */
PTRHASH_API int ptrhash_query_multi_noalloc(const ptrhash_query_desc *descs, int k, hipStream_t stream);

/* ---- Serving: continuous batching over resident MPHFs (row A8) ---- */

/* streams: launch slots in flight at once (1..16; a process gets
 * GPU_MAX_HW_QUEUES hardware queues, 4 by default, and streams beyond that
 * share them, so more than 4 slots add queueing, not concurrency); max_batches: requests per
 * launch (1..ptrhash_multi_max()); slot_keys: keys one launch can hold (its
 * device arena; also the largest request); max_queued_keys: admission limit
 * of keys waiting for a slot (submit returns E_RANGE beyond it);
 * copy_threads: extra host threads for the copies into and out of the
 * pinned staging buffers; zero_copy: see the field. */
typedef struct ptrhash_server_config {
    int streams;
    int max_batches;
    uint64_t slot_keys;
    uint64_t max_queued_keys;
    int copy_threads;     /* host threads helping with key/index copies (0..64) */
    int zero_copy;        /* 1: kernels read keys and write indices in mapped host memory;
                             0: keys and indices are copied to/from device arenas */
    int keys_per_lane;    /* launch shape of the multi-MPHF kernel, as in */
    int block;            /* ptrhash_multi_plan_set_kernel; keys_per_lane = 0 */
    int blocks_per_cu;    /* takes the process default for all three */
} ptrhash_server_config;

typedef struct ptrhash_server_metrics {
    uint64_t completed;   /* requests finished since the last reset */
    uint64_t launches;    /* multi-MPHF launches */
    uint64_t keys;        /* keys answered */
    uint64_t queued;      /* requests waiting for a slot now */
    double p50_us, p99_us, max_us;  /* submit -> indices delivered, over the most recent
                                       2^20 requests completed since the last reset */
    double wait_p50_us, wait_p99_us; /* submit -> launch enqueued (queueing + copy-in), same window */
    uint64_t slots_busy_max; /* most launch slots busy at once since the last reset (launched, not retired) */
    uint64_t overlap_max;    /* most launches running at once on the device, from each launch's start and
                                done events (timing events on its stream), over the most recent 2^16 */
    double overlap_mean;     /* mean number of launches running over the time at least one runs, same window */
} ptrhash_server_metrics;

/* One request of a replayed arrival schedule (host keys and output). */
typedef struct ptrhash_server_request {
    ptrhash_handle *handle;
    const uint64_t *keys;
    uint64_t n_q;
    void *out;
    double arrival_us;    /* offset from the start of the replay */
    uint32_t mapped;      /* 1: keys/out in ptrhash_host_alloc memory (as ptrhash_server_submit_mapped) */
    uint32_t pad_;
} ptrhash_server_request;

/*
 * A server owns `streams` launch slots (device arena, pinned staging, a
 * multi-MPHF plan and a stream each) and a dispatcher thread. Requests are
 * host arrays of u64 keys against a loaded u64-key handle; indices are
 * written to the caller's host buffer (index_bits of that handle). Whenever
 * a slot is free, queued requests are admitted in arrival order while they
 * fit its arena and batch count, and run as one launch; slots overlap on the
 * device, so requests arriving while others run join the next launch. Each
 * request's result is the same as a lone ptrhash_query of its keys. Keys and
 * out must stay valid until the request is waited for; every ticket is waited
 * for at most once. Handles must outlive the requests that use them.
 * submit: E_RANGE when the request exceeds slot_keys or the queue is full.
 * wait: blocks until the request is delivered; latency_us may be NULL.
 * replay: submits reqs at their arrival times (open loop, retrying while the
 * queue is full), waits for all, and reports the makespan.
 * destroy drains the queue, then frees everything.
 */
typedef struct ptrhash_server ptrhash_server;
PTRHASH_API int ptrhash_server_default_config(ptrhash_server_config *cfg);
PTRHASH_API int ptrhash_server_create(const ptrhash_server_config *cfg, ptrhash_server **out);
PTRHASH_API int ptrhash_server_submit(ptrhash_server *srv, ptrhash_handle *h, const uint64_t *keys, uint64_t n_q,
                                      void *out, uint64_t *ticket);
PTRHASH_API int ptrhash_server_wait(ptrhash_server *srv, uint64_t ticket, double *latency_us);

/*
 * Mapped requests: keys and out lie inside memory from ptrhash_host_alloc
 * (mapped, coherent, pinned host memory), so the multi-MPHF kernel reads
 * the keys and writes the indices there in place, over PCIe, with no host
 * copy on either side; otherwise as ptrhash_server_submit (the request
 * still counts against slot_keys). E_INVAL if a buffer is not inside one
 * such allocation. ptrhash_host_free releases an allocation; no request
 * may still use it. Errors of host_alloc: E_INVAL, E_NOMEM, E_HIP.
 */
PTRHASH_API int ptrhash_server_submit_mapped(ptrhash_server *srv, ptrhash_handle *h, const uint64_t *keys,
                                             uint64_t n_q, void *out, uint64_t *ticket);
PTRHASH_API int ptrhash_host_alloc(uint64_t bytes, void **out);
PTRHASH_API int ptrhash_host_free(void *p);
PTRHASH_API int ptrhash_server_replay(ptrhash_server *srv, const ptrhash_server_request *reqs, uint64_t count,
                                      double *makespan_s);
PTRHASH_API int ptrhash_server_stats(ptrhash_server *srv, ptrhash_server_metrics *out);
PTRHASH_API int ptrhash_server_reset_stats(ptrhash_server *srv);
PTRHASH_API int ptrhash_server_destroy(ptrhash_server *srv);

/* Kernel choice for a handle's queries: kernel 0 = one key per lane,
 * 1 = keys_per_lane keys per lane with every pilot load issued before the
 * first is used; block = threads per workgroup (64..1024, multiple of 64).
 * keys_per_lane in {1, 2, 4, 8, 16}. Errors: E_INVAL. */
enum { PTRHASH_KERNEL_PLAIN = 0, PTRHASH_KERNEL_PIPELINED = 1 };
PTRHASH_API int ptrhash_set_kernel(ptrhash_handle *h, int kernel, int keys_per_lane, int block);

/* Occupancy cap for a handle's queries: reserve LDS so that at most
 * blocks_per_cu workgroups of the query kernel are resident on a compute
 * unit (0 = no cap). *effective (may be NULL) receives the cap the device's
 * LDS limits allow. Used by the autotuner together with keys_per_lane (loads
 * in flight per lane) and block. Errors: E_INVAL, E_HIP. */
PTRHASH_API int ptrhash_set_occupancy(ptrhash_handle *h, int blocks_per_cu, int *effective);

/* Message of the calling thread's last failure ("" if none). */
PTRHASH_API const char *ptrhash_last_error(void);

/* ---- Construction (host; Section 3.2, Section 3.4) ---- */

typedef struct ptrhash_build_info {
    uint64_t attempts;        /* seeds tried */
    uint64_t evictions;       /* total over parts, final attempt */
    uint64_t max_part_evictions;
    uint64_t max_bucket_size;
} ptrhash_build_info;

/*
 * Build an MPHF on n distinct u64 keys (host memory) with hash-evict pilot
 * search: buckets largest first, the smallest free pilot in [0, 256), else
 * evict the buckets of the pilot with the least sum of squared sizes of
 * colliding buckets, never one of the 16 most recently placed; a part fails
 * after 10*S evictions and the whole build retries with seed+1 (at most 16
 * seeds). params: in/out (a retry stores the seed used). pilots: host,
 * P*B bytes. remap: host, ptrhash_remap_bytes(params) bytes. threads: worker
 * threads (0 = all cores). info may be NULL. Errors: E_INVAL, E_DUPLICATE,
 * E_BUILD (a part over S keys, or all seeds failed), E_REMAP_RANGE, E_NOMEM.
 */
PTRHASH_API int ptrhash_build_u64(const uint64_t *keys, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                                  void *remap, int threads, ptrhash_build_info *info);

/* As ptrhash_build_u64 with the keys in device memory: the hashes are
 * computed and radix-sorted on the device (sorted hashes come grouped by part
 * and bucket), copied to the host, and the pilot search runs on host threads.
 * Same result as ptrhash_build_u64 on the same keys. Needs 16*n bytes of
 * device memory plus the sort's scratch for the duration of the call; stream
 * orders the device work and is synchronised before return. */
PTRHASH_API int ptrhash_build_u64_device(const uint64_t *keys, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                                         void *remap, int threads, ptrhash_build_info *info, hipStream_t stream);

/* As ptrhash_build_u64 with the keys in device memory and the whole pilot
 * search on the device too (Section 3.2 "Construction"): the hashes are
 * radix-sorted, bucket boundaries and a per-part (size descending, bucket
 * id) order are built on the device, and one workgroup per part runs the
 * hash-evict search: one wavefront places the buckets with the part's
 * taken-slot bitvector in LDS while look-ahead wavefronts find the smallest
 * free pilot of the buckets it will take next (PTRHASH_SEARCH_HELPERS = 0, 1,
 * 2, 3, 6 or 7 sets their number; 7 by default). The result is the same as
 * ptrhash_build_u64 on the same keys, byte for byte, whatever that number;
 * the remap table is built on the device too, from the taken-slot bitvector.
 * Limits: the S bits of a part must fit one workgroup's LDS (S <= 2^20 on
 * gfx950), S a multiple of 32 when P > 1, buckets of at most 2048 keys;
 * outside them the call returns E_RANGE and ptrhash_build_u64_device
 * (host search) applies. Device memory: about 16*n + 33*P*B + 5*P*S/8 +
 * 20*(P*S - n) bytes plus 16*S bytes per compute unit, for the duration of
 * the call. A seed whose search runs three times longer than a normal one
 * would (a part caught in an eviction cycle) has the next three seeds
 * searched beside it on streams of the library's own, each with another
 * P*B + P*S/8 + 16*S per compute unit of device memory when that much is
 * free; seeds are still taken in order, so the result does not change
 * (PTRHASH_SPECULATE_MS sets the threshold in ms). stream orders the device
 * work and is synchronised before return. Errors: E_INVAL, E_DUPLICATE,
 * E_BUILD (a part with more than S keys, or 16 failed seeds), E_RANGE,
 * E_NOMEM, E_HIP. */
PTRHASH_API int ptrhash_build_u64_gpu(const uint64_t *keys, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                                      void *remap, ptrhash_build_info *info, hipStream_t stream);

/* As ptrhash_build_u64_gpu for byte strings in device memory: key i =
 * data[offsets[i] .. offsets[i+1]), data 8-byte aligned, data_len bytes with
 * at least 64 readable bytes after the last string (the layout the query
 * takes). The offsets are checked on the device before any string is read:
 * decreasing offsets, or a string ending later than data_len - 16, give
 * E_INVAL. The
 * string hash depends on the seed, so every attempt hashes and sorts again;
 * equal hashes of distinct strings cause a reseed, equal strings E_DUPLICATE,
 * like ptrhash_build_bytes (same result, byte for byte). With 128-bit
 * hashes (hash_bits = 128) keys are sorted by the high half, which picks
 * part and bucket, and the slots come from the low half; only keys equal in
 * both halves collide. E_RANGE when more than 64 pairs of keys share a hash
 * (the host construction examines them all) or, with 128-bit hashes, three
 * keys share a high half. Device memory: about 32*n (48*n with 128-bit
 * hashes) + 33*P*B + 5*P*S/8 + 20*(P*S - n) bytes plus 16*S bytes per
 * compute unit. Seeds
 * are searched one after the other. */
PTRHASH_API int ptrhash_build_bytes_gpu(const uint8_t *data, uint64_t data_len, const uint64_t *offsets, uint64_t n,
                                        ptrhash_params *params, uint8_t *pilots, void *remap,
                                        ptrhash_build_info *info, hipStream_t stream);

/* As ptrhash_build_u64 for byte strings data[offsets[i] .. offsets[i+1])
 * (host memory, data_len bytes; offsets non-decreasing and at most data_len,
 * else E_INVAL before any string is read); equal 64-bit hashes of distinct
 * strings cause a reseed. */
PTRHASH_API int ptrhash_build_bytes(const uint8_t *data, uint64_t data_len, const uint64_t *offsets, uint64_t n,
                                    ptrhash_params *params, uint8_t *pilots, void *remap, int threads,
                                    ptrhash_build_info *info);

/* ---- Roofline microbenchmarks (device; the denominators of the metric) ----
 * gather: out[i] = keys[i] xor table[hi(keys[i] * table_len)] -- stream a
 * key in, one random byte from a table_len-byte table, stream a u64 out;
 * the memory pattern of a query without its arithmetic. copy: out[i] =
 * keys[i]. Both asynchronous on stream; keys_per_lane/block as in
 * ptrhash_set_kernel; blocks_per_cu as in ptrhash_set_occupancy (0 = no cap),
 * so the gather is tuned over the same knobs as the query. */
PTRHASH_API int ptrhash_bench_gather(const uint64_t *keys, uint64_t n_q, const uint8_t *table,
                                     uint64_t table_len, uint64_t *out, int keys_per_lane, int block,
                                     int blocks_per_cu, hipStream_t stream);
/* pure gather: n random byte reads table[hi(mix(i) * table_len)] with no key
 * or index streams (mix = the SplitMix64 output mixer), spread over `lanes`
 * threads (a multiple of 256); sink receives one u32 sum per lane. */
PTRHASH_API int ptrhash_bench_gather_pure(uint64_t n, const uint8_t *table, uint64_t table_len, uint32_t *sink,
                                          uint32_t lanes, hipStream_t stream);
/* line-size probe: as the pure gather, and each random offset o also reads
 * the byte at o ^ xor_dist (32: same 64-byte half, 64: other half of the
 * same 128-byte line, 128: the next line). table_len a positive multiple of
 * 256; xor_dist 32, 64 or 128, else E_INVAL. */
PTRHASH_API int ptrhash_bench_gather_pair(uint64_t n, const uint8_t *table, uint64_t table_len, uint32_t *sink,
                                          uint32_t lanes, uint32_t xor_dist, hipStream_t stream);
PTRHASH_API int ptrhash_bench_copy(const uint64_t *keys, uint64_t n_q, uint64_t *out, int keys_per_lane,
                                   int block, hipStream_t stream);
/* like-for-like gather of a loaded u64-key MPHF: out[i] = keys[i] xor
 * pilots[bucket(keys[i])], the query's own hash, part and global bucket
 * (eq. partbucket) without the slot hash and the remap, so the gathers hit
 * the caches as the query's do (keys/out: device, n_q u64). */
PTRHASH_API int ptrhash_bench_gather_buckets(ptrhash_handle *h, const uint64_t *keys, uint64_t n_q, uint64_t *out,
                                             int keys_per_lane, int block, int blocks_per_cu, hipStream_t stream);
/* string-stream gather of a loaded MPHF: for each key of (data, data_len,
 * offsets) as in ptrhash_query_bytes, read its offsets and the aligned words
 * of its bytes, fold them by xor, mix once, read the pilot of the bucket
 * that value maps to, and stream a u32 out (the memory pattern of a byte-key
 * query without the string hash's arithmetic). */
PTRHASH_API int ptrhash_bench_gather_bytes(ptrhash_handle *h, const uint8_t *data, uint64_t data_len,
                                           const uint64_t *offsets, uint64_t n_q, uint32_t *out, int keys_per_lane,
                                           int block, int blocks_per_cu, hipStream_t stream);
/* un-permute probe: out[(i * A) mod 2^log2_n] = in[i] for every i < 2^log2_n
 * (A odd, so every slot of out is written once): one streamed read and one
 * random 8-byte write per element. in/out: device, 2^log2_n u64 each,
 * log2_n in [8, 34]. */
PTRHASH_API int ptrhash_bench_scatter(const uint64_t *in, uint32_t log2_n, uint64_t *out, hipStream_t stream);

/* ---- Synthetic inputs (device; for benchmarks and tests) ----
 * Key i of a key set = SplitMix64 output i of the stream seeded seed
 * (distinct for distinct i). gen_u64_keys writes keys start..start+count-1.
 * gen_query_stream writes members of the n-key set in a seeded shuffled
 * order: entry i is key pi(i), pi a 4-round Feistel bijection of [0, n) with
 * cycle walking keyed by order_seed. Asynchronous on stream. */
PTRHASH_API int ptrhash_gen_u64_keys(uint64_t seed, uint64_t start, uint64_t count, uint64_t *out,
                                     hipStream_t stream);
PTRHASH_API int ptrhash_gen_query_stream(uint64_t n, uint64_t key_seed, uint64_t order_seed, uint64_t start,
                                         uint64_t count, uint64_t *out, hipStream_t stream);
/* Random strings of a set of n: string s has length 10 + (r mod 41) and
 * byte j = 0x20 + ((r_j & 0xff) mod 95), r and r_j SplitMix64 outputs of
 * (seed, s) and (seed ^ 0x2545F4914F6CDD1D, 64 s + j). Entry i of the
 * generated range is string i (shuffled == 0) or string pi(i) (shuffled,
 * the Feistel order of gen_query_stream). lengths: count u64 lengths of
 * entries start..; bytes: writes entry start+i at data + offsets[i], with
 * offsets (count+1 entries) the caller's running sum of those lengths. */
PTRHASH_API int ptrhash_gen_string_lengths(uint64_t n, uint64_t seed, uint64_t order_seed, int shuffled,
                                           uint64_t start, uint64_t count, uint64_t *lengths, hipStream_t stream);
PTRHASH_API int ptrhash_gen_string_bytes(uint64_t n, uint64_t seed, uint64_t order_seed, int shuffled,
                                         uint64_t start, uint64_t count, const uint64_t *offsets, uint8_t *data,
                                         hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
