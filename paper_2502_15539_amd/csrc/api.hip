// C ABI of the query library: handles, parameter rule, validation, device
// residency of an MPHF and kernel dispatch. All compute happens in the HIP
// kernels; this layer only checks arguments and launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"
#include "ptrhash.h"

using namespace ptrhash;

struct ptrhash_handle {
    ptrhash_params params{};
    bool loaded = false;
    uint8_t *d_pilots = nullptr;
    uint8_t *d_remap = nullptr;
    Tuning tuning{};
};

namespace {

thread_local char g_err[512] = "";

}  // namespace

namespace ptrhash {
int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}
}  // namespace ptrhash

namespace {

#define fail ptrhash::set_error

int hip_fail(hipError_t e, const char *what) {
    return fail(PTRHASH_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

uint64_t next_pow2(uint64_t v) {
    uint64_t r = 1;
    while (r < v) r <<= 1;
    return r;
}

uint32_t log2_of(uint64_t pow2) {
    uint32_t l = 0;
    while ((1ull << l) < pow2) ++l;
    return l;
}

void free_device(ptrhash_handle *h) {
    if (h->d_pilots) (void)hipFree(h->d_pilots);
    if (h->d_remap) (void)hipFree(h->d_remap);
    h->d_pilots = h->d_remap = nullptr;
    h->loaded = false;
}

DevMphf device_view(const ptrhash_handle *h) {
    DevMphf m{};
    m.pilots = h->d_pilots;
    m.remap = h->d_remap;
    m.n = h->params.n;
    m.seed = h->params.seed;
    m.parts = (uint32_t)h->params.num_parts;
    m.buckets = h->params.buckets_per_part;
    m.log2_slots = h->params.log2_slots;
    m.gamma = h->params.gamma;
    m.remap_kind = h->params.remap_kind;
    return m;
}

constexpr uint64_t kMaxIndexSpace = 1ull << 40;  // CacheLineEF values are 40-bit

int check_params(const ptrhash_params *p) {
    if (!p) return fail(PTRHASH_E_INVAL, "params is NULL");
    if (p->n == 0) return fail(PTRHASH_E_INVAL, "n must be positive");
    if (p->num_parts == 0 || p->num_parts > 0xffffffffull)
        return fail(PTRHASH_E_INVAL, "num_parts must be in [1, 2^32)");
    if (p->buckets_per_part == 0) return fail(PTRHASH_E_INVAL, "buckets_per_part must be positive");
    if (p->log2_slots > 40) return fail(PTRHASH_E_RANGE, "log2_slots %u > 40", p->log2_slots);
    const uint64_t S = 1ull << p->log2_slots;
    if (p->num_parts > kMaxIndexSpace / S) return fail(PTRHASH_E_RANGE, "P*S >= 2^40");
    if (p->num_parts * (uint64_t)p->buckets_per_part > kMaxIndexSpace) return fail(PTRHASH_E_RANGE, "P*B > 2^40");
    if (p->num_parts * S < p->n) return fail(PTRHASH_E_INVAL, "P*S < n");
    if (p->remap_len != p->num_parts * S - p->n)
        return fail(PTRHASH_E_INVAL, "remap_len %llu != P*S - n = %llu", (unsigned long long)p->remap_len,
                    (unsigned long long)(p->num_parts * S - p->n));
    if (p->gamma > PTRHASH_GAMMA_LINEAR) return fail(PTRHASH_E_INVAL, "unknown gamma %u", p->gamma);
    if (p->remap_kind > PTRHASH_REMAP_NONE) return fail(PTRHASH_E_INVAL, "unknown remap_kind %u", p->remap_kind);
    if (p->key_kind > PTRHASH_KEY_BYTES) return fail(PTRHASH_E_INVAL, "unknown key_kind %u", p->key_kind);
    if (p->index_bits != 32 && p->index_bits != 64) return fail(PTRHASH_E_INVAL, "index_bits must be 32 or 64");
    const uint64_t max_out = p->remap_kind == PTRHASH_REMAP_NONE ? p->num_parts * S : p->n;
    if (p->index_bits == 32 && max_out > (1ull << 32))
        return fail(PTRHASH_E_RANGE, "32-bit indices cannot hold values up to %llu", (unsigned long long)max_out);
    if (p->remap_kind == PTRHASH_REMAP_U32 && p->n > (1ull << 32))
        return fail(PTRHASH_E_RANGE, "u32 remap needs n <= 2^32");
    return PTRHASH_OK;
}

}  // namespace

namespace ptrhash {
bool valid_tuning(int kernel, int keys_per_lane, int block) {
    if (kernel != kKernelPlain && kernel != kKernelPipelined) return false;
    if (block < 64 || block > 1024 || block % 64) return false;
    return keys_per_lane == 1 || keys_per_lane == 2 || keys_per_lane == 4 || keys_per_lane == 8 ||
           keys_per_lane == 16;
}
}  // namespace ptrhash

extern "C" {

PTRHASH_API const char *ptrhash_last_error(void) { return g_err; }

PTRHASH_API int ptrhash_create(ptrhash_handle **out) {
    if (!out) return fail(PTRHASH_E_INVAL, "out is NULL");
    *out = new (std::nothrow) ptrhash_handle();
    if (!*out) return fail(PTRHASH_E_NOMEM, "handle allocation failed");
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_destroy(ptrhash_handle *h) {
    if (!h) return PTRHASH_OK;
    free_device(h);
    delete h;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_params_default(uint64_t n, int preset, uint32_t key_kind, uint32_t index_bits,
                                       uint64_t seed, ptrhash_params *out) {
    if (!out) return fail(PTRHASH_E_INVAL, "out is NULL");
    if (n == 0) return fail(PTRHASH_E_INVAL, "n must be positive");
    if (key_kind > PTRHASH_KEY_BYTES) return fail(PTRHASH_E_INVAL, "unknown key_kind %u", key_kind);
    const double alpha = 0.99;
    double lambda;
    uint32_t gamma, remap;
    switch (preset) {
    case PTRHASH_PRESET_DEFAULT: lambda = 3.5; gamma = PTRHASH_GAMMA_CUBIC; remap = PTRHASH_REMAP_CLEF; break;
    case PTRHASH_PRESET_FAST: lambda = 3.0; gamma = PTRHASH_GAMMA_LINEAR; remap = PTRHASH_REMAP_U32; break;
    case PTRHASH_PRESET_COMPACT: lambda = 4.0; gamma = PTRHASH_GAMMA_CUBIC; remap = PTRHASH_REMAP_CLEF; break;
    default: return fail(PTRHASH_E_INVAL, "unknown preset %d", preset);
    }
    // alpha*S >= 80000*ln(n/80000) keys per part, at least 80000.
    double keys_per_part = 80000.0 * std::log((double)n / 80000.0);
    if (keys_per_part < 80000.0) keys_per_part = 80000.0;
    uint64_t S = next_pow2((uint64_t)std::ceil(keys_per_part / alpha));
    uint64_t P = (uint64_t)std::ceil((double)n / (alpha * (double)S));
    if (P < 1) P = 1;
    if (P == 1) S = next_pow2((uint64_t)std::ceil((double)n / alpha));
    uint64_t B = (uint64_t)std::ceil(alpha * (double)S / lambda);
    if (B < 1) B = 1;
    if (B > 0xffffffffull) return fail(PTRHASH_E_RANGE, "too many buckets per part");
    ptrhash_params p{};
    p.n = n;
    p.num_parts = P;
    p.log2_slots = log2_of(S);
    p.buckets_per_part = (uint32_t)B;
    p.seed = seed;
    p.gamma = gamma;
    p.remap_kind = remap;
    p.remap_len = P * S - n;
    p.key_kind = key_kind;
    p.index_bits = index_bits ? index_bits : (n <= (1ull << 32) ? 32u : 64u);
    const int rc = check_params(&p);
    if (rc) return rc;
    *out = p;
    return PTRHASH_OK;
}

PTRHASH_API uint64_t ptrhash_remap_bytes(const ptrhash_params *p) {
    if (!p) return 0;
    switch (p->remap_kind) {
    case PTRHASH_REMAP_CLEF: return (p->remap_len + 43) / 44 * 64;
    case PTRHASH_REMAP_U32: return p->remap_len * 4;
    default: return 0;
    }
}

PTRHASH_API int ptrhash_load(ptrhash_handle *h, const uint8_t *pilots, const void *remap,
                             const ptrhash_params *params) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    int rc = check_params(params);
    if (rc) return rc;
    if (!pilots) return fail(PTRHASH_E_INVAL, "pilots is NULL");
    const uint64_t pbytes = params->num_parts * (uint64_t)params->buckets_per_part;
    const uint64_t rbytes = ptrhash_remap_bytes(params);
    if (rbytes && !remap) return fail(PTRHASH_E_INVAL, "remap is NULL but %llu bytes are needed",
                                      (unsigned long long)rbytes);
    free_device(h);
    hipError_t e = hipMalloc(&h->d_pilots, pbytes);
    if (e != hipSuccess) {
        h->d_pilots = nullptr;
        return fail(PTRHASH_E_NOMEM, "hipMalloc(%llu) for pilots: %s", (unsigned long long)pbytes,
                    hipGetErrorString(e));
    }
    if (rbytes) {
        e = hipMalloc(&h->d_remap, rbytes);
        if (e != hipSuccess) {
            h->d_remap = nullptr;
            free_device(h);
            return fail(PTRHASH_E_NOMEM, "hipMalloc(%llu) for remap: %s", (unsigned long long)rbytes,
                        hipGetErrorString(e));
        }
    }
    e = hipMemcpy(h->d_pilots, pilots, pbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && rbytes) e = hipMemcpy(h->d_remap, remap, rbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_device(h);
        return hip_fail(e, "hipMemcpy to device");
    }
    h->params = *params;
    h->loaded = true;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_get_params(const ptrhash_handle *h, ptrhash_params *out) {
    if (!h || !out) return fail(PTRHASH_E_INVAL, "NULL argument");
    if (!h->loaded) return fail(PTRHASH_E_STATE, "handle has no MPHF loaded");
    *out = h->params;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_set_kernel(ptrhash_handle *h, int kernel, int keys_per_lane, int block) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    if (!valid_tuning(kernel, keys_per_lane, block))
        return fail(PTRHASH_E_INVAL, "bad kernel choice (%d, %d, %d)", kernel, keys_per_lane, block);
    h->tuning.kernel = kernel;
    h->tuning.keys_per_lane = keys_per_lane;
    h->tuning.block = block;
    return PTRHASH_OK;
}

static int check_grid(uint64_t n_q, const Tuning &t) {
    const uint64_t per_block = (uint64_t)t.block * (t.kernel == kKernelPlain ? 1 : t.keys_per_lane);
    if ((n_q + per_block - 1) / per_block > 0x7fffffffull)
        return fail(PTRHASH_E_RANGE, "n_q %llu too large for one launch", (unsigned long long)n_q);
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_query(ptrhash_handle *h, const uint64_t *keys, uint64_t n_q, void *out,
                              hipStream_t stream) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    if (!h->loaded) return fail(PTRHASH_E_STATE, "handle has no MPHF loaded");
    if (h->params.key_kind != PTRHASH_KEY_U64) return fail(PTRHASH_E_STATE, "MPHF is for byte keys");
    if (n_q == 0) return PTRHASH_OK;
    if (!keys || !out) return fail(PTRHASH_E_INVAL, "keys/out is NULL");
    const int rc = check_grid(n_q, h->tuning);
    if (rc) return rc;
    const hipError_t e =
        launch_query_u64(device_view(h), keys, n_q, out, h->params.index_bits == 64, h->tuning, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "query launch");
}

PTRHASH_API int ptrhash_query_bytes(ptrhash_handle *h, const uint8_t *data, const uint64_t *offsets,
                                    uint64_t n_q, void *out, hipStream_t stream) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    if (!h->loaded) return fail(PTRHASH_E_STATE, "handle has no MPHF loaded");
    if (h->params.key_kind != PTRHASH_KEY_BYTES) return fail(PTRHASH_E_STATE, "MPHF is for u64 keys");
    if (n_q == 0) return PTRHASH_OK;
    if (!data || !offsets || !out) return fail(PTRHASH_E_INVAL, "data/offsets/out is NULL");
    if (reinterpret_cast<uintptr_t>(data) & 7u) return fail(PTRHASH_E_INVAL, "data must be 8-byte aligned");
    const int rc = check_grid(n_q, h->tuning);
    if (rc) return rc;
    const hipError_t e = launch_query_bytes(device_view(h), data, offsets, n_q, out, h->params.index_bits == 64,
                                            h->tuning, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "query_bytes launch");
}

PTRHASH_API int ptrhash_bench_gather(const uint64_t *keys, uint64_t n_q, const uint8_t *table, uint64_t table_len,
                                     uint64_t *out, int keys_per_lane, int block, hipStream_t stream) {
    if (!valid_tuning(kKernelPipelined, keys_per_lane, block)) return fail(PTRHASH_E_INVAL, "bad tuning");
    if (n_q == 0) return PTRHASH_OK;
    if (!keys || !table || !out || table_len == 0) return fail(PTRHASH_E_INVAL, "NULL or empty argument");
    const Tuning t{kKernelPipelined, keys_per_lane, block};
    const int rc = check_grid(n_q, t);
    if (rc) return rc;
    const hipError_t e = launch_bench_gather(keys, n_q, table, table_len, out, keys_per_lane, block, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "gather launch");
}

PTRHASH_API int ptrhash_bench_copy(const uint64_t *keys, uint64_t n_q, uint64_t *out, int keys_per_lane, int block,
                                   hipStream_t stream) {
    if (!valid_tuning(kKernelPipelined, keys_per_lane, block)) return fail(PTRHASH_E_INVAL, "bad tuning");
    if (n_q == 0) return PTRHASH_OK;
    if (!keys || !out) return fail(PTRHASH_E_INVAL, "NULL argument");
    const Tuning t{kKernelPipelined, keys_per_lane, block};
    const int rc = check_grid(n_q, t);
    if (rc) return rc;
    const hipError_t e = launch_bench_copy(keys, n_q, out, keys_per_lane, block, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "copy launch");
}

}  // extern "C"
