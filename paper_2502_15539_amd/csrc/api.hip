// C ABI of the query library: handles, parameter rule, validation, device
// residency of an MPHF and kernel dispatch. All compute happens in the HIP
// kernels; this layer only checks arguments and launches.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

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

struct ptrhash_multi_plan {
    int max = 0;
    MultiTable *d_table = nullptr;  // device copy read by the kernel
    MultiTable *h_stage = nullptr;  // pinned, mapped host staging copy
    void *v_stage = nullptr;        // its device address
    size_t used_bytes = 0;
    ptrhash::MultiTuning tuning;
    uint32_t grid = 0;
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
    m.reduce_kind = h->params.reduce_kind;
    m.hash128 = h->params.hash_bits == 128;
    if (h->params.reduce_kind == PTRHASH_REDUCE_MOD) {
        m.mod_slots = (uint32_t)h->params.slots;
        m.mod_magic = ~0ull / h->params.slots;  // = floor(2^64/S) since S is not a power of two
    }
    return m;
}

constexpr uint64_t kMaxIndexSpace = 1ull << 40;  // CacheLineEF values are 40-bit

int check_params(const ptrhash_params *p) {
    if (!p) return fail(PTRHASH_E_INVAL, "params is NULL");
    if (p->n == 0) return fail(PTRHASH_E_INVAL, "n must be positive");
    if (p->num_parts == 0 || p->num_parts > 0xffffffffull)
        return fail(PTRHASH_E_INVAL, "num_parts must be in [1, 2^32)");
    if (p->buckets_per_part == 0) return fail(PTRHASH_E_INVAL, "buckets_per_part must be positive");
    if (p->reduce_kind > PTRHASH_REDUCE_MOD) return fail(PTRHASH_E_INVAL, "unknown reduce_kind %u", p->reduce_kind);
    uint64_t S;
    if (p->reduce_kind == PTRHASH_REDUCE_MOD) {
        if (p->num_parts != 1) return fail(PTRHASH_E_INVAL, "the mod reduce needs a single part");
        if (p->slots < 2 || p->slots >= (1ull << 32) || (p->slots & (p->slots - 1)) == 0)
            return fail(PTRHASH_E_INVAL, "the mod reduce needs 2 <= S < 2^32, S not a power of two");
        S = p->slots;
    } else {
        if (p->log2_slots > 40) return fail(PTRHASH_E_RANGE, "log2_slots %u > 40", p->log2_slots);
        S = 1ull << p->log2_slots;
    }
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
    if (p->hash_bits != 0 && p->hash_bits != 64 && p->hash_bits != 128)
        return fail(PTRHASH_E_INVAL, "hash_bits must be 64 or 128");
    if (p->hash_bits == 128 && p->key_kind != PTRHASH_KEY_BYTES)
        return fail(PTRHASH_E_INVAL, "128-bit hashing is for byte keys");
    return PTRHASH_OK;
}

}  // namespace

namespace {

MultiSpan span_of(const void *p, uint64_t bytes, int batch) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    return MultiSpan{a, a + bytes, batch};
}

// The input byte ranges a batch reads.
int batch_inputs(const ptrhash_query_desc &d, int i, MultiSpan *in) {
    if (d.handle->params.key_kind == PTRHASH_KEY_U64) {
        in[0] = span_of(d.keys, d.n_q * sizeof(uint64_t), i);
        return 1;
    }
    in[0] = span_of(d.data, d.data_len, i);
    in[1] = span_of(d.offsets, (d.n_q + 1) * sizeof(uint64_t), i);
    return 2;
}

// No batch's output range overlaps another output or any batch's input:
// the outputs are sorted by start and must be disjoint; then each input is
// checked against the last output that starts before it ends (outputs are
// disjoint, so their ends ascend with their starts). outs: room for k spans.
int check_batch_overlaps(const ptrhash_query_desc *descs, int k, MultiSpan *outs) {
    int no = 0;
    for (int i = 0; i < k; ++i)
        if (descs[i].n_q)
            outs[no++] = span_of(descs[i].out, descs[i].n_q * (descs[i].handle->params.index_bits / 8), i);
    std::sort(outs, outs + no, [](const MultiSpan &a, const MultiSpan &b) { return a.lo < b.lo; });
    for (int j = 1; j < no; ++j)
        if (outs[j].lo < outs[j - 1].hi)
            return fail(PTRHASH_E_INVAL, "batches %d and %d: outputs overlap", outs[j - 1].batch, outs[j].batch);
    for (int i = 0; i < k; ++i) {
        if (!descs[i].n_q) continue;
        MultiSpan in[2];
        const int m = batch_inputs(descs[i], i, in);
        for (int r = 0; r < m; ++r) {
            const MultiSpan *it = std::lower_bound(outs, outs + no, in[r].hi,
                                                   [](const MultiSpan &o, uintptr_t end) { return o.lo < end; });
            if (it != outs && (it - 1)->hi > in[r].lo)
                return fail(PTRHASH_E_INVAL, "batch %d: an input overlaps the output of batch %d", i, (it - 1)->batch);
        }
    }
    return PTRHASH_OK;
}

// Slot of handle h in the open-addressing table of w (inserted with index
// `next` if absent; *fresh tells which).
// Relative work of a batch in a multi-MPHF launch: 1 per key, plus
// kRemapCost for the expected share of its keys that are remapped (slot >=
// n: the share of slots at or past n in the MPHF's geometry), plus
// kPilotCost times the MPHF's pilot bytes over a die's 4 MB L2 (at most 1),
// which stands in for the pilot gathers that miss the L2. The weights are a
// least-squares fit of the per-die run times (workgroup clocks) of the
// 4096-request, 64-MPHF mix under two different splits (residuals within
// 3.5 us of 140-160 us).
constexpr double kRemapCost = 1.7, kPilotCost = 0.45, kDieL2Bytes = 4.0 * (1 << 20);
double multi_batch_cost(const MultiBatch &b, const DevMphf &m) {
    const double per_part = m.reduce_kind == kReduceMod ? (double)m.mod_slots : (double)(1ull << m.log2_slots);
    const double slots = (double)m.parts * per_part;
    const double remapped = m.remap_kind == kRemapNone || slots <= 0 ? 0.0 : (slots - (double)m.n) / slots;
    const double pilots = (double)m.parts * (double)m.buckets;
    const double l2 = pilots < kDieL2Bytes ? pilots / kDieL2Bytes : 1.0;
    return (double)b.nq * (1.0 + kRemapCost * remapped + kPilotCost * l2);
}

uint32_t handle_slot(MultiWork &w, const ptrhash_handle *h, uint32_t next, bool *fresh) {
    const uint32_t mask = w.hcap - 1;
    uint32_t i = (uint32_t)((reinterpret_cast<uintptr_t>(h) >> 4) * 0x9E3779B97F4A7C15ull >> 40) & mask;
    while (w.handles[i] && w.handles[i] != h) i = (i + 1) & mask;
    *fresh = !w.handles[i];
    if (*fresh) {
        w.handles[i] = h;
        w.index[i] = next;
    }
    return w.index[i];
}

}  // namespace

namespace ptrhash {
int fill_multi_table(MultiTable *t, const ptrhash_query_desc *descs, int k, uint32_t tile) {
    uint32_t cap = 2;
    const size_t kk = (size_t)(k > 0 ? k : 1);
    while (cap < 2u * (uint32_t)kk) cap <<= 1;
    std::vector<MultiSpan> outs(kk);
    std::vector<const ptrhash_handle *> handles(cap);
    std::vector<uint32_t> index(cap), batch_mphf(kk), mphf_start(kk + 1);
    MultiWork w{outs.data(), handles.data(), index.data(), cap, batch_mphf.data(), mphf_start.data()};
    return fill_multi_table_ws(t, descs, k, tile, w);
}

int fill_multi_table_ws(MultiTable *t, const ptrhash_query_desc *descs, int k, uint32_t tile, MultiWork &w) {
    // validate everything before touching the table
    for (int i = 0; i < k; ++i) {
        const ptrhash_query_desc &d = descs[i];
        if (!d.handle) return fail(PTRHASH_E_INVAL, "batch %d: handle is NULL", i);
        if (!d.handle->loaded) return fail(PTRHASH_E_STATE, "batch %d: handle has no MPHF loaded", i);
        if (d.n_q == 0) continue;
        if (!d.out) return fail(PTRHASH_E_INVAL, "batch %d: out is NULL", i);
        if (d.handle->params.key_kind == PTRHASH_KEY_U64) {
            if (!d.keys) return fail(PTRHASH_E_INVAL, "batch %d: keys is NULL for a u64-key MPHF", i);
        } else {
            if (!d.data || !d.offsets) return fail(PTRHASH_E_INVAL, "batch %d: data/offsets is NULL", i);
            if (reinterpret_cast<uintptr_t>(d.data) & 7u)
                return fail(PTRHASH_E_INVAL, "batch %d: data must be 8-byte aligned", i);
            if (d.data_len < kBytesPadding)
                return fail(PTRHASH_E_INVAL, "batch %d: data_len %llu is below the %llu bytes of padding", i,
                            (unsigned long long)d.data_len, (unsigned long long)kBytesPadding);
        }
    }
    if (k > 1 || (k == 1 && descs[0].n_q)) {
        const int rc = check_batch_overlaps(descs, k, w.outs);
        if (rc) return rc;
    }
    uint32_t c = 0;
    for (int i = 0; i < k; ++i) c += descs[i].n_q != 0;
    t->count = c;  // fixes where the arrays after the header start
    uint64_t *tb = multi_tile_begin(t);
    MultiBatch *bt = multi_batches(t);
    DevMphf *mp = multi_mphfs(t);
    // each distinct handle once, numbered in order of first appearance
    for (uint32_t i = 0; i < w.hcap; ++i) w.handles[i] = nullptr;
    uint32_t j = 0, mphfs = 0;
    for (int i = 0; i < k; ++i) {
        const ptrhash_query_desc &d = descs[i];
        if (d.n_q == 0) continue;
        bool fresh = false;
        const uint32_t mi = handle_slot(w, d.handle, mphfs, &fresh);
        if (fresh) mp[mphfs++] = device_view(d.handle);
        w.batch_mphf[j++] = mi;
    }
    // batches grouped by MPHF (a stable counting sort), so that the tiles
    // of one MPHF are contiguous
    for (uint32_t m = 0; m <= mphfs; ++m) w.mphf_start[m] = 0;
    for (uint32_t b = 0; b < c; ++b) w.mphf_start[w.batch_mphf[b] + 1]++;
    for (uint32_t m = 0; m < mphfs; ++m) w.mphf_start[m + 1] += w.mphf_start[m];
    j = 0;
    for (int i = 0; i < k; ++i) {
        const ptrhash_query_desc &d = descs[i];
        if (d.n_q == 0) continue;
        const uint32_t mi = w.batch_mphf[j++];
        const bool bytes = d.handle->params.key_kind == PTRHASH_KEY_BYTES;
        MultiBatch &b = bt[w.mphf_start[mi]++];
        b.keys = bytes ? static_cast<const void *>(d.data) : static_cast<const void *>(d.keys);
        b.offsets = bytes ? d.offsets : nullptr;
        b.out = d.out;
        b.nq = d.n_q;
        b.end_limit = bytes ? bytes_end_limit(d.data_len) : 0;
        b.mphf = mi;
        b.flags = (bytes ? kBatchBytes : 0u) | (d.handle->params.index_bits == 64 ? kBatchOut64 : 0u);
    }
    uint64_t tiles = 0;
    double cost = 0;
    for (uint32_t b = 0; b < c; ++b) {
        tb[b] = tiles;
        tiles += (bt[b].nq + tile - 1) / tile;
        cost += multi_batch_cost(bt[b], mp[bt[b].mphf]);
    }
    t->mphfs = mphfs;
    t->tile = tile;
    t->tiles = tiles;
    // die x's range starts where the running cost reaches x/8 of the total,
    // each batch's cost spread evenly over its tiles
    t->die_first[0] = 0;
    uint32_t b = 0;
    double before = 0;  // cost of the batches before b
    for (uint32_t x = 1; x < kDies; ++x) {
        const double target = cost * x / kDies;
        while (b < c) {
            const double cb = multi_batch_cost(bt[b], mp[bt[b].mphf]);
            if (before + cb > target) break;
            before += cb;
            ++b;
        }
        uint64_t first = tiles;
        if (b < c) {
            const uint64_t nt = (bt[b].nq + tile - 1) / tile;
            const double per = multi_batch_cost(bt[b], mp[bt[b].mphf]) / (double)nt;
            const uint64_t in = (uint64_t)((target - before) / per);
            first = tb[b] + (in < nt ? in : nt);
        }
        t->die_first[x] = first > t->die_first[x - 1] ? first : t->die_first[x - 1];
    }
    t->die_first[kDies] = tiles;
    return PTRHASH_OK;
}

uint32_t multi_grid(const MultiTuning &t) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 1;
    int per_cu = multi_blocks_per_cu(t);
    if (t.blocks_per_cu > 0 && t.blocks_per_cu < per_cu) per_cu = t.blocks_per_cu;
    return (uint32_t)cus * (uint32_t)per_cu;
}

bool valid_multi_tuning(int keys_per_lane, int block, int blocks_per_cu) {
    if (keys_per_lane != 1 && keys_per_lane != 2 && keys_per_lane != 4 && keys_per_lane != 8) return false;
    if (block < 64 || block > 1024 || block % 64) return false;
    return blocks_per_cu >= 0 && blocks_per_cu <= 64;
}

namespace {
std::atomic<int> g_multi_kpl{4}, g_multi_block{256}, g_multi_bpc{0};
}

MultiTuning multi_default_tuning() {
    MultiTuning t;
    t.keys_per_lane = g_multi_kpl.load();
    t.block = g_multi_block.load();
    t.blocks_per_cu = g_multi_bpc.load();
    return t;
}

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
    const bool single_mod = (preset & PTRHASH_PRESET_SINGLE_MOD) != 0;
    preset &= ~PTRHASH_PRESET_SINGLE_MOD;
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
    p.hash_bits = (key_kind == PTRHASH_KEY_BYTES && n > (1ull << 32)) ? 128u : 64u;
    if (single_mod && P == 1) {
        uint64_t Sm = (uint64_t)std::ceil((double)n / alpha);
        if (Sm < n + 16) Sm = n + 16;  // at least 16 free slots for tiny inputs
        if ((Sm & (Sm - 1)) == 0) ++Sm;
        uint64_t Bm = (uint64_t)std::ceil(alpha * (double)Sm / lambda);
        if (Bm < 1) Bm = 1;
        p.reduce_kind = PTRHASH_REDUCE_MOD;
        p.slots = Sm;
        p.log2_slots = 0;
        p.buckets_per_part = (uint32_t)Bm;
        p.remap_len = Sm - n;
    }
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

// LDS bytes per workgroup that cap residency at blocks_per_cu workgroups per
// CU (0 = no cap); *effective gets the cap the device's limits allow.
static int occupancy_lds(int blocks_per_cu, uint32_t *lds, int *effective) {
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(PTRHASH_E_INVAL, "blocks_per_cu must be 0..64");
    *lds = 0;
    if (effective) *effective = 0;
    if (blocks_per_cu == 0) return PTRHASH_OK;
    int dev = 0, per_cu = 0, per_block = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
        return hip_fail(e, "device query");
    uint32_t bytes = (uint32_t)(per_cu / blocks_per_cu) & ~255u;
    if (bytes > (uint32_t)per_block) bytes = (uint32_t)per_block & ~255u;
    *lds = bytes;
    if (effective) *effective = bytes ? per_cu / (int)bytes : 0;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_set_occupancy(ptrhash_handle *h, int blocks_per_cu, int *effective) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    uint32_t lds = 0;
    const int rc = occupancy_lds(blocks_per_cu, &lds, effective);
    if (rc) return rc;
    h->tuning.lds_bytes = lds;
    return PTRHASH_OK;
}

// The benchmark kernels run as one launch: its work-items (the grid times
// the block) must stay below 2^32.
static int check_grid(uint64_t n_q, const Tuning &t) {
    const uint64_t per_block = (uint64_t)t.block * (t.kernel == kKernelPlain ? 1 : t.keys_per_lane);
    if ((n_q + per_block - 1) / per_block * (uint64_t)t.block > 0xffffffffull)
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
    if (n_q > (~0ull >> 4)) return fail(PTRHASH_E_RANGE, "n_q %llu too large", (unsigned long long)n_q);
    if (ranges_overlap(keys, n_q * sizeof(uint64_t), out, n_q * (h->params.index_bits / 8)))
        return fail(PTRHASH_E_INVAL, "keys and out overlap");
    const hipError_t e =
        launch_query_u64(device_view(h), keys, n_q, out, h->params.index_bits == 64, h->tuning, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "query launch");
}

PTRHASH_API int ptrhash_query_bytes(ptrhash_handle *h, const uint8_t *data, uint64_t data_len,
                                    const uint64_t *offsets, uint64_t n_q, void *out, hipStream_t stream) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    if (!h->loaded) return fail(PTRHASH_E_STATE, "handle has no MPHF loaded");
    if (h->params.key_kind != PTRHASH_KEY_BYTES) return fail(PTRHASH_E_STATE, "MPHF is for u64 keys");
    if (n_q == 0) return PTRHASH_OK;
    if (!data || !offsets || !out) return fail(PTRHASH_E_INVAL, "data/offsets/out is NULL");
    if (reinterpret_cast<uintptr_t>(data) & 7u) return fail(PTRHASH_E_INVAL, "data must be 8-byte aligned");
    if (data_len < kBytesPadding)
        return fail(PTRHASH_E_INVAL, "data_len %llu is below the %llu bytes of padding", (unsigned long long)data_len,
                    (unsigned long long)kBytesPadding);
    if (n_q > (~0ull >> 4)) return fail(PTRHASH_E_RANGE, "n_q %llu too large", (unsigned long long)n_q);
    const uint64_t out_bytes = n_q * (h->params.index_bits / 8);
    if (ranges_overlap(data, data_len, out, out_bytes) ||
        ranges_overlap(offsets, (n_q + 1) * sizeof(uint64_t), out, out_bytes))
        return fail(PTRHASH_E_INVAL, "out overlaps data or offsets");
    const hipError_t e = launch_query_bytes(device_view(h), data, bytes_end_limit(data_len), offsets, n_q, out,
                                            h->params.index_bits == 64, h->tuning, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "query_bytes launch");
}

// ---- many MPHFs per launch ----

static constexpr int kMultiMax = 4096;
static constexpr int kRingSlots = 8;

PTRHASH_API int ptrhash_multi_max(void) { return kMultiMax; }

PTRHASH_API int ptrhash_multi_plan_destroy(ptrhash_multi_plan *plan) {
    if (!plan) return PTRHASH_OK;
    if (plan->d_table) (void)hipFree(plan->d_table);
    if (plan->h_stage) (void)hipHostFree(plan->h_stage);
    delete plan;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_multi_plan_create(int max_descs, ptrhash_multi_plan **out) {
    if (!out) return fail(PTRHASH_E_INVAL, "out is NULL");
    if (max_descs < 1 || max_descs > kMultiMax) return fail(PTRHASH_E_RANGE, "max_descs must be in [1, %d]", kMultiMax);
    ptrhash_multi_plan *p = new (std::nothrow) ptrhash_multi_plan();
    if (!p) return fail(PTRHASH_E_NOMEM, "plan allocation failed");
    p->max = max_descs;
    // rounded up for the 16-byte copy of the stage-in kernel
    const size_t bytes = (multi_table_capacity(max_descs) + 255) & ~(size_t)255;
    hipError_t e = hipMalloc(&p->d_table, bytes);
    if (e != hipSuccess) {
        p->d_table = nullptr;
        ptrhash_multi_plan_destroy(p);
        return fail(PTRHASH_E_NOMEM, "hipMalloc for the batch table: %s", hipGetErrorString(e));
    }
    e = hipHostMalloc(&p->h_stage, bytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) p->h_stage = nullptr;
    if (e == hipSuccess) e = hipHostGetDevicePointer(&p->v_stage, p->h_stage, 0);
    if (e != hipSuccess) {
        ptrhash_multi_plan_destroy(p);
        return fail(PTRHASH_E_NOMEM, "hipHostMalloc for the staging table: %s", hipGetErrorString(e));
    }
    std::memset(p->h_stage, 0, bytes);
    p->tuning = multi_default_tuning();
    p->h_stage->tile = multi_tile(p->tuning);
    p->grid = multi_grid(p->tuning);
    p->used_bytes = multi_table_bytes(0, 0);
    *out = p;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_multi_plan_set(ptrhash_multi_plan *plan, const ptrhash_query_desc *descs, int k) {
    if (!plan) return fail(PTRHASH_E_INVAL, "plan is NULL");
    if (k < 0 || (k > 0 && !descs)) return fail(PTRHASH_E_INVAL, "bad descriptor array");
    if (k > plan->max) return fail(PTRHASH_E_RANGE, "%d batches exceed the plan's %d", k, plan->max);
    const int rc = fill_multi_table(plan->h_stage, descs, k, multi_tile(plan->tuning));
    if (rc) return rc;
    plan->used_bytes = multi_table_bytes(plan->h_stage->count, plan->h_stage->mphfs);
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_multi_plan_set_kernel(ptrhash_multi_plan *plan, int keys_per_lane, int block,
                                              int blocks_per_cu) {
    if (!plan) return fail(PTRHASH_E_INVAL, "plan is NULL");
    if (!valid_multi_tuning(keys_per_lane, block, blocks_per_cu))
        return fail(PTRHASH_E_INVAL, "keys_per_lane in {1, 2, 4, 8}, block 64..1024 (multiple of 64), "
                                     "blocks_per_cu 0..64");
    plan->tuning.keys_per_lane = keys_per_lane;
    plan->tuning.block = block;
    plan->tuning.blocks_per_cu = blocks_per_cu;
    plan->grid = multi_grid(plan->tuning);
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_set_multi_kernel(int keys_per_lane, int block, int blocks_per_cu) {
    if (!valid_multi_tuning(keys_per_lane, block, blocks_per_cu))
        return fail(PTRHASH_E_INVAL, "keys_per_lane in {1, 2, 4, 8}, block 64..1024 (multiple of 64), "
                                     "blocks_per_cu 0..64");
    g_multi_kpl.store(keys_per_lane);
    g_multi_block.store(block);
    g_multi_bpc.store(blocks_per_cu);
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_multi_plan_launch(ptrhash_multi_plan *plan, hipStream_t stream) {
    if (!plan) return fail(PTRHASH_E_INVAL, "plan is NULL");
    if (plan->h_stage->tile != multi_tile(plan->tuning))
        return fail(PTRHASH_E_STATE, "the kernel changed after ptrhash_multi_plan_set: set the batches again");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing && plan->h_stage->tiles == 0) return PTRHASH_OK;
    // a captured copy must cover any later table, so it copies all of it
    const size_t bytes = capturing ? multi_table_capacity(plan->max) : plan->used_bytes;
    e = launch_stage_in(plan->v_stage, plan->d_table, bytes, stream);
    if (e != hipSuccess) return hip_fail(e, "batch table copy");
    e = launch_query_multi(plan->d_table, plan->tuning, plan->grid, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "query_multi launch");
}

namespace {
struct PlanRing {
    std::mutex mu;
    ptrhash_multi_plan *plans[kRingSlots] = {};
    hipEvent_t done[kRingSlots] = {};
    bool pending[kRingSlots] = {};
    int next = 0;
};
constexpr int kMaxDevices = 64;
PlanRing g_rings[kMaxDevices];
}  // namespace

PTRHASH_API int ptrhash_query_multi(const ptrhash_query_desc *descs, int k, hipStream_t stream) {
    if (k < 0 || (k > 0 && !descs)) return fail(PTRHASH_E_INVAL, "bad descriptor array");
    if (k > kMultiMax) return fail(PTRHASH_E_RANGE, "%d batches exceed %d", k, kMultiMax);
    if (k == 0) return PTRHASH_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) return fail(PTRHASH_E_STATE, "stream is capturing: capture a plan instead");
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PTRHASH_E_RANGE, "device %d out of range", dev);
    PlanRing &r = g_rings[dev];
    std::lock_guard<std::mutex> lock(r.mu);
    const int slot = r.next;
    r.next = (r.next + 1) % kRingSlots;
    if (!r.plans[slot]) {
        int rc = ptrhash_multi_plan_create(kMultiMax, &r.plans[slot]);
        if (rc) return rc;
        if ((e = hipEventCreateWithFlags(&r.done[slot], hipEventDisableTiming)) != hipSuccess) {
            ptrhash_multi_plan_destroy(r.plans[slot]);
            r.plans[slot] = nullptr;
            return hip_fail(e, "hipEventCreate");
        }
    }
    if (r.pending[slot]) {
        if ((e = hipEventSynchronize(r.done[slot])) != hipSuccess) return hip_fail(e, "waiting for a plan slot");
        r.pending[slot] = false;
    }
    const MultiTuning t = multi_default_tuning();
    ptrhash_multi_plan *plan = r.plans[slot];
    if (t.keys_per_lane != plan->tuning.keys_per_lane || t.block != plan->tuning.block ||
        t.blocks_per_cu != plan->tuning.blocks_per_cu) {
        int rc = ptrhash_multi_plan_set_kernel(plan, t.keys_per_lane, t.block, t.blocks_per_cu);
        if (rc) return rc;
    }
    int rc = ptrhash_multi_plan_set(plan, descs, k);
    if (rc) return rc;
    rc = ptrhash_multi_plan_launch(plan, stream);
    if (rc) return rc;
    if ((e = hipEventRecord(r.done[slot], stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    r.pending[slot] = true;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_bench_gather(const uint64_t *keys, uint64_t n_q, const uint8_t *table, uint64_t table_len,
                                     uint64_t *out, int keys_per_lane, int block, int blocks_per_cu,
                                     hipStream_t stream) {
    if (!valid_tuning(kKernelPipelined, keys_per_lane, block)) return fail(PTRHASH_E_INVAL, "bad tuning");
    if (n_q == 0) return PTRHASH_OK;
    if (!keys || !table || !out || table_len == 0) return fail(PTRHASH_E_INVAL, "NULL or empty argument");
    Tuning t{kKernelPipelined, keys_per_lane, block};
    int rc = occupancy_lds(blocks_per_cu, &t.lds_bytes, nullptr);
    if (rc) return rc;
    rc = check_grid(n_q, t);
    if (rc) return rc;
    const hipError_t e = launch_bench_gather(keys, n_q, table, table_len, out, keys_per_lane, block, t.lds_bytes,
                                             stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "gather launch");
}

PTRHASH_API int ptrhash_bench_gather_buckets(ptrhash_handle *h, const uint64_t *keys, uint64_t n_q, uint64_t *out,
                                             int keys_per_lane, int block, int blocks_per_cu, hipStream_t stream) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    if (!h->loaded) return fail(PTRHASH_E_STATE, "handle has no MPHF loaded");
    if (h->params.key_kind != PTRHASH_KEY_U64) return fail(PTRHASH_E_STATE, "MPHF is for byte keys");
    if (!valid_tuning(kKernelPipelined, keys_per_lane, block)) return fail(PTRHASH_E_INVAL, "bad tuning");
    if (n_q == 0) return PTRHASH_OK;
    if (!keys || !out) return fail(PTRHASH_E_INVAL, "NULL argument");
    if (ranges_overlap(keys, n_q * 8, out, n_q * 8)) return fail(PTRHASH_E_INVAL, "keys and out overlap");
    Tuning t{kKernelPipelined, keys_per_lane, block};
    int rc = occupancy_lds(blocks_per_cu, &t.lds_bytes, nullptr);
    if (rc) return rc;
    rc = check_grid(n_q, t);
    if (rc) return rc;
    const hipError_t e = launch_bench_gather_bucket(keys, n_q, device_view(h), out, keys_per_lane, block, t.lds_bytes,
                                                    stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "bucket gather launch");
}

PTRHASH_API int ptrhash_bench_gather_bytes(ptrhash_handle *h, const uint8_t *data, uint64_t data_len,
                                           const uint64_t *offsets, uint64_t n_q, uint32_t *out, int keys_per_lane,
                                           int block, int blocks_per_cu, hipStream_t stream) {
    if (!h) return fail(PTRHASH_E_INVAL, "handle is NULL");
    if (!h->loaded) return fail(PTRHASH_E_STATE, "handle has no MPHF loaded");
    if (!valid_tuning(kKernelPipelined, keys_per_lane, block)) return fail(PTRHASH_E_INVAL, "bad tuning");
    if (n_q == 0) return PTRHASH_OK;
    if (!data || !offsets || !out) return fail(PTRHASH_E_INVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(data) & 7u) return fail(PTRHASH_E_INVAL, "data must be 8-byte aligned");
    if (data_len < kBytesPadding) return fail(PTRHASH_E_INVAL, "data_len is below the padding");
    if (ranges_overlap(data, data_len, out, n_q * 4) || ranges_overlap(offsets, (n_q + 1) * 8, out, n_q * 4))
        return fail(PTRHASH_E_INVAL, "out overlaps data or offsets");
    Tuning t{kKernelPipelined, keys_per_lane, block};
    int rc = occupancy_lds(blocks_per_cu, &t.lds_bytes, nullptr);
    if (rc) return rc;
    rc = check_grid(n_q, t);
    if (rc) return rc;
    const hipError_t e = launch_bench_gather_bytes(data, bytes_end_limit(data_len), offsets, n_q, device_view(h), out,
                                                   keys_per_lane, block, t.lds_bytes, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "string gather launch");
}

PTRHASH_API int ptrhash_bench_scatter(const uint64_t *in, uint32_t log2_n, uint64_t *out, hipStream_t stream) {
    if (!in || !out) return fail(PTRHASH_E_INVAL, "NULL argument");
    if (log2_n < 8 || log2_n > 34) return fail(PTRHASH_E_INVAL, "log2_n must be 8..34");
    if (ranges_overlap(in, 8ull << log2_n, out, 8ull << log2_n)) return fail(PTRHASH_E_INVAL, "in and out overlap");
    const hipError_t e = launch_bench_scatter(in, log2_n, out, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "scatter launch");
}

PTRHASH_API int ptrhash_bench_gather_pure(uint64_t n, const uint8_t *table, uint64_t table_len, uint32_t *sink,
                                          uint32_t lanes, hipStream_t stream) {
    if (n == 0) return PTRHASH_OK;
    if (!table || !sink || table_len == 0) return fail(PTRHASH_E_INVAL, "NULL or empty argument");
    if (lanes < 256 || lanes % 256) return fail(PTRHASH_E_INVAL, "lanes must be a positive multiple of 256");
    const hipError_t e = launch_bench_gather_pure(n, table, table_len, sink, lanes / 256, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "pure gather launch");
}

PTRHASH_API int ptrhash_bench_gather_pair(uint64_t n, const uint8_t *table, uint64_t table_len, uint32_t *sink,
                                          uint32_t lanes, uint32_t xor_dist, hipStream_t stream) {
    if (n == 0) return PTRHASH_OK;
    if (!table || !sink || table_len < 256 || table_len % 256)
        return fail(PTRHASH_E_INVAL, "NULL table/sink, or table_len not a positive multiple of 256");
    if (lanes < 256 || lanes % 256) return fail(PTRHASH_E_INVAL, "lanes must be a positive multiple of 256");
    if (xor_dist != 32 && xor_dist != 64 && xor_dist != 128) return fail(PTRHASH_E_INVAL, "xor_dist: 32, 64 or 128");
    const hipError_t e = launch_bench_gather_pair(n, table, table_len, xor_dist, sink, lanes / 256, stream);
    return e == hipSuccess ? PTRHASH_OK : hip_fail(e, "pair gather launch");
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
