// Serving core: continuous batching of query requests against resident
// MPHFs (the throughput argument of Appendix A -- many queries known in
// advance -- recovered from a stream of independent small requests).
//
// Requests (host keys in, host indices out) queue up; a dispatcher thread
// owns `streams` launch slots, each with a device arena of `slot_keys` keys
// and a multi-batch plan. Whenever a slot is free it admits queued requests
// in arrival order while they fit the arena (memory) and the plan (batch
// count), copies their keys to the device, runs one persistent multi-MPHF
// launch and copies the indices back, all asynchronously on the slot's
// stream; slots overlap on the device. Completed slots are retired by
// polling their events, and each request's latency (submit -> indices in
// the caller's buffer) is recorded.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "errors.h"
#include "internal.h"
#include "ptrhash.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    ptrhash_handle *handle = nullptr;
    const uint64_t *keys = nullptr;
    uint64_t n_q = 0;
    void *out = nullptr;
    uint32_t out_bytes = 4;   // bytes per index
    bool mapped = false;      // keys/out in mapped host memory: the kernel uses them in place
    const uint64_t *v_keys = nullptr;  // their device addresses
    void *v_out = nullptr;
    Clock::time_point t_submit{};
    Clock::time_point t_launch{};
    uint64_t key_off = 0;     // placement inside the slot arena
    uint64_t out_off = 0;     // byte offset inside the slot's output arena
};

// Fork-join pool for the host copies of a launch (keys into pinned staging,
// indices out of it): the copies of one launch are split into chunks that
// the pool's threads and the dispatcher take from a shared counter.
class CopyPool {
  public:
    struct Job {
        void *dst;
        const void *src;
        size_t bytes;
    };

    explicit CopyPool(int threads) {
        for (int i = 0; i < threads; ++i) workers_.emplace_back([this] { loop(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> l(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }

    // Run every job; returns when all are done and no pool thread still
    // holds the job list.
    void run(std::vector<Job> &jobs) {
        if (jobs.empty()) return;
        if (workers_.empty() || jobs.size() == 1) {
            for (const Job &j : jobs) std::memcpy(j.dst, j.src, j.bytes);
            return;
        }
        {
            std::lock_guard<std::mutex> l(mu_);
            jobs_ = &jobs;
            next_.store(0);
            left_.store(jobs.size());
            ++gen_;
        }
        cv_.notify_all();
        take(jobs);
        while (left_.load(std::memory_order_acquire) != 0) std::this_thread::yield();
        for (;;) {  // threads join only under the lock while jobs_ is set
            std::unique_lock<std::mutex> l(mu_);
            if (active_.load(std::memory_order_acquire) == 0) {
                jobs_ = nullptr;
                return;
            }
            l.unlock();
            std::this_thread::yield();
        }
    }

  private:
    void take(std::vector<Job> &jobs) {
        for (;;) {
            const size_t i = next_.fetch_add(1);
            if (i >= jobs.size()) return;
            const Job &j = jobs[i];
            std::memcpy(j.dst, j.src, j.bytes);
            left_.fetch_sub(1, std::memory_order_release);
        }
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            std::vector<Job> *jobs;
            {
                std::unique_lock<std::mutex> l(mu_);
                cv_.wait(l, [&] { return stop_ || (gen_ != seen && jobs_); });
                if (stop_) return;
                seen = gen_;
                jobs = jobs_;
                active_.fetch_add(1, std::memory_order_acq_rel);
            }
            take(*jobs);
            active_.fetch_sub(1, std::memory_order_acq_rel);
        }
    }

    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::vector<Job> *jobs_ = nullptr;
    std::atomic<size_t> next_{0}, left_{0};
    std::atomic<int> active_{0};
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// Mapped, coherent host allocations handed out by ptrhash_host_alloc, so
// that a request's buffers (any range inside one allocation) can be turned
// into device addresses without a runtime call per request.
struct MappedAlloc {
    uintptr_t end;
    uintptr_t dev;
};
std::mutex g_mapped_mu;
std::map<uintptr_t, MappedAlloc> g_mapped;  // host base -> end, device base

// Device address of [p, p + bytes) if it lies inside one mapped allocation.
bool mapped_view(const void *p, uint64_t bytes, void **dev) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> l(g_mapped_mu);
    auto it = g_mapped.upper_bound(a);
    if (it == g_mapped.begin()) return false;
    --it;
    if (a < it->first || a >= it->second.end || bytes > it->second.end - a) return false;
    *dev = reinterpret_cast<void *>(it->second.dev + (a - it->first));
    return true;
}

// Split a copy into chunks of at most 256 KiB.
void add_copy(std::vector<CopyPool::Job> &jobs, void *dst, const void *src, size_t bytes) {
    constexpr size_t kChunk = 256 << 10;
    for (size_t o = 0; o < bytes; o += kChunk)
        jobs.push_back({static_cast<uint8_t *>(dst) + o, static_cast<const uint8_t *>(src) + o,
                        std::min(kChunk, bytes - o)});
}

// The most recent kStatWindow samples (a ring once full), so that a server
// that runs for hours keeps bounded memory and its percentiles describe
// recent traffic.
constexpr size_t kStatWindow = size_t(1) << 20;
struct StatWindow {
    std::vector<double> v;
    size_t next = 0;
    void add(double x) {
        if (v.size() < kStatWindow) {
            v.push_back(x);
        } else {
            v[next] = x;
            next = (next + 1) % kStatWindow;
        }
    }
    void clear() {
        v.clear();
        next = 0;
    }
};

// Device-timeline intervals of recent launches (ms after the server's base
// event), for the overlap metrics.
constexpr size_t kSpanWindow = size_t(1) << 16;
struct SpanWindow {
    std::vector<std::pair<double, double>> v;
    size_t next = 0;
    void add(double a, double b) {
        if (v.size() < kSpanWindow) {
            v.emplace_back(a, b);
        } else {
            v[next] = {a, b};
            next = (next + 1) % kSpanWindow;
        }
    }
    void clear() {
        v.clear();
        next = 0;
    }
    // Most intervals open at one instant, and the mean number open over the
    // time at least one is (sum of lengths / length of their union).
    void overlap(uint64_t &most, double &mean) const {
        std::vector<std::pair<double, int>> ev;
        ev.reserve(2 * v.size());
        for (const auto &iv : v) {
            ev.emplace_back(iv.first, +1);
            ev.emplace_back(iv.second, -1);
        }
        std::sort(ev.begin(), ev.end());  // an end sorts before a start at the same instant
        int open = 0, top = 0;
        double busy = 0, total = 0, prev = 0;
        for (const auto &e : ev) {
            if (open > 0) busy += e.first - prev;
            open += e.second;
            if (open > top) top = open;
            prev = e.first;
        }
        for (const auto &iv : v) total += iv.second - iv.first;
        most = (uint64_t)top;
        mean = busy > 0 ? total / busy : (v.empty() ? 0.0 : 1.0);
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr;  // recorded before the slot's launch (timing events)
    hipEvent_t done = nullptr;   // recorded after it
    ptrhash_multi_plan *plan = nullptr;        // copy mode
    uint64_t *d_keys = nullptr, *h_keys = nullptr;
    uint8_t *d_out = nullptr, *h_out = nullptr;
    ptrhash::MultiTable *h_table = nullptr;             // zero-copy mode: mapped host table
    ptrhash::MultiTable *v_table = nullptr;             // its device address
    uint64_t *v_keys = nullptr;                // device addresses of h_keys / h_out
    uint8_t *v_out = nullptr;
    std::vector<Request> reqs;
    bool busy = false;
};

}  // namespace

struct ptrhash_server {
    ptrhash_server_config cfg{};
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    uint64_t queued_keys = 0;
    uint64_t next_ticket = 1;
    std::unordered_set<uint64_t> outstanding;       // submitted, not finished
    std::unordered_map<uint64_t, double> finished;  // ticket -> latency (us), until waited for
    StatWindow latencies;                            // completed requests (recent ones)
    StatWindow waits;                                // submit -> launch enqueued
    SpanWindow spans;                                // device start/done of recent launches
    hipEvent_t base = nullptr;                       // time origin of the spans
    CopyPool *pool = nullptr;
    uint64_t launches = 0, completed = 0, keys_done = 0;
    int busy_now = 0, busy_max = 0;                  // slots launched and not yet retired
    int error = PTRHASH_OK;
    bool stop = false;
    int device = 0;
    ptrhash::MultiTuning tuning;  // launch shape of the multi-MPHF kernel
    uint32_t grid = 0;
    std::thread worker;
};

namespace {

int hip_err(hipError_t e, const char *what) {
    return ptrhash::set_error(PTRHASH_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

void free_slot(Slot &s) {
    if (s.plan) ptrhash_multi_plan_destroy(s.plan);
    if (s.d_keys) (void)hipFree(s.d_keys);
    if (s.d_out) (void)hipFree(s.d_out);
    if (s.h_keys) (void)hipHostFree(s.h_keys);
    if (s.h_out) (void)hipHostFree(s.h_out);
    if (s.h_table) (void)hipHostFree(s.h_table);
    if (s.start) (void)hipEventDestroy(s.start);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = Slot{};
}

// Retire a finished slot: copy indices to the callers' buffers.
void retire(ptrhash_server *srv, Slot &s) {
    std::vector<CopyPool::Job> jobs;
    for (const Request &r : s.reqs)
        if (!r.mapped) add_copy(jobs, r.out, s.h_out + r.out_off, r.n_q * r.out_bytes);
    srv->pool->run(jobs);
    const auto now = Clock::now();
    float t0 = 0, t1 = 0;
    const bool timed = hipEventElapsedTime(&t0, srv->base, s.start) == hipSuccess &&
                       hipEventElapsedTime(&t1, srv->base, s.done) == hipSuccess;
    std::lock_guard<std::mutex> lock(srv->mu);
    if (timed) srv->spans.add(t0, t1);
    srv->busy_now--;
    for (const Request &r : s.reqs) {
        srv->waits.add(std::chrono::duration<double, std::micro>(r.t_launch - r.t_submit).count());
        const double us = std::chrono::duration<double, std::micro>(now - r.t_submit).count();
        srv->outstanding.erase(r.ticket);
        srv->finished[r.ticket] = us;
        srv->latencies.add(us);
        srv->completed++;
        srv->keys_done += r.n_q;
    }
    s.reqs.clear();
    s.busy = false;
    srv->cv_done.notify_all();
}

// Admit queued requests into a free slot and launch them. Called with the
// lock held; releases it around the copies and the launch.
int admit(ptrhash_server *srv, Slot &s, std::unique_lock<std::mutex> &lock) {
    uint64_t used = 0, out_used = 0, budget = 0;
    while (!srv->queue.empty() && (int)s.reqs.size() < srv->cfg.max_batches) {
        Request &r = srv->queue.front();
        if (budget + r.n_q > srv->cfg.slot_keys) break;
        budget += r.n_q;
        if (!r.mapped) {  // arena space for the copies
            r.key_off = used;
            r.out_off = out_used;
            used += r.n_q;
            out_used += (r.n_q * r.out_bytes + 7) & ~7ull;
        }
        srv->queued_keys -= r.n_q;
        s.reqs.push_back(r);
        srv->queue.pop_front();
    }
    if (s.reqs.empty()) return PTRHASH_OK;
    s.busy = true;
    if (++srv->busy_now > srv->busy_max) srv->busy_max = srv->busy_now;
    lock.unlock();
    const bool zc = srv->cfg.zero_copy != 0;
    std::vector<ptrhash_query_desc> descs(s.reqs.size());
    std::vector<CopyPool::Job> jobs;
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        const Request &r = s.reqs[i];
        if (r.mapped) {
            descs[i] = ptrhash_query_desc{r.handle, r.v_keys, nullptr, 0, nullptr, r.n_q, r.v_out};
            continue;
        }
        add_copy(jobs, s.h_keys + r.key_off, r.keys, r.n_q * sizeof(uint64_t));
        uint64_t *k = (zc ? s.v_keys : s.d_keys) + r.key_off;
        uint8_t *o = (zc ? s.v_out : s.d_out) + r.out_off;
        descs[i] = ptrhash_query_desc{r.handle, k, nullptr, 0, nullptr, r.n_q, o};
    }
    srv->pool->run(jobs);
    int rc;
    hipError_t e = hipSuccess;
    if (zc) {
        // the kernel reads keys and the batch table from, and writes indices
        // to, mapped coherent host memory: one kernel per launch
        rc = ptrhash::fill_multi_table(s.h_table, descs.data(), (int)descs.size(), ptrhash::multi_tile(srv->tuning));
        if (rc == PTRHASH_OK) {
            e = hipEventRecord(s.start, s.stream);
            if (e == hipSuccess) e = ptrhash::launch_query_multi(s.v_table, srv->tuning, srv->grid, s.stream);
            if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
            if (e != hipSuccess) rc = hip_err(e, "serving launch");
        }
    } else if ((rc = ptrhash_multi_plan_set(s.plan, descs.data(), (int)descs.size())) == PTRHASH_OK) {
        e = hipEventRecord(s.start, s.stream);
        if (e == hipSuccess && used)
            e = hipMemcpyAsync(s.d_keys, s.h_keys, used * sizeof(uint64_t), hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess) rc = ptrhash_multi_plan_launch(s.plan, s.stream);
        if (e == hipSuccess && rc == PTRHASH_OK && out_used)
            e = hipMemcpyAsync(s.h_out, s.d_out, out_used, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess && rc == PTRHASH_OK) e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) rc = hip_err(e, "serving launch");
    }
    const auto launched = Clock::now();
    for (Request &r : s.reqs) r.t_launch = launched;
    lock.lock();
    if (rc == PTRHASH_OK) srv->launches++;
    return rc;
}

void run(ptrhash_server *srv) {
    (void)hipSetDevice(srv->device);
    auto idle_since = Clock::now();
    std::unique_lock<std::mutex> lock(srv->mu);
    for (;;) {
        bool any_busy = false;
        // retire finished slots
        for (Slot &s : srv->slots) {
            if (!s.busy) continue;
            lock.unlock();
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipSuccess) {
                retire(srv, s);
            } else if (q != hipErrorNotReady) {
                lock.lock();
                srv->error = hip_err(q, "serving completion");
                srv->stop = true;
                srv->cv_done.notify_all();
                return;
            }
            lock.lock();
            any_busy |= s.busy;
        }
        // admit into free slots
        for (Slot &s : srv->slots) {
            if (s.busy || srv->queue.empty()) continue;
            const int rc = admit(srv, s, lock);
            if (rc != PTRHASH_OK) {
                srv->error = rc;
                srv->stop = true;
                srv->cv_done.notify_all();
                return;
            }
            any_busy |= s.busy;
        }
        if (srv->stop && srv->queue.empty() && !any_busy) return;
        if (any_busy || !srv->queue.empty()) {
            idle_since = Clock::now();
            lock.unlock();
            std::this_thread::yield();
            lock.lock();
        } else if (Clock::now() - idle_since < std::chrono::microseconds(500)) {
            // stay awake briefly: a new request is likely soon
            lock.unlock();
            std::this_thread::yield();
            lock.lock();
        } else {
            srv->cv_work.wait(lock, [&] { return srv->stop || !srv->queue.empty(); });
            idle_since = Clock::now();
        }
    }
}

}  // namespace

extern "C" {

PTRHASH_API int ptrhash_server_default_config(ptrhash_server_config *cfg) {
    if (!cfg) return ptrhash::set_error(PTRHASH_E_INVAL, "cfg is NULL");
    cfg->streams = 2;
    cfg->max_batches = 1024;
    cfg->slot_keys = 1u << 22;
    cfg->max_queued_keys = 1ull << 28;
    cfg->copy_threads = 4;
    cfg->zero_copy = 1;
    cfg->keys_per_lane = 0;  // the process default launch shape
    cfg->block = 0;
    cfg->blocks_per_cu = 0;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_server_create(const ptrhash_server_config *cfg, ptrhash_server **out) {
    if (!cfg || !out) return ptrhash::set_error(PTRHASH_E_INVAL, "NULL argument");
    if (cfg->streams < 1 || cfg->streams > 16) return ptrhash::set_error(PTRHASH_E_INVAL, "streams must be 1..16");
    if (cfg->max_batches < 1 || cfg->max_batches > ptrhash_multi_max())
        return ptrhash::set_error(PTRHASH_E_INVAL, "max_batches must be 1..%d", ptrhash_multi_max());
    if (cfg->slot_keys < 1 || cfg->slot_keys > (1ull << 32))
        return ptrhash::set_error(PTRHASH_E_INVAL, "slot_keys must be 1..2^32");
    if (cfg->max_queued_keys < cfg->slot_keys)
        return ptrhash::set_error(PTRHASH_E_INVAL, "max_queued_keys must be >= slot_keys");
    if (cfg->copy_threads < 0 || cfg->copy_threads > 64)
        return ptrhash::set_error(PTRHASH_E_INVAL, "copy_threads must be 0..64");
    ptrhash::MultiTuning tuning = ptrhash::multi_default_tuning();
    if (cfg->keys_per_lane != 0) {
        if (!ptrhash::valid_multi_tuning(cfg->keys_per_lane, cfg->block, cfg->blocks_per_cu))
            return ptrhash::set_error(PTRHASH_E_INVAL, "keys_per_lane in {1, 2, 4, 8}, block 64..1024 "
                                                       "(multiple of 64), blocks_per_cu 0..64");
        tuning.keys_per_lane = cfg->keys_per_lane;
        tuning.block = cfg->block;
        tuning.blocks_per_cu = cfg->blocks_per_cu;
    }
    ptrhash_server *srv = new (std::nothrow) ptrhash_server();
    if (!srv) return ptrhash::set_error(PTRHASH_E_NOMEM, "server allocation failed");
    srv->cfg = *cfg;
    hipError_t e = hipGetDevice(&srv->device);
    int rc = e == hipSuccess ? PTRHASH_OK : hip_err(e, "hipGetDevice");
    srv->slots.resize(cfg->streams);
    srv->tuning = tuning;
    srv->grid = ptrhash::multi_grid(tuning);
    const bool zc = cfg->zero_copy != 0;
    const unsigned pin = zc ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault;
    for (Slot &s : srv->slots) {
        if (rc) break;
        const uint64_t kb = cfg->slot_keys * sizeof(uint64_t);
        const uint64_t ob = cfg->slot_keys * sizeof(uint64_t) + 8 * (uint64_t)cfg->max_batches;
        if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreate(&s.start)) != hipSuccess || (e = hipEventCreate(&s.done)) != hipSuccess) {
            rc = hip_err(e, "stream/event creation");
            break;
        }
        if (hipHostMalloc(&s.h_keys, kb, pin) != hipSuccess || hipHostMalloc(&s.h_out, ob, pin) != hipSuccess) {
            rc = ptrhash::set_error(PTRHASH_E_NOMEM, "serving staging allocation failed");
            break;
        }
        if (zc) {
            if (hipHostMalloc(&s.h_table, ptrhash::multi_table_capacity(cfg->max_batches), pin) != hipSuccess ||
                hipHostGetDevicePointer((void **)&s.v_table, s.h_table, 0) != hipSuccess ||
                hipHostGetDevicePointer((void **)&s.v_keys, s.h_keys, 0) != hipSuccess ||
                hipHostGetDevicePointer((void **)&s.v_out, s.h_out, 0) != hipSuccess) {
                rc = ptrhash::set_error(PTRHASH_E_NOMEM, "mapped serving buffers failed");
                break;
            }
        } else {
            if (hipMalloc(&s.d_keys, kb) != hipSuccess || hipMalloc(&s.d_out, ob) != hipSuccess) {
                rc = ptrhash::set_error(PTRHASH_E_NOMEM, "serving arena allocation failed");
                break;
            }
            rc = ptrhash_multi_plan_create(cfg->max_batches, &s.plan);
            if (rc == PTRHASH_OK)
                rc = ptrhash_multi_plan_set_kernel(s.plan, tuning.keys_per_lane, tuning.block, tuning.blocks_per_cu);
        }
    }
    if (rc == PTRHASH_OK) {
        if ((e = hipEventCreate(&srv->base)) != hipSuccess ||
            (e = hipEventRecord(srv->base, srv->slots[0].stream)) != hipSuccess ||
            (e = hipEventSynchronize(srv->base)) != hipSuccess)
            rc = hip_err(e, "server base event");
    }
    if (rc) {
        for (Slot &s : srv->slots) free_slot(s);
        if (srv->base) (void)hipEventDestroy(srv->base);
        delete srv;
        return rc;
    }
    srv->pool = new CopyPool(cfg->copy_threads);
    srv->worker = std::thread(run, srv);
    *out = srv;
    return PTRHASH_OK;
}

static int submit_at(ptrhash_server *srv, ptrhash_handle *h, const uint64_t *keys, uint64_t n_q, void *out,
                     uint64_t *ticket, Clock::time_point arrival, bool mapped) {
    if (!srv || !h || !ticket || (n_q && (!keys || !out))) return ptrhash::set_error(PTRHASH_E_INVAL, "NULL argument");
    ptrhash_params p;
    int rc = ptrhash_get_params(h, &p);
    if (rc) return rc;
    if (p.key_kind != PTRHASH_KEY_U64) return ptrhash::set_error(PTRHASH_E_STATE, "serving takes u64-key MPHFs");
    if (n_q > srv->cfg.slot_keys)
        return ptrhash::set_error(PTRHASH_E_RANGE, "request of %llu keys exceeds slot_keys",
                                  (unsigned long long)n_q);
    Request r;
    r.handle = h;
    r.keys = keys;
    r.n_q = n_q;
    r.out = out;
    r.out_bytes = p.index_bits / 8;
    if (mapped && n_q) {
        void *vk = nullptr, *vo = nullptr;
        if (!mapped_view(keys, n_q * sizeof(uint64_t), &vk) || !mapped_view(out, n_q * r.out_bytes, &vo))
            return ptrhash::set_error(PTRHASH_E_INVAL, "mapped request: keys/out not inside ptrhash_host_alloc memory");
        r.mapped = true;
        r.v_keys = static_cast<const uint64_t *>(vk);
        r.v_out = vo;
    }
    std::unique_lock<std::mutex> lock(srv->mu);
    if (srv->error) return ptrhash::set_error(srv->error, "server stopped after an error");
    if (srv->stop) return ptrhash::set_error(PTRHASH_E_STATE, "server is stopping");
    if (srv->queued_keys + n_q > srv->cfg.max_queued_keys)
        return ptrhash::set_error(PTRHASH_E_RANGE, "queue full");
    r.ticket = srv->next_ticket++;
    r.t_submit = arrival;
    *ticket = r.ticket;
    if (n_q == 0) {
        srv->finished[r.ticket] = 0.0;
        srv->completed++;
        srv->latencies.add(0.0);
        srv->cv_done.notify_all();
        return PTRHASH_OK;
    }
    srv->queued_keys += n_q;
    srv->outstanding.insert(r.ticket);
    srv->queue.push_back(r);
    srv->cv_work.notify_one();
    return PTRHASH_OK;
}

}  // extern "C"

extern "C" {

PTRHASH_API int ptrhash_server_submit(ptrhash_server *srv, ptrhash_handle *h, const uint64_t *keys, uint64_t n_q,
                                      void *out, uint64_t *ticket) {
    return submit_at(srv, h, keys, n_q, out, ticket, Clock::now(), false);
}

PTRHASH_API int ptrhash_server_submit_mapped(ptrhash_server *srv, ptrhash_handle *h, const uint64_t *keys,
                                             uint64_t n_q, void *out, uint64_t *ticket) {
    return submit_at(srv, h, keys, n_q, out, ticket, Clock::now(), true);
}

PTRHASH_API int ptrhash_host_alloc(uint64_t bytes, void **out) {
    if (!out || bytes == 0) return ptrhash::set_error(PTRHASH_E_INVAL, "NULL out or zero bytes");
    void *h = nullptr, *d = nullptr;
    hipError_t e = hipHostMalloc(&h, bytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) return ptrhash::set_error(PTRHASH_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    if ((e = hipHostGetDevicePointer(&d, h, 0)) != hipSuccess) {
        (void)hipHostFree(h);
        return ptrhash::set_error(PTRHASH_E_HIP, "hipHostGetDevicePointer: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> l(g_mapped_mu);
        g_mapped[reinterpret_cast<uintptr_t>(h)] = {reinterpret_cast<uintptr_t>(h) + bytes,
                                                    reinterpret_cast<uintptr_t>(d)};
    }
    *out = h;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_host_free(void *p) {
    if (!p) return PTRHASH_OK;
    {
        std::lock_guard<std::mutex> l(g_mapped_mu);
        auto it = g_mapped.find(reinterpret_cast<uintptr_t>(p));
        if (it == g_mapped.end()) return ptrhash::set_error(PTRHASH_E_INVAL, "not a ptrhash_host_alloc pointer");
        g_mapped.erase(it);
    }
    const hipError_t e = hipHostFree(p);
    return e == hipSuccess ? PTRHASH_OK : ptrhash::set_error(PTRHASH_E_HIP, "hipHostFree: %s", hipGetErrorString(e));
}

PTRHASH_API int ptrhash_server_wait(ptrhash_server *srv, uint64_t ticket, double *latency_us) {
    if (!srv) return ptrhash::set_error(PTRHASH_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lock(srv->mu);
    if (!srv->outstanding.count(ticket) && !srv->finished.count(ticket))
        return ptrhash::set_error(PTRHASH_E_INVAL, "unknown or already collected ticket");
    srv->cv_done.wait(lock, [&] { return srv->finished.count(ticket) || srv->error; });
    auto it = srv->finished.find(ticket);
    if (it == srv->finished.end()) return ptrhash::set_error(srv->error, "server stopped after an error");
    if (latency_us) *latency_us = it->second;
    srv->finished.erase(it);
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_server_stats(ptrhash_server *srv, ptrhash_server_metrics *st) {
    if (!srv || !st) return ptrhash::set_error(PTRHASH_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    st->completed = srv->completed;
    st->launches = srv->launches;
    st->keys = srv->keys_done;
    st->queued = srv->queue.size();
    std::vector<double> v(srv->latencies.v);
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) { return v.empty() ? 0.0 : v[std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5))]; };
    st->p50_us = pct(0.50);
    st->p99_us = pct(0.99);
    st->max_us = v.empty() ? 0.0 : v.back();
    std::vector<double> w(srv->waits.v);
    std::sort(w.begin(), w.end());
    auto wp = [&](double q) { return w.empty() ? 0.0 : w[std::min(w.size() - 1, (size_t)(q * (w.size() - 1) + 0.5))]; };
    st->wait_p50_us = wp(0.50);
    st->wait_p99_us = wp(0.99);
    st->slots_busy_max = (uint64_t)srv->busy_max;
    srv->spans.overlap(st->overlap_max, st->overlap_mean);
    return srv->error;
}

PTRHASH_API int ptrhash_server_reset_stats(ptrhash_server *srv) {
    if (!srv) return ptrhash::set_error(PTRHASH_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->latencies.clear();
    srv->waits.clear();
    srv->spans.clear();
    srv->busy_max = srv->busy_now;
    srv->completed = srv->launches = srv->keys_done = 0;
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_server_replay(ptrhash_server *srv, const ptrhash_server_request *reqs, uint64_t count,
                                      double *makespan_s) {
    if (!srv || (count && !reqs)) return ptrhash::set_error(PTRHASH_E_INVAL, "NULL argument");
    std::vector<uint64_t> tickets(count);
    const auto t0 = Clock::now();
    for (uint64_t i = 0; i < count; ++i) {
        const auto due = t0 + std::chrono::duration_cast<Clock::duration>(
                                  std::chrono::duration<double, std::micro>(reqs[i].arrival_us));
        while (Clock::now() < due) {
        }
        for (;;) {
            const int rc = submit_at(srv, reqs[i].handle, reqs[i].keys, reqs[i].n_q, reqs[i].out, &tickets[i], due,
                                     reqs[i].mapped != 0);
            if (rc == PTRHASH_OK) break;
            if (rc != PTRHASH_E_RANGE || reqs[i].n_q > srv->cfg.slot_keys) return rc;
            std::this_thread::yield();  // queue full: the open loop backs off
        }
    }
    for (uint64_t i = 0; i < count; ++i) {
        const int rc = ptrhash_server_wait(srv, tickets[i], nullptr);
        if (rc) return rc;
    }
    if (makespan_s) *makespan_s = std::chrono::duration<double>(Clock::now() - t0).count();
    return PTRHASH_OK;
}

PTRHASH_API int ptrhash_server_destroy(ptrhash_server *srv) {
    if (!srv) return PTRHASH_OK;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    for (Slot &s : srv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        free_slot(s);
    }
    const int err = srv->error;
    if (srv->base) (void)hipEventDestroy(srv->base);
    delete srv->pool;
    delete srv;
    return err;
}

}  // extern "C"
