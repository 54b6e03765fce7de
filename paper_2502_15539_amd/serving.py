"""Serving workload: many resident MPHFs, Poisson arrivals of query
batches of mixed sizes, continuous batching through ``ptrhash.Server``.

Workload: 64 MPHFs with n log-uniform in [1e4, 1e7] over uniform u64 keys
(Default parameters, u32 indices); requests target a uniformly chosen MPHF
with a batch of member keys (drawn with replacement) of size log-uniform in
[1, 65536]. The saturated request rate is measured first (every request
queued at t = 0), then open-loop Poisson arrivals at fractions of it; each
run reports p50/p99 latency (arrival -> indices delivered) and throughput.
The comparison is one plain one-key-per-lane launch per request on the same
GPU (keys copied in, one query, indices copied out, in arrival order).

Server configurations are swept over streams, launch size, copy threads,
zero-copy or copied arenas, and whether the requests' keys and outputs are
ordinary host arrays (copied by the server into its staging buffers) or
live in mapped pinned memory from ``ptrhash.HostBuffer`` (read and written
in place by the kernel); the fastest is used for the latency runs.

Before serving, the batched form alone is measured with every request's keys
already in device memory: one persistent multi-MPHF launch over up to 4096
requests (launch shape picked by the autotuner, also as a replayed HIP
graph) against one plain launch per request. The server then uses the
tuned launch shape.
"""
from __future__ import annotations

import time

import numpy as np

from . import keygen as K
from . import ptrhash as P


def build_fleet(count=64, lo=10**4, hi=10**7, seed=5, threads=0, single_mod=True, log=print):
    """count MPHFs with log-uniform sizes in [lo, hi], Default parameters:
    a list of (keys, resident Mphf, Built).
    single_mod: an MPHF that the parameter rule gives a single part uses the
    x mod S reduce with S ~ n/alpha (load ~0.99) instead of the next power of
    two (load down to ~0.5), which keeps its remap fraction near 1 %."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(np.log(lo) + rng.uniform(0, 1, size=count) * np.log(hi / lo)).astype(np.int64)
    preset = P.PRESET_DEFAULT | (P.PRESET_SINGLE_MOD if single_mod else 0)
    fleet = []
    t0 = time.time()
    for j, n in enumerate(sizes):
        keys = K.u64_keys(int(n), seed=1000 + j)
        b = P.build_u64(keys, index_bits=32, threads=threads, preset=preset)
        fleet.append((keys, P.Mphf.from_built(b), b))
    single = sum(1 for _, _, b in fleet if b.params.reduce_kind == P.REDUCE_MOD)
    log(f"[serve] built {count} MPHFs ({single} single-part with the mod reduce), {int(sizes.sum())} keys in "
        f"{time.time() - t0:.1f}s")
    return fleet


def make_requests(fleet, count, seed=6, max_size=65536, with_index=False):
    """count requests (Mphf, member keys drawn with replacement, u32 output
    array); with_index also returns each request's fleet index."""
    rng = np.random.default_rng(seed)
    reqs, js = [], []
    for _ in range(count):
        j = int(rng.integers(len(fleet)))
        keys, m = fleet[j][:2]
        size = min(max_size, max(1, int(np.exp(rng.uniform(0, np.log(max_size))))))
        q = keys[rng.integers(0, len(keys), size=size)]
        reqs.append((m, q, np.zeros(size, dtype=np.uint32)))
        js.append(j)
    return (reqs, js) if with_index else reqs


def poisson_arrivals(count, rate_per_s, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1e6 / rate_per_s, size=count))  # microseconds


def run_server(srv, reqs, arrivals, mapped=False):
    srv.reset_stats()
    span = srv.replay([(m, q, o, t) for (m, q, o), t in zip(reqs, arrivals)], mapped=mapped)
    st = srv.stats()
    keys = sum(len(q) for _, q, _ in reqs)
    return {"requests": len(reqs), "keys": keys, "makespan_s": span, "req_per_s": len(reqs) / span,
            "keys_per_s": keys / span, "p50_us": st["p50_us"], "p99_us": st["p99_us"], "max_us": st["max_us"],
            "wait_p50_us": st["wait_p50_us"], "wait_p99_us": st["wait_p99_us"], "launches": st["launches"],
            "slots_busy_max": st["slots_busy_max"], "device_overlap_max": st["overlap_max"],
            "device_overlap_mean": st["overlap_mean"]}


def run_plain_baseline(reqs, torch):
    """One plain one-key-per-lane launch per request, back to back."""
    lat = []
    outs = []
    t0 = time.perf_counter()
    for m, q, _ in reqs:
        a = time.perf_counter()
        m.set_kernel(P.KERNEL_PLAIN, 1, 256)
        qt = torch.from_numpy(q.view(np.int64)).to("cuda", non_blocking=False)
        o = m.query(qt)
        oh = o.cpu().numpy()
        lat.append((time.perf_counter() - a) * 1e6)
        outs.append(oh.view(np.uint32))
        m.set_kernel(P.KERNEL_PIPELINED, 4, 256)
    span = time.perf_counter() - t0
    keys = sum(len(q) for _, q, _ in reqs)
    lat = np.array(lat)
    return {"requests": len(reqs), "keys": keys, "makespan_s": span, "req_per_s": len(reqs) / span,
            "keys_per_s": keys / span, "p50_us": float(np.percentile(lat, 50)),
            "p99_us": float(np.percentile(lat, 99))}, outs


SERVER_CONFIGS = [  # (streams, slot_keys, copy_threads, zero_copy, mapped requests)
    (2, 1 << 22, 4, 0, 0), (4, 1 << 20, 8, 0, 0), (8, 1 << 20, 8, 0, 0),
    (2, 1 << 22, 4, 1, 0), (4, 1 << 20, 8, 1, 0), (8, 1 << 20, 8, 1, 0), (4, 1 << 18, 8, 1, 0),
    (4, 1 << 20, 12, 1, 0), (2, 1 << 22, 0, 1, 1), (4, 1 << 20, 0, 1, 1), (8, 1 << 20, 0, 1, 1),
]

# Launch shapes tried for the chosen server configuration (keys per lane,
# block, resident workgroups per CU; 0 = no cap). A zero-copy launch reads
# its keys over PCIe and may want more wavefronts in flight than the shape
# tuned on device-resident batches.
SERVER_SHAPES = [(2, 64, 0), (4, 64, 0), (8, 64, 0), (4, 128, 0), (8, 128, 0), (4, 256, 0)]


def mapped_copies(reqs):
    """The same requests with keys and outputs in one mapped pinned buffer
    (as a caller that produces its requests there would hold them)."""
    total = sum(len(q) * 8 + ((len(o) * o.itemsize + 7) // 8) * 8 for _, q, o in reqs)
    buf = P.HostBuffer(total)
    out = []
    off = 0
    for m, q, o in reqs:
        k = buf.view(off, len(q), np.uint64)
        k[:] = q
        off += len(q) * 8
        oo = buf.view(off, len(o), o.dtype)
        off += ((len(o) * o.itemsize + 7) // 8) * 8
        out.append((m, k, oo))
    return buf, out


def run_batched(torch, reqs, log=print, reps=5):
    """Device-resident batches: tuned multi-MPHF plan launch (and its graph
    replay) vs one plain launch per request. Returns (results, shape)."""
    from . import autotune

    reqs = reqs[:P.multi_max()]
    keys = sum(len(q) for _, q, _ in reqs)
    dev = [(m, torch.from_numpy(q.view(np.int64)).to("cuda"), torch.empty(len(q), dtype=torch.int32, device="cuda"))
           for m, q, _ in reqs]
    plan = P.MultiPlan(len(dev))
    shape, sweep = autotune.tune_multi(torch, plan, dev, use_cache=False)
    torch.cuda.synchronize()
    t_multi = autotune._time(torch, plan.launch, reps)
    multi_out = [o.clone() for _, _, o in dev]
    graph = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        plan.launch(stream)
    torch.cuda.synchronize()
    t_graph = autotune._time(torch, graph.replay, reps)

    def plain_all():
        for m, q, o in dev:
            m.query_into(q, o)

    for m, _, _ in dev:
        m.set_kernel(P.KERNEL_PLAIN, 1, 256)
    t_plain = autotune._time(torch, plain_all, max(1, reps // 2))
    for m, _, _ in dev:
        m.set_kernel(P.KERNEL_PIPELINED, 4, 256)
    agree = all(torch.equal(a, o) for a, (_, _, o) in zip(multi_out, dev))
    plan.close()
    res = {"requests": len(dev), "keys": keys, "multi_shape": {"keys_per_lane": shape[0], "block": shape[1],
                                                               "blocks_per_cu": shape[2]},
           "multi_ms": t_multi, "multi_keys_per_s": keys / t_multi * 1e3,
           "graph_replay_ms": t_graph, "plain_per_request_ms": t_plain, "plain_keys_per_s": keys / t_plain * 1e3,
           "speedup": t_plain / t_multi, "multi_equals_plain": agree,
           "shape_sweep_ms": {f"{c[0]}/{c[1]}/{c[2]}": v for c, v in sorted(sweep.items())}}
    log(f"[serve] batched on device: {len(dev)} requests, {keys} keys: multi launch {t_multi:.3f} ms "
        f"({keys / t_multi / 1e6:.1f} G keys/s, shape {shape}), graph replay {t_graph:.3f} ms, "
        f"plain per request {t_plain:.3f} ms ({t_plain / t_multi:.1f}x), agree={agree}")
    return res, shape


def run_c5(torch, n_requests=20000, loads=(0.25, 0.5, 0.8, 1.0, 1.2), threads=0, log=print):
    fleet = build_fleet(threads=threads, log=log)
    reqs = make_requests(fleet, n_requests)
    batched, shape = run_batched(torch, reqs, log=log)
    # pick the server configuration by its saturated rate (everything queued at t = 0)
    buf, mreqs = mapped_copies(reqs)
    tried = {}
    for streams, slot, copiers, zc, mp in SERVER_CONFIGS:
        rq = mreqs if mp else reqs
        srv = P.Server(streams=streams, max_batches=1024, slot_keys=slot, max_queued_keys=1 << 31,
                       copy_threads=copiers, zero_copy=zc, multi_kernel=shape)
        run_server(srv, rq[:500], np.zeros(500), mp)
        r = run_server(srv, rq, np.zeros(len(rq)), mp)
        # latency at a light open-loop load (25 % of this configuration's saturated rate)
        light = run_server(srv, rq[:5000], poisson_arrivals(5000, 0.25 * r["req_per_s"], seed=99), mp)
        r["light_p50_us"], r["light_p99_us"] = light["p50_us"], light["p99_us"]
        tried[(streams, slot, copiers, zc, mp)] = r
        log(f"[serve] config streams={streams} slot={slot} copiers={copiers} zero_copy={zc} mapped={mp}: "
            f"{r['req_per_s']:.0f} req/s {r['keys_per_s'] / 1e9:.2f} G keys/s launches={r['launches']} "
            f"light-load p50 {light['p50_us']:.0f}us p99 {light['p99_us']:.0f}us")
        srv.close()
    best_copied = max((c for c in tried if not c[4]), key=lambda c: tried[c]["req_per_s"])
    best = max(tried, key=lambda c: tried[c]["req_per_s"])
    streams, slot, copiers, zc, mp = best
    sat = tried[best]
    rq = mreqs if mp else reqs
    # then its launch shape, by the saturated rate again (and the light-load
    # latency of a new winner)
    shape_rates = {tuple(shape): sat["req_per_s"]}
    for sh in SERVER_SHAPES:
        if sh in shape_rates:
            continue
        srv = P.Server(streams=streams, max_batches=1024, slot_keys=slot, max_queued_keys=1 << 31,
                       copy_threads=copiers, zero_copy=zc, multi_kernel=sh)
        run_server(srv, rq[:500], np.zeros(500), mp)
        r = run_server(srv, rq, np.zeros(len(rq)), mp)
        if r["req_per_s"] > sat["req_per_s"]:
            light = run_server(srv, rq[:5000], poisson_arrivals(5000, 0.25 * r["req_per_s"], seed=99), mp)
            r["light_p50_us"], r["light_p99_us"] = light["p50_us"], light["p99_us"]
            sat = r
        srv.close()
        shape_rates[sh] = r["req_per_s"]
        log(f"[serve] launch shape {sh}: {r['req_per_s']:.0f} req/s {r['keys_per_s'] / 1e9:.2f} G keys/s")
    served_shape = max(shape_rates, key=shape_rates.get)
    srv = P.Server(streams=streams, max_batches=1024, slot_keys=slot, max_queued_keys=1 << 31,
                   copy_threads=copiers, zero_copy=zc, multi_kernel=served_shape)
    run_server(srv, rq[:500], np.zeros(500), mp)
    log(f"[serve] saturated: {sat['req_per_s']:.0f} req/s, {sat['keys_per_s'] / 1e9:.2f} G keys/s")
    runs = []
    for i, f in enumerate(loads):
        rate = f * sat["req_per_s"]
        arr = poisson_arrivals(len(rq), rate, seed=100 + i)
        r = run_server(srv, rq, arr, mp)
        r["offered_fraction"] = f
        r["offered_req_per_s"] = rate
        runs.append(r)
        log(f"[serve] load {f:.2f}: {r['req_per_s']:.0f} req/s p50 {r['p50_us']:.0f}us p99 {r['p99_us']:.0f}us "
            f"(wait p50 {r['wait_p50_us']:.0f}us p99 {r['wait_p99_us']:.0f}us) launches={r['launches']} "
            f"slots busy <= {r['slots_busy_max']}, on the device <= {r['device_overlap_max']} at once "
            f"({r['device_overlap_mean']:.2f} on average)")
    srv.close()
    served = [o.copy() for _, _, o in rq]
    buf.close()
    base, base_out = run_plain_baseline(reqs[:2000], torch)
    agree = all(np.array_equal(a, b) for a, b in zip(served[:2000], base_out))
    log(f"[serve] plain per-request baseline: {base['req_per_s']:.0f} req/s p50 {base['p50_us']:.0f}us "
        f"agree={agree}")
    return {"batched_on_device": batched, "saturated": sat, "open_loop": runs, "plain_per_request": base,
            "served_equals_plain": agree,
            "mphfs": len(fleet), "resident_keys": int(sum(len(f[0]) for f in fleet)),
            "server_config": {"streams": streams, "slot_keys": slot, "copy_threads": copiers, "zero_copy": zc,
                              "mapped_requests": mp, "max_batches": 1024, "multi_shape": list(served_shape)},
            "server_shape_sweep_req_per_s": {f"{k[0]}/{k[1]}/{k[2]}": v for k, v in shape_rates.items()},
            "saturated_copied_requests": tried[best_copied],
            "config_sweep": {f"streams={c[0]},slot={c[1]},copiers={c[2]},zero_copy={c[3]},mapped={c[4]}":
                             {"req_per_s": v["req_per_s"], "keys_per_s": v["keys_per_s"],
                              "light_p50_us": v["light_p50_us"], "light_p99_us": v["light_p99_us"]}
                             for c, v in tried.items()}}
