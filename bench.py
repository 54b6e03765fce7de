#!/usr/bin/env python3
"""Benchmark: PtrHash queries on one MI355X.

Default workload (one "step" = one pass of the query path over the whole
stream): n = 10^9 distinct uniform u64 keys, Default parameters (cubic
bucket function, lambda 3.5, alpha 0.99, CacheLineEF remap), a seeded
shuffled stream of all 10^9 members resident in HBM, u64 indices out.

Prints ONE JSON line with queries/s, ns/key, the fraction of a measured
random-gather roofline (the same memory pattern with no hashing), the HBM
roofline of the query kernel, and the CPU oracle timed on a bounded sample.
Other workloads (--workload): the Fast, Compact and non-minimal variants at
10^9, the 10^8 and 10^6 u64 sets, 3*10^8 byte strings, a cache-resident
single-part MPHF queried 10^9 times (mod or power-of-two slot reduce), one
multi-MPHF launch over 4096 device-resident requests, and the 64-MPHF
serving workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector-ALU issue peak: 256 CUs x 4 SIMDs x 2.4e9 cycles/s, one wave64
# instruction per SIMD every 4 cycles (16 lanes per cycle).
VALU_PEAK_GINSTS = 256 * 4 * 2.4 / 4
METRIC = "queries/s (ns/key) at n=1e9 u64 keys; % of random-gather HBM roofline"

WORKLOADS = {
    # name: (n, key kind, index bits, description)
    "u64_1e9": (10**9, "u64", 64, "n=1e9 distinct uniform u64 keys (SplitMix64), shuffled stream of all 1e9 "
                                  "members, u64 indices, Default params (gamma_3, lambda=3.5, alpha=0.99, "
                                  "CacheLineEF remap)"),
    "u64_1e9_fast": (10**9, "u64", 64, "n=1e9 distinct uniform u64 keys, shuffled stream of all members, u64 "
                                       "indices, Fast params (gamma_1, lambda=3.0, alpha=0.99, plain u32 remap)"),
    "u64_1e9_compact": (10**9, "u64", 64, "n=1e9 distinct uniform u64 keys, shuffled stream of all members, u64 "
                                          "indices, Compact params (gamma_3, lambda=4.0, alpha=0.99, CacheLineEF)"),
    "u64_1e9_phf": (10**9, "u64", 64, "n=1e9 distinct uniform u64 keys, shuffled stream of all members, u64 "
                                      "slots (non-minimal: no remap), Default params"),
    "u64_1e8": (10**8, "u64", 32, "n=1e8 distinct uniform u64 keys, shuffled stream of all members, u32 indices, "
                                  "Default params"),
    "u64_1e6": (10**6, "u64", 32, "n=1e6 distinct uniform u64 keys, shuffled stream of all members, u32 indices, "
                                  "Default params"),
    "bytes_3e8": (3 * 10**8, "bytes", 32, "n=3e8 distinct random byte strings, length uniform 10-50 over printable "
                                          "ASCII, packed with u64 offsets; shuffled stream of all members, u32 "
                                          "indices, Default params"),
    "u64_1e5_cached_mod": (10**5, "cached", 32, "n=1e5 distinct uniform u64 keys in one part with the x mod S "
                                                 "reduce (S=101011), 1e9 queries: the shuffled member stream "
                                                 "repeated 1e4 times, u32 indices, Default params; the MPHF stays "
                                                 "cache-resident"),
    "u64_1e5_cached_pow2": (10**5, "cached", 32, "n=1e5 distinct uniform u64 keys in one part of S=2^17 slots "
                                                  "(power-of-two reduce), 1e9 queries: the shuffled member stream "
                                                  "repeated 1e4 times, u32 indices, Default params; the MPHF stays "
                                                  "cache-resident"),
    "multi_c5": (0, "multi", 32, "4096 requests against the 64-MPHF serving fleet (n log-uniform in [1e4, 1e7] u64 "
                                 "keys, Default params, the single-part ones with the x mod S reduce; batch sizes "
                                 "log-uniform in [1, 65536], 24.1M member keys drawn with replacement), resident in "
                                 "HBM, all answered by one multi-MPHF launch per step"),
    "bytes_3e8_h128": (3 * 10**8, "bytes", 32, "as bytes_3e8, with the 128-bit string hash that the parameter rule "
                                               "takes beyond 2^32 keys (high half: part and bucket, low half: "
                                               "slot) forced on"),
    "serve_c5": (0, "serve", 32, "64 resident MPHFs, n log-uniform in [1e4, 1e7] u64 keys, Default params (the "
                                 "23 that get one part use the x mod S reduce); "
                                 "Poisson arrivals of batches log-uniform in [1, 65536] keys, each against one "
                                 "MPHF; continuous batching"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="u64_1e9", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel", default="auto",
                    help="auto | plain | K,BLOCK[,BLOCKS_PER_CU] (pipelined; occupancy cap 0 = none)")
    ap.add_argument("--gather", default="auto", help="auto | K,BLOCK[,BLOCKS_PER_CU] for the gather roofline")
    ap.add_argument("--cpu-sample", type=int, default=200_000_000, help="oracle sample size (keys); 0 = skip")
    ap.add_argument("--threads", type=int, default=0, help="host threads for the build (0 = all, max 16)")
    ap.add_argument("--requests", type=int, default=20000, help="serving workload: requests per run")
    return ap.parse_args()


def host_cpu():
    """Host threads the CPU baselines use and what the host offers: the
    threads this process may run on (its affinity mask), capped at the CPU
    share of one GPU on a shared box (OMP_NUM_THREADS, else 16), plus nproc
    and the CPU model."""
    affinity = len(os.sched_getaffinity(0))
    share = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"threads": max(1, min(affinity, share)), "affinity_cpus": affinity, "nproc": os.cpu_count(),
            "omp_num_threads": share, "cpu_model": model}


def time_launches(torch, fn, steps, warmup):
    """Average duration of fn() (one kernel launch) on torch's current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps  # ms


def kernel_candidates(P, spec, bytes_keys=False):
    from paper_2502_15539_amd import autotune

    if spec == "plain":
        return [(P.KERNEL_PLAIN, 1, 256, 0)]
    if spec != "auto":
        v = [int(x) for x in spec.split(",")]
        return [(P.KERNEL_PIPELINED, v[0], v[1], v[2] if len(v) > 2 else 0)]
    return autotune.candidates_for(P.KEY_BYTES if bytes_keys else P.KEY_U64)


def tune_and_time(torch, P, mphf, run, args, n_q, bytes_keys=False):
    """Autotune the kernel choice (keys per lane, block, occupancy cap), then
    time exactly args.steps launches."""
    from paper_2502_15539_amd import autotune

    best, sweep = autotune.tune(torch, mphf, run, n_q, cands=kernel_candidates(P, args.kernel, bytes_keys),
                                use_cache=False)
    log("[bench] sweep (kernel/keys-per-lane/block/occupancy): " +
        ", ".join(f"{c[0]}/{c[1]}/{c[2]}/{c[3]}={v:.3f}ms" for c, v in sorted(sweep.items())))
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        run()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    return best, sweep, ev0.elapsed_time(ev1) / args.steps, wall


def bijective(torch, out, n):
    seen = torch.zeros(n, dtype=torch.bool, device=out.device)
    o64 = out.long()
    ok = int(o64.min()) >= 0 and int(o64.max()) < n
    seen[o64] = True
    return bool(ok and seen.all())


def kernel_name(P, best):
    if best[0] == P.KERNEL_PLAIN:
        return "plain"
    occ = f",blocks_per_cu<={best[3]}" if best[3] else ""
    return f"pipelined(keys_per_lane={best[1]},block={best[2]}{occ})"


def profiled_traffic(workload, ms, n):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload, if the kernel sources still match the ones profiled."""
    from paper_2502_15539_amd import profsum

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None, None
    t = json.load(open(path))
    if t.get("kernel_source_sha256") != profsum.kernel_source_hash():
        return None, {"stale_profile": os.path.relpath(path, ROOT)}
    b = t["traffic_bytes_per_launch"]
    info = {"level": t.get("level", ""), "traffic_GBps": b / (ms / 1e3) / 1e9,
            "traffic_frac_of_peak": b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, "traffic_bytes_per_key": b / n,
            "read_bytes": t.get("read_bytes"), "write_bytes": t.get("write_bytes"),
            "memory_read_bytes": t.get("memory_read_bytes"),
            "fetch_size_check": (t.get("fetch_size_check") or {}).get("fetch_bytes_scaled"),
            "profiled_kernel": t.get("kernel"), "source": os.path.relpath(path, ROOT)}
    return b, info


def profiled_valu(workload, ms, kernel):
    """Vector-ALU roofline of the query kernel from the committed rocprofv3
    counter summary of this workload (instructions per launch, counted per
    wavefront), if the kernel sources still match the ones profiled and the
    profiled kernel takes as many keys per lane as the timed one (the count
    depends on that, not on the workgroup size)."""
    from paper_2502_15539_amd import profsum

    path = os.path.join(ROOT, "profiles", f"valu_{workload}.json")
    roof = {"bound": "alu", "achieved": None, "peak": VALU_PEAK_GINSTS, "unit": "G wave64 VALU instructions/s",
            "frac": None, "traffic": None}
    if not os.path.exists(path):
        return roof
    t = json.load(open(path))
    if t.get("kernel_source_sha256") != profsum.kernel_source_hash():
        roof["stale_profile"] = os.path.relpath(path, ROOT)
        return roof
    if t.get("kernel") != kernel:
        roof["profiled_kernel"] = t.get("kernel")
        return roof
    achieved = t["valu_insts_per_launch"] / (ms / 1e3) / 1e9
    roof.update(achieved=achieved, frac=achieved / VALU_PEAK_GINSTS, valu_insts_per_launch=t["valu_insts_per_launch"],
                valu_busy_pct_profiled=t["valu_busy_pct"], valu_utilization_pct_profiled=t["valu_utilization_pct"],
                source=os.path.relpath(path, ROOT))
    return roof


def record(args, n, ms, wall, desc, extra_config, dtype, per_key, **fields):
    achieved = per_key * n / (ms / 1e3) / 1e9
    traffic, tinfo = profiled_traffic(args.workload, ms, n)
    rec = {
        "metric": METRIC,
        "value": n / (ms / 1e3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded SplitMix64 keys, Feistel-shuffled member stream)",
        "config": {"workload": desc, "n": n, **extra_config, "parallelism": "single GPU"},
        "ns_per_key": ms * 1e6 / n,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_key": per_key,
                     "traffic_info": tinfo},
        "timed_wall_s": wall,
    }
    rec.update(fields)
    return rec


def remap_fraction(torch, P, params, pilots, queries=None, data=None, offsets=None):
    """Fraction of member queries whose slot is >= n (non-minimal view of the same pilots)."""
    phf = P.Mphf()
    pp = params.copy()
    pp.remap_kind = P.REMAP_NONE
    pp.index_bits = 64
    phf.load(pp, pilots, None)
    slots = phf.query(queries) if queries is not None else phf.query_bytes(data, offsets)
    frac = float((slots >= params.n).sum().item()) / params.n
    phf.close()
    return frac


def oracle_mphf(P, p, built):
    """The oracle's view of a built MPHF (same parameters, pilots and remap)."""
    from oracle import oracle as O

    if p.reduce_kind == P.REDUCE_MOD:
        op = O.params_single_mod(p.n, S=p.slots, B=p.buckets_per_part, gamma=p.gamma, seed=p.seed)
    else:
        op = O.params_explicit(p.n, p.num_parts, p.log2_slots, p.buckets_per_part, gamma=p.gamma, seed=p.seed)
    return O.Mphf(op, built.pilots, None, built.remap, None)


def oracle_baseline(args, p, built, q, out, bits, n, P=None):
    """The oracle's plain query loop on the first args.cpu_sample queries of the
    same stream and MPHF: once on one thread, once split over the host's cores
    (one slice per thread; the C loop runs outside the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_2502_15539_amd import ptrhash as PH

    ns = min(args.cpu_sample, len(q))
    qs = q[:ns].cpu().numpy().view(np.uint64)
    m = oracle_mphf(P or PH, p, built)
    one = qs[: max(1, ns // 4)]
    c0 = time.perf_counter()
    O.query_u64(m, one, O.REMAP_CLEF)
    single = (time.perf_counter() - c0) / len(one)
    host = host_cpu()
    cores = host["threads"]
    chunks = np.array_split(qs, cores)
    c0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        parts = list(ex.map(lambda c: O.query_u64(m, c, O.REMAP_CLEF), chunks))
    cdt = time.perf_counter() - c0
    res = np.concatenate(parts)
    go = out[:ns].cpu().numpy()
    go = go.view(np.uint64) if bits == 64 else go.view(np.uint32).astype(np.uint64)
    cpu = {"value": ns / cdt, "unit": "queries/s", "cores": cores, "kind": "oracle", "ns_per_key": cdt / ns * 1e9,
           "sample": f"first {ns} queries of the same shuffled stream on the same MPHF, the C oracle's plain query "
                     f"loop on {cores} threads (one slice each)",
           "single_thread_ns_per_key": single * 1e9, "single_thread_sample": len(one), "host": host,
           "matches_gpu": bool(np.array_equal(res, go))}
    log(f"[bench] cpu oracle: {cores} threads {cdt / ns * 1e9:.2f} ns/key, one thread {single * 1e9:.1f} ns/key, "
        f"matches_gpu={cpu['matches_gpu']}")
    return cpu


def oracle_baseline_bytes(args, p, built, qd, qo, out, n):
    """As oracle_baseline, for byte-string keys: the first queries of the
    same shuffled string stream (at most 5*10^7 of them)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    ns = min(args.cpu_sample, n, 50_000_000)
    offs = qo[:ns + 1].cpu().numpy().view(np.uint64)
    data = qd[:int(offs[-1]) + 64].cpu().numpy()
    op = O.params_explicit(p.n, p.num_parts, p.log2_slots, p.buckets_per_part, gamma=p.gamma, seed=p.seed)
    op.hash_bits = p.hash_bits or 64
    m = O.Mphf(op, built.pilots, None, built.remap, None)

    def run(lo, hi):
        o = offs[lo:hi + 1]
        return O.query_bytes(m, data[int(o[0]):int(o[-1]) + 64], o - o[0], O.REMAP_CLEF)

    one = max(1, ns // 4)
    c0 = time.perf_counter()
    run(0, one)
    single = (time.perf_counter() - c0) / one
    host = host_cpu()
    cores = host["threads"]
    bounds = np.linspace(0, ns, cores + 1).astype(np.int64)
    c0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        parts = list(ex.map(lambda i: run(int(bounds[i]), int(bounds[i + 1])), range(cores)))
    cdt = time.perf_counter() - c0
    res = np.concatenate(parts)
    go = out[:ns].cpu().numpy().view(np.uint32).astype(np.uint64)
    cpu = {"value": ns / cdt, "unit": "queries/s", "cores": cores, "kind": "oracle", "ns_per_key": cdt / ns * 1e9,
           "sample": f"first {ns} strings of the same shuffled stream on the same MPHF, the C oracle's plain query "
                     f"loop on {cores} threads (one slice each)",
           "single_thread_ns_per_key": single * 1e9, "single_thread_sample": one, "host": host,
           "matches_gpu": bool(np.array_equal(res, go))}
    log(f"[bench] cpu oracle: {cores} threads {cdt / ns * 1e9:.2f} ns/key, one thread {single * 1e9:.1f} ns/key, "
        f"matches_gpu={cpu['matches_gpu']}")
    return cpu


def run_u64(args, torch, K, P):
    n, _, bits, desc = WORKLOADS[args.workload]
    dev = "cuda"
    threads = args.threads or min(16, os.cpu_count() or 1)
    t0 = time.time()
    # the key set is generated in HBM; construction hashes and sorts it and
    # runs the pilot search on the device
    keys = P.gen_u64_keys(torch.empty(n, dtype=torch.int64, device=dev), K.KEY_SEED)
    torch.cuda.synchronize()
    t1 = time.time()
    preset = {"u64_1e9_fast": P.PRESET_FAST, "u64_1e9_compact": P.PRESET_COMPACT}.get(args.workload,
                                                                                      P.PRESET_DEFAULT)
    log(f"[bench] keygen {time.time() - t0:.1f}s; building the MPHF")
    built = P.build_u64_device(keys, index_bits=bits, threads=threads, preset=preset)
    t2 = time.time()
    del keys
    torch.cuda.empty_cache()
    if args.workload == "u64_1e9_phf":  # same pilots, queried without the remap
        built.params.remap_kind = P.REMAP_NONE
        built.remap = np.zeros(0, dtype=np.uint8)
    p = built.params
    log(f"[bench] keygen {t1 - t0:.1f}s build {t2 - t1:.1f}s ({built.placement} search)  P={p.num_parts} S=2^{p.log2_slots} "
        f"B={p.buckets_per_part} bits/key={built.bits_per_key:.3f} evictions={built.info.evictions}")
    mphf = P.Mphf.from_built(built)

    q = torch.empty(n, dtype=torch.int64, device=dev)
    P.gen_query_stream(q, n, K.KEY_SEED, K.ORDER_SEED)
    out = torch.empty(n, dtype=torch.int64 if bits == 64 else torch.int32, device=dev)
    torch.cuda.synchronize()

    best, sweep, ms, wall = tune_and_time(torch, P, mphf, lambda: mphf.query_into(q, out), args, n)
    bij = bijective(torch, out, n) if p.remap_kind != P.REMAP_NONE else bool(int(out.max()) < p.num_parts << p.log2_slots)
    rfrac = remap_fraction(torch, P, p, built.pilots, queries=q)

    # roofline microbenchmarks on the same key stream
    table = torch.randint(0, 256, (p.num_parts * p.buckets_per_part,), dtype=torch.uint8, device=dev)
    gout = torch.empty(n, dtype=torch.int64, device=dev)
    # tuned over the same knobs as the query (keys per lane, block, occupancy cap)
    from paper_2502_15539_amd import autotune

    gcands = [(k, b, o) for k in autotune.DEFAULT_KPL for b in autotune.DEFAULT_BLOCKS
              for o in autotune.DEFAULT_OCCUPANCY]
    if args.gather != "auto":
        g = tuple(int(x) for x in args.gather.split(","))
        gcands = [g if len(g) == 3 else g + (0,)]
    gsweep = {c: time_launches(torch, lambda: P.bench_gather(q, table, gout, c[0], c[1], c[2]), 3, 1)
              for c in gcands}
    gbest = min(gsweep, key=gsweep.get)
    gather_ms = gsweep[gbest]
    # like-for-like: the same pilot table read at each key's own bucket (the
    # cubic bucket function's skew included), no slot hash, no remap
    bsweep = {c: time_launches(torch, lambda: P.bench_gather_buckets(mphf, q, gout, c[0], c[1], c[2]), 3, 1)
              for c in gcands}
    bbest = min(bsweep, key=bsweep.get)
    bucket_ms = bsweep[bbest]
    copy_ms = min(time_launches(torch, lambda: P.bench_copy(q, gout, k, 256), 3, 1) for k in (1, 4, 8))
    del gout, table
    log(f"[bench] query {ms:.3f} ms  gather-roofline {gather_ms:.3f} ms {gbest}  own-bucket gather {bucket_ms:.3f} "
        f"ms {bbest}  copy {copy_ms:.3f} ms  bijective={bij} remap_frac={rfrac:.5f}")

    cpu = None
    if args.cpu_sample and p.remap_kind == P.REMAP_CLEF and p.gamma == P.GAMMA_CUBIC:
        cpu = oracle_baseline(args, p, built, q, out, bits, n)

    remap_line = {P.REMAP_CLEF: 64, P.REMAP_U32: 4, P.REMAP_NONE: 0}[p.remap_kind]
    per_key = 8 + bits // 8 + 1 + rfrac * remap_line
    rec = record(args, n, ms, wall, desc,
                 {"kernel": kernel_name(P, best), "index_bits": bits, "num_parts": p.num_parts,
                  "log2_slots": p.log2_slots, "buckets_per_part": p.buckets_per_part,
                  "bits_per_key": round(built.bits_per_key, 4)},
                 "u64", per_key,
                 pct_gather_roofline=100.0 * gather_ms / ms,
                 gather_roofline={"ms": gather_ms, "ns_per_key": gather_ms * 1e6 / n, "keys_per_lane": gbest[0],
                                  "block": gbest[1], "blocks_per_cu": gbest[2],
                                  "table_bytes": p.num_parts * p.buckets_per_part,
                                  "index": "uniform hi(key * T) over a table of the pilot array's size"},
                 pct_bucket_gather_roofline=100.0 * bucket_ms / ms,
                 bucket_gather_roofline={"ms": bucket_ms, "ns_per_key": bucket_ms * 1e6 / n,
                                         "keys_per_lane": bbest[0], "block": bbest[1], "blocks_per_cu": bbest[2],
                                         "index": "each key's own global bucket in the MPHF's pilot array (same "
                                                  "hash, part and bucket function as the query; no slot hash, "
                                                  "no remap)"},
                 stream_copy_ms=copy_ms,
                 plain_kernel_ms=sweep.get((P.KERNEL_PLAIN, 1, 256, 0)),
                 cpu_baseline=cpu,
                 parity={"bijective_members": bij, "remap_fraction": rfrac},
                 build_s=t2 - t1, build_search=built.placement,
                 paper_cpu_context_ns_per_key={"loop": 12, "stream": 8, "default_clef_loop": 21.0,
                                               "default_clef_stream": 8.7})
    if args.workload != "u64_1e9":
        rec["metric"] = f"queries/s (ns/key) at n={n:.0e} u64 keys"
    return rec, bij and (cpu is None or cpu["matches_gpu"])


def run_cached(args, torch, K, P):
    """A small single-part MPHF queried 10^9 times: its pilots and remap stay in
    the caches, so the time is the kernel's arithmetic plus the key and index
    streams. The _mod and _pow2 workloads differ only in the slot reduce."""
    n, _, bits, desc = WORKLOADS[args.workload]
    dev = "cuda"
    reps = 10**4
    n_q = n * reps
    keys = P.gen_u64_keys(torch.empty(n, dtype=torch.int64, device=dev), K.KEY_SEED)
    mod = args.workload.endswith("_mod")
    params = P.params_default(n, P.PRESET_DEFAULT | (P.PRESET_SINGLE_MOD if mod else 0), index_bits=bits)
    t1 = time.time()
    built = P.build_u64_device(keys, params=params)
    t2 = time.time()
    p = built.params
    assert p.num_parts == 1 and (p.reduce_kind == P.REDUCE_MOD) == mod
    log(f"[bench] build {t2 - t1:.2f}s ({built.placement} search) S={p.slots_per_part} B={p.buckets_per_part} "
        f"reduce={'mod' if mod else 'pow2'} bits/key={built.bits_per_key:.3f}")
    mphf = P.Mphf.from_built(built)
    period = torch.empty(n, dtype=torch.int64, device=dev)
    P.gen_query_stream(period, n, K.KEY_SEED, K.ORDER_SEED)
    q = period.repeat(reps)
    out = torch.empty(n_q, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    best, sweep, ms, wall = tune_and_time(torch, P, mphf, lambda: mphf.query_into(q, out), args, n_q)
    head = out[:n]
    bij = bijective(torch, head, n)
    periodic = bool((out.view(reps, n) == head).all())
    gout = torch.empty(n_q, dtype=torch.int64, device=dev)
    copy_ms = min(time_launches(torch, lambda: P.bench_copy(q, gout, k, 256), 3, 1) for k in (1, 4, 8))
    del gout
    log(f"[bench] query {ms:.3f} ms  copy (16 B/key) {copy_ms:.3f} ms  bijective={bij} periodic={periodic}")

    from oracle import oracle as O

    want = O.query_u64(oracle_mphf(P, p, built), period.cpu().numpy().view(np.uint64), O.REMAP_CLEF)
    first = bool(np.array_equal(head.cpu().numpy().view(np.uint32).astype(np.uint64), want))
    cpu = oracle_baseline(args, p, built, q, out, bits, n_q, P) if args.cpu_sample else None
    per_key = 8 + bits // 8  # key in, index out; the tables are served by the caches
    rec = record(args, n_q, ms, wall, desc,
                 {"kernel": kernel_name(P, best), "index_bits": bits, "keys": n, "num_slots": p.slots_per_part,
                  "reduce": "mod" if mod else "pow2", "buckets_per_part": p.buckets_per_part,
                  "bits_per_key": round(built.bits_per_key, 4)},
                 "u64", per_key,
                 stream_copy_ms=copy_ms,
                 plain_kernel_ms=sweep.get((P.KERNEL_PLAIN, 1, 256, 0)),
                 cpu_baseline=cpu,
                 parity={"bijective_members": bij, "every_period_equal": periodic,
                         "first_period_equals_oracle": first},
                 build_s=t2 - t1, build_search=built.placement)
    # the tables are cache-resident and the streams take 12 B/key: the kernel's
    # vector arithmetic bounds it, so the roofline is the VALU issue rate
    rec["stream_roofline"] = rec["roofline"]
    timed = f"query_pipelined<{best[1]}, unsigned int>" if best[0] == P.KERNEL_PIPELINED else "query_plain"
    rec["roofline"] = profiled_valu(args.workload, ms, timed)
    rec["metric"] = f"queries/s (ns/key): 1e9 queries against a cache-resident n=1e5 MPHF ({rec['config']['reduce']} reduce)"
    return rec, bij and periodic and first and (cpu is None or cpu["matches_gpu"])


def run_bytes(args, torch, K, P):
    n, _, bits, desc = WORKLOADS[args.workload]
    threads = args.threads or min(16, os.cpu_count() or 1)
    t0 = time.time()
    # the key set is generated in HBM and built there (hash, sort and pilot
    # search on the device)
    d_data, d_off = P.gen_strings(n, K.KEY_SEED)
    torch.cuda.synchronize()
    t1 = time.time()
    params = None
    if args.workload.endswith("_h128"):
        params = P.params_default(n, P.PRESET_DEFAULT, key_kind=P.KEY_BYTES, index_bits=bits)
        params.hash_bits = 128
    built = P.build_bytes_device(d_data, d_off, params=params, index_bits=bits, threads=threads)
    t2 = time.time()
    total_bytes = int(d_off[-1].item())
    del d_data, d_off
    torch.cuda.empty_cache()
    p = built.params
    log(f"[bench] strings {t1 - t0:.1f}s ({total_bytes / n:.1f} B/key) build {t2 - t1:.1f}s ({built.placement} "
        f"search) P={p.num_parts} bits/key={built.bits_per_key:.3f} seed={p.seed}")
    mphf = P.Mphf.from_built(built)
    qd, qo = P.gen_strings(n, K.KEY_SEED, K.ORDER_SEED, shuffled=True)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    mphf.query_bytes_into(qd, qo, out)  # checks once that the strings end 64 bytes before the buffer does
    best, sweep, ms, wall = tune_and_time(torch, P, mphf, lambda: mphf.query_bytes_into(qd, qo, out, check_end=False),
                                          args, n, bytes_keys=True)
    bij = bijective(torch, out, n)
    rfrac = remap_fraction(torch, P, p, built.pilots, data=qd, offsets=qo)
    per_key = total_bytes / n + 8 + 4 + 1 + rfrac * 64
    # string-stream roofline: the same offsets, string words and u32 index
    # streams and one pilot byte per key, with the hash reduced to a xor fold
    from paper_2502_15539_amd import autotune

    gout = torch.empty(n, dtype=torch.int32, device="cuda")
    gcands = [(k, b, o) for k in (1, 2, 4) for b in autotune.DEFAULT_BLOCKS for o in autotune.DEFAULT_OCCUPANCY]
    if args.gather != "auto":
        g = tuple(int(x) for x in args.gather.split(","))
        gcands = [g if len(g) == 3 else g + (0,)]
    gsweep = {c: time_launches(torch, lambda: P.bench_gather_bytes(mphf, qd, qo, gout, c[0], c[1], c[2]), 3, 1)
              for c in gcands}
    gbest = min(gsweep, key=gsweep.get)
    gather_ms = gsweep[gbest]
    del gout
    log(f"[bench] query {ms:.3f} ms  string-stream gather roofline {gather_ms:.3f} ms {gbest}  bijective={bij}")
    cpu = oracle_baseline_bytes(args, p, built, qd, qo, out, n) if args.cpu_sample else None
    rec = record(args, n, ms, wall, desc,
                 {"kernel": kernel_name(P, best), "index_bits": bits, "num_parts": p.num_parts,
                  "bits_per_key": round(built.bits_per_key, 4), "mean_key_bytes": total_bytes / n},
                 "u64", per_key,
                 plain_kernel_ms=sweep.get((P.KERNEL_PLAIN, 1, 256, 0)),
                 pct_gather_roofline=100.0 * gather_ms / ms,
                 gather_roofline={"ms": gather_ms, "ns_per_key": gather_ms * 1e6 / n, "keys_per_lane": gbest[0],
                                  "block": gbest[1], "blocks_per_cu": gbest[2],
                                  "index": "string-stream gather: offsets, the string words and the u32 index "
                                           "streamed, one pilot byte at the bucket of a xor fold of the words"},
                 cpu_baseline=cpu,
                 parity={"bijective_members": bij, "remap_fraction": rfrac}, build_s=t2 - t1,
                 build_search=built.placement,
                 paper_cpu_context_ns_per_key={"default_clef_loop": 37, "default_clef_stream": 23})
    rec["config"]["hash_bits"] = p.hash_bits or 64
    rec["metric"] = "queries/s (ns/key) at n=3e8 byte-string keys"
    return rec, bij and (cpu is None or cpu["matches_gpu"])


def run_multi(args, torch, K, P):
    """One multi-MPHF launch over 4096 device-resident requests (each against
    its own resident MPHF) per step, with the launch shape the autotuner
    picks; parity: equal to one plain query per request and to the oracle on
    every request."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_2502_15539_amd import autotune, serving

    threads = args.threads or min(16, os.cpu_count() or 1)
    fleet = serving.build_fleet(threads=threads, log=log)
    reqs, js = serving.make_requests(fleet, P.multi_max(), with_index=True)
    n_keys = sum(len(q) for _, q, _ in reqs)
    dev = [(m, torch.from_numpy(q.view(np.int64)).to("cuda"), torch.empty(len(q), dtype=torch.int32, device="cuda"))
           for m, q, _ in reqs]
    plan = P.MultiPlan(len(dev))
    cands = None
    if args.kernel not in ("auto", "plain"):
        v = [int(x) for x in args.kernel.split(",")]
        cands = [(v[0], v[1], v[2] if len(v) > 2 else 0)]
    shape, sweep = autotune.tune_multi(torch, plan, dev, cands=cands, use_cache=False)
    log("[bench] multi shape sweep (keys-per-lane/block/blocks-per-cu): " +
        ", ".join(f"{c[0]}/{c[1]}/{c[2]}={v:.4f}ms" for c, v in sorted(sweep.items())))
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        plan.launch()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1) / args.steps
    got = [o.clone() for _, _, o in dev]

    # parity: one plain launch per request, and the oracle on every request
    for m, q, o in dev:
        m.set_kernel(P.KERNEL_PLAIN, 1, 256)
        m.query_into(q, o)
    torch.cuda.synchronize()
    plain_equal = all(torch.equal(a, o) for a, (_, _, o) in zip(got, dev))
    oracles = [oracle_mphf(P, b.params, b) for _, _, b in fleet]
    host = [g.cpu().numpy().view(np.uint32).astype(np.uint64) for g in got]
    # slot >= n fraction of the requests' keys (non-minimal view of the same pilots)
    phf = {}
    remapped = 0
    for (m, q, _), j in zip(dev, js):
        if j not in phf:
            b = fleet[j][2]
            pp = b.params.copy()
            pp.remap_kind = P.REMAP_NONE
            pp.index_bits = 64
            phf[j] = P.Mphf().load(pp, b.pilots, None)
        remapped += int((phf[j].query(q) >= fleet[j][2].params.n).sum().item())
    for h in phf.values():
        h.close()
    rfrac = remapped / n_keys

    def check(i):
        q = reqs[i][1]
        return np.array_equal(O.query_u64(oracles[js[i]], q, O.REMAP_CLEF), host[i])

    cpu = None
    with ThreadPoolExecutor(threads) as ex:
        c0 = time.perf_counter()
        oracle_equal = all(ex.map(check, range(len(reqs))))
        cdt = time.perf_counter() - c0
    if args.cpu_sample:
        cpu = {"value": n_keys / cdt, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "ns_per_key": cdt / n_keys * 1e9,
               "sample": f"all {len(reqs)} requests ({n_keys} keys): the C oracle's plain query loop per request, "
                         f"requests spread over {threads} threads",
               "matches_gpu": oracle_equal}
    plan.close()
    log(f"[bench] multi launch {ms:.4f} ms ({n_keys / ms / 1e6:.1f} G keys/s, shape {shape}) remap_frac={rfrac:.4f} "
        f"plain_equal={plain_equal} oracle_equal={oracle_equal} (oracle {cdt / n_keys * 1e9:.2f} ns/key)")
    per_key = 8 + 4 + 1 + rfrac * 64
    rec = record(args, n_keys, ms, wall, WORKLOADS["multi_c5"][3],
                 {"requests": len(reqs), "mphfs": len(fleet), "resident_keys": int(sum(len(f[0]) for f in fleet)),
                  "multi_shape": {"keys_per_lane": shape[0], "block": shape[1], "blocks_per_cu": shape[2]},
                  "index_bits": 32},
                 "u64", per_key, cpu_baseline=cpu,
                 parity={"multi_equals_plain": plain_equal, "multi_equals_oracle": oracle_equal,
                         "remap_fraction": rfrac},
                 shape_sweep_ms={f"{c[0]}/{c[1]}/{c[2]}": v for c, v in sorted(sweep.items())})
    rec["metric"] = "queries/s of one multi-MPHF launch over 4096 device-resident requests (64 MPHFs)"
    return rec, plain_equal and oracle_equal


def run_serve(args, torch, K, P):
    from paper_2502_15539_amd import serving

    res = serving.run_c5(torch, n_requests=args.requests, threads=args.threads or min(16, os.cpu_count() or 1),
                         log=log)
    sat = res["saturated"]
    rec = {"metric": "serving: queries/s with p50/p99 latency, 64 resident MPHFs", "value": sat["keys_per_s"],
           "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": sat["makespan_s"] * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
           "data": "synthetic (seeded SplitMix64 keys, log-uniform sizes, Poisson arrivals)",
           "config": {"workload": WORKLOADS["serve_c5"][3], "requests": args.requests, "parallelism": "single GPU"},
           "serving": res}
    return rec, res["served_equals_plain"] and res["batched_on_device"]["multi_equals_plain"]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the query stream would be split across GPUs with no exchange; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2502_15539_amd import keygen as K
    from paper_2502_15539_amd import ptrhash as P

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    P.lib()  # fail loudly if the HIP library is missing
    kind = WORKLOADS[args.workload][1]
    run = {"u64": run_u64, "cached": run_cached, "bytes": run_bytes, "multi": run_multi, "serve": run_serve}[kind]
    rec, ok = run(args, torch, K, P)
    print(json.dumps(rec), flush=True)
    if not ok:
        sys.exit(3)


if __name__ == "__main__":
    main()
