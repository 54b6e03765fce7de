"""Random-gather roofline of the device, as a function of table size.

    python -m paper_2502_15539_amd.roofline [--n 1e9]
    python -m paper_2502_15539_amd.roofline --lines [--n 2.68e8]

For each table size T (from L2-resident to far beyond the MALL) it times,
on n keys: the streaming gather (u64 key in, one random byte of T, u64 out;
the memory pattern of a query), the pure gather (random bytes only, no
streams) and, once, the stream copy (16 B per key). Prints one JSON object.

--lines times, for a few table sizes, the pure gather alone and with a
second byte read at o xor D of every random offset o (D = 32, 64, 128): a
second byte in the same 128-byte line costs nothing if a miss fills the
whole line, and a second miss if it does not.

--memtypes times the pure gather (2^28 random bytes) from a table of the
10^9-key pilot array's size in default, fine-grained and uncached device
memory (hipExtMallocWithFlags); run it under rocprofv3 --pmc with the
TCC_EA0_RDREQ_<size>B counters to see the request size. The tables are not
freed before the process ends (uncached memory that a kernel has read must
stay allocated until then).

--partition prices answering the 10^9-key stream part by part: the query
over the same stream grouped by part (each part's 296 KB of pilots then
stays in the L2), against the query over the shuffled stream, next to the
un-permute that grouping would need (one random 8-byte write per index,
2^30 of them) and the streaming copy (the least a partition pass costs).
"""
from __future__ import annotations

import argparse
import json

from . import ptrhash as P

SIZES = [1 << 20, 4 << 20, 16 << 20, 64 << 20, 128 << 20, 256 << 20, 285_920_472, 512 << 20, 1 << 30, 4 << 30,
         16 << 30]


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=float, default=1e9)
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--lines", action="store_true", help="line-size probe instead of the size sweep")
    ap.add_argument("--partition", action="store_true", help="price of querying part by part")
    ap.add_argument("--memtypes", action="store_true", help="pure gather from default, fine-grained, uncached memory")
    args = ap.parse_args()
    if args.lines:
        return lines(args)
    if args.memtypes:
        return memtypes(args)
    if args.partition:
        return partition(args)
    n = int(args.n)
    keys = torch.empty(n, dtype=torch.int64, device="cuda")
    P.gen_u64_keys(keys, 1)
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    sink = torch.empty(256 * 8192, dtype=torch.int32, device="cuda")

    def t(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.reps

    res = {"n": n, "copy_ms": min(t(lambda: P.bench_copy(keys, out, k, 256)) for k in (1, 2, 4)), "tables": []}
    for T in SIZES:
        table = torch.randint(0, 256, (T,), dtype=torch.uint8, device="cuda")
        g = min(t(lambda: P.bench_gather(keys, table, out, k, b, o)) for k in (1, 4) for b in (128, 512)
                for o in (0, 4))
        pure = t(lambda: P.bench_gather_pure(n, table, sink))
        res["tables"].append({"table_bytes": T, "gather_ms": g, "gather_G_per_s": n / g / 1e6,
                              "pure_gather_ms": pure, "pure_G_per_s": n / pure / 1e6})
        print(f"T={T / 2**20:8.1f} MiB  gather {g:7.3f} ms ({n / g / 1e6:6.1f} G/s)  "
              f"pure {pure:7.3f} ms ({n / pure / 1e6:6.1f} G/s)", flush=True)
        del table
    print(json.dumps(res), flush=True)


def lines(args):
    import torch

    n = int(args.n) if args.n != 1e9 else 1 << 28
    sink = torch.empty(256 * 4096, dtype=torch.int32, device="cuda")

    def t(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.reps

    res = {"n": n, "tables": []}
    for T in (64 << 20, 1 << 30, 4 << 30):
        table = torch.randint(0, 256, (T,), dtype=torch.uint8, device="cuda")
        row = {"table_bytes": T, "single_ms": t(lambda: P.bench_gather_pure(n, table, sink))}
        for d in (32, 64, 128):
            row[f"pair_xor{d}_ms"] = t(lambda: P.bench_gather_pair(n, table, sink, d))
        res["tables"].append(row)
        print(f"T={T >> 20:5d} MiB  single {row['single_ms']:.3f} ms  +o^32 {row['pair_xor32_ms']:.3f}  "
              f"+o^64 {row['pair_xor64_ms']:.3f}  +o^128 {row['pair_xor128_ms']:.3f} ms", flush=True)
        del table
    print(json.dumps(res), flush=True)


_KEEP = []  # tables allocated by memtypes(), held until the process ends


def memtypes(args):
    import ctypes as C

    import torch

    hip = C.CDLL("libamdhip64.so")
    hip.hipExtMallocWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_size_t, C.c_uint]
    hip.hipExtMallocWithFlags.restype = C.c_int
    hip.hipMemset.argtypes = [C.c_void_p, C.c_int, C.c_size_t]
    hip.hipMemset.restype = C.c_int
    T = SIZES[6]  # the pilot array of the 10^9-key MPHF
    n = 1 << 28
    torch.cuda.init()
    sink = torch.empty(256 * 8192, dtype=torch.int32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {"n": n, "table_bytes": T}
    for name, flag in (("default", 0x0), ("finegrained", 0x1), ("uncached", 0x3)):
        p = C.c_void_p()
        if hip.hipExtMallocWithFlags(C.byref(p), T, flag) != 0 or not p.value:
            raise SystemExit(f"hipExtMallocWithFlags({name}) failed")
        _KEEP.append(p)
        if hip.hipMemset(p, 0x5A, T) != 0:
            raise SystemExit("hipMemset failed")

        def run():
            rc = P.lib().ptrhash_bench_gather_pure(n, p, T, C.c_void_p(sink.data_ptr()), sink.numel(), stream)
            if rc:
                raise SystemExit(f"gather failed: {rc}")

        run()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.reps):
            run()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.reps
        res[name] = {"ms": ms, "G_per_s": n / ms / 1e6}
        print(f"{name:12s} {ms:.3f} ms  {n / ms / 1e6:.1f} G random bytes/s", flush=True)
    print(json.dumps(res), flush=True)


def partition(args):
    import torch

    from . import keygen as K

    n = int(args.n)
    dev = "cuda"

    def t(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.reps

    keys = P.gen_u64_keys(torch.empty(n, dtype=torch.int64, device=dev), K.KEY_SEED)
    built = P.build_u64_device(keys, index_bits=64, placement="device")
    del keys
    mphf = P.Mphf.from_built(built)
    q = P.gen_query_stream(torch.empty(n, dtype=torch.int64, device=dev), n, K.KEY_SEED, K.ORDER_SEED)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    res = {"n": n}
    for kpl, block, occ in ((1, 128, 6), (2, 64, 6), (4, 256, 0)):
        mphf.set_kernel(P.KERNEL_PIPELINED, kpl, block)
        mphf.set_occupancy(occ)
        res[f"query_shuffled_ms_{kpl}_{block}_{occ}"] = t(lambda: mphf.query_into(q, out))
    # the same stream grouped by part: sort it by the slot the MPHF gives
    # each key (slot = part * S + local), taken from a non-minimal view of
    # the same pilots
    pp = built.params.copy()
    pp.remap_kind, pp.index_bits = P.REMAP_NONE, 64
    phf = P.Mphf().load(pp, built.pilots, None)
    order = torch.argsort(phf.query(q))
    phf.close()
    qp = q[order]
    del order
    for kpl, block, occ in ((1, 128, 6), (2, 64, 6), (4, 256, 0)):
        mphf.set_kernel(P.KERNEL_PIPELINED, kpl, block)
        mphf.set_occupancy(occ)
        res[f"query_by_part_ms_{kpl}_{block}_{occ}"] = t(lambda: mphf.query_into(qp, out))
    del qp
    res["copy_16B_per_key_ms"] = min(t(lambda: P.bench_copy(q, out, k, 256)) for k in (1, 2, 4))
    del q, out
    torch.cuda.empty_cache()
    src = torch.empty(1 << 30, dtype=torch.int64, device=dev)
    src.random_()
    dst = torch.empty_like(src)
    res["scatter_2^30_ms"] = t(lambda: P.bench_scatter(src, 30, dst))
    res["scatter_ns_per_index"] = res["scatter_2^30_ms"] * 1e6 / (1 << 30)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
