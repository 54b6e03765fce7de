"""Summaries of rocprofv3 results (rocpd SQLite databases).

    python -m paper_2502_15539_amd.profsum trace DB
        per-kernel calls / total / average duration (markdown)
    python -m paper_2502_15539_amd.profsum counters DB [DB ...]
        mean value of each collected counter per kernel (markdown)
    python -m paper_2502_15539_amd.profsum traffic --reads DB --write DB --kernel SUBSTR --out JSON
        Bytes per launch of a kernel between the L2 caches and the memory
        fabric: read requests counted by size (TCC_EA0_RDREQ_<size>B_sum,
        each times its size) plus WRITE_SIZE; beside them the read bytes
        addressed to memory rather than to other agents
        (TCC_EA0_RDREQ_DRAM_32B_sum, in 32-byte units), which still include
        what the MALL on the memory side serves. The JSON records a hash of
        the kernel sources so that a later change voids it. With --fetch DB
        (a FETCH_SIZE run of the same command) it also records FETCH_SIZE
        scaled by the factor that maps the copy kernel's FETCH_SIZE onto the
        bytes it reads, as a cross-check of the read bytes.
    python -m paper_2502_15539_amd.profsum overlap DB --kernel SUBSTR
        from a kernel trace: dispatches of the kernel, the most running at
        one instant, the time-weighted mean number running while any runs,
        and the share of their busy time with two or more running
    python -m paper_2502_15539_amd.profsum steps DB --kernel NAME --before SUBSTR --count N
        durations of the timed launches in a kernel trace of bench.py: the
        last N dispatches of the kernel named NAME (exactly) that start
        before the first dispatch whose name contains SUBSTR (the benchmark
        times its query steps right before its roofline kernels)
    python -m paper_2502_15539_amd.profsum valu --db DB --kernel SUBSTR --out JSON
        vector-ALU instructions per launch of a kernel (SQ_INSTS_VALU, counted
        per wavefront) with the VALUBusy and VALUUtilization metrics, and the
        same source hash.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/kernels.hip", "csrc/mphf_device.h"]


def _code_only(text: str) -> str:
    """The source without comments and blank lines, so that a comment edit
    does not void a profile."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", line).rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line.strip())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", name).replace("void ", "")


def trace(db: str) -> str:
    cur = sqlite3.connect(db).cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["| kernel | calls | total ms | avg ms | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:  # durations in microseconds
        out.append(f"| `{short(name)}` | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.4f} | {pct:.1f} |")
    return "\n".join(out)


def counter_means(db: str):
    cur = sqlite3.connect(db).cursor()
    return list(cur.execute("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                            "group by kernel_name, counter_name"))


def counters(dbs) -> str:
    out = ["| kernel | counter | mean per dispatch | dispatches |", "|---|---|---|---|"]
    for db in dbs:
        for k, c, v, cnt in counter_means(db):
            if "ptrhash" in k:
                out.append(f"| `{short(k)}` | {c} | {v:,.0f} | {cnt} |")
    return "\n".join(out)


def _mean(db, kernel_sub, counter):
    vals = [(k, v) for k, c, v, _ in counter_means(db) if c == counter and kernel_sub in k]
    if not vals:
        raise SystemExit(f"no {counter} for a kernel matching {kernel_sub!r} in {db}")
    return vals[0][1]


def traffic(args) -> dict:
    reads = [(c, v) for k, c, v, _ in counter_means(args.reads) if args.kernel in k]
    sized = {}
    for c, v in reads:
        m = re.fullmatch(r"TCC_EA0_RDREQ_(\d+)B_sum", c)
        if m:
            sized[int(m.group(1))] = v
    if not sized:
        raise SystemExit(f"no TCC_EA0_RDREQ_<size>B_sum counters for {args.kernel!r} in {args.reads}")
    read_bytes = sum(size * v for size, v in sized.items())
    dram32 = dict(reads).get("TCC_EA0_RDREQ_DRAM_32B_sum")
    k_write = _mean(args.write, args.kernel, "WRITE_SIZE") * 1024.0
    other = {c: v for c, v in reads if not re.fullmatch(r"TCC_EA0_RDREQ_(\d+)B_sum", c)}
    other.pop("TCC_EA0_RDREQ_DRAM_32B_sum", None)
    other.pop("TCC_EA0_RDREQ_DRAM_sum", None)
    fetch = None
    if getattr(args, "fetch", None):
        # cross-check: FETCH_SIZE scaled by the factor that maps a copy
        # kernel's FETCH_SIZE onto the bytes it reads
        copy_fetch = _mean(args.fetch, args.copy, "FETCH_SIZE") * 1024.0
        scale = args.copy_bytes / copy_fetch
        k_fetch = _mean(args.fetch, args.kernel, "FETCH_SIZE") * 1024.0
        fetch = {"fetch_size_bytes_raw": k_fetch, "copy_kernel": args.copy, "copy_read_bytes": args.copy_bytes,
                 "scale": scale, "fetch_bytes_scaled": k_fetch * scale}
    res = {"kernel": args.kernel,
           "level": "L2 to memory fabric: read requests by size plus WRITE_SIZE (includes MALL hits)",
           "read_requests_by_size": {f"{k}B": v for k, v in sorted(sized.items())},
           "read_bytes": read_bytes, "write_bytes": k_write,
           "memory_read_bytes": None if dram32 is None else 32.0 * dram32,
           "read_requests": other.get("TCC_EA0_RDREQ_sum"),
           "traffic_bytes_per_launch": read_bytes + k_write, "kernel_source_sha256": kernel_source_hash()}
    if fetch:
        res["fetch_size_check"] = fetch
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    return res


def dispatches(db: str):
    """(name, start, end) of every dispatch in a rocpd kernel trace, by start."""
    cur = sqlite3.connect(db).cursor()
    cur.execute("select * from kernels limit 1")
    cols = [d[0] for d in cur.description]
    name = next(c for c in ("name", "kernel_name") if c in cols)
    start = next(c for c in ("start", "start_ns", "begin") if c in cols)
    end = next(c for c in ("end", "end_ns", "stop") if c in cols)
    rows = cur.execute(f'select "{name}", "{start}", "{end}" from kernels').fetchall()
    return sorted(((n, float(b), float(e)) for n, b, e in rows), key=lambda r: r[1])


def dispatch_spans(db: str, kernel_sub: str):
    """(start, end) of every dispatch of a kernel in a rocpd kernel trace."""
    return [(b, e) for n, b, e in dispatches(db) if kernel_sub in n]


def timed_steps(rows, kernel: str, before: str, count: int) -> dict:
    """The last `count` dispatches of the kernel whose short name is `kernel`
    that start before the first dispatch whose name contains `before`
    (times in ns, durations reported in ms)."""
    stop = next((b for n, b, _ in rows if before in n), float("inf"))
    mine = [(b, e) for n, b, e in rows if short(n) == kernel and b < stop][-count:]
    if len(mine) < count:
        raise SystemExit(f"only {len(mine)} dispatches of {kernel} before {before}")
    d = [(e - b) / 1e6 for b, e in mine]
    return {"kernel": kernel, "dispatches": len(d), "avg_ms": sum(d) / len(d), "min_ms": min(d), "max_ms": max(d),
            "first_to_last_ms_per_step": (mine[-1][1] - mine[0][0]) / 1e6 / len(d)}


def overlap_stats(spans) -> dict:
    ev = sorted([(b, 1) for b, _ in spans] + [(e, -1) for _, e in spans])  # an end sorts first at a tie
    open_, top, prev, busy, multi = 0, 0, 0.0, 0.0, 0.0
    for t, d in ev:
        if open_ > 0:
            busy += t - prev
            if open_ > 1:
                multi += t - prev
        open_ += d
        top = max(top, open_)
        prev = t
    total = sum(e - b for b, e in spans)
    return {"dispatches": len(spans), "max_concurrent": top, "mean_concurrent": total / busy if busy else 0.0,
            "share_of_busy_time_with_2_or_more": multi / busy if busy else 0.0}


def valu(args) -> dict:
    res = {"kernel": args.kernel, "valu_insts_per_launch": _mean(args.db, args.kernel, "SQ_INSTS_VALU"),
           "valu_busy_pct": _mean(args.db, args.kernel, "VALUBusy"),
           "valu_utilization_pct": _mean(args.db, args.kernel, "VALUUtilization"),
           "kernel_source_sha256": kernel_source_hash()}
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    return res


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    r = sub.add_parser("traffic")
    r.add_argument("--reads", required=True, help="DB with TCC_EA0_RDREQ_<size>B_sum (and _DRAM_sum) counters")
    r.add_argument("--write", required=True, help="DB with WRITE_SIZE")
    r.add_argument("--kernel", required=True)
    r.add_argument("--out", required=True)
    r.add_argument("--fetch", help="DB with FETCH_SIZE, for the copy-scaled cross-check")
    r.add_argument("--copy", default="bench_copy_k<1>", help="copy kernel of the cross-check")
    r.add_argument("--copy-bytes", type=float, default=8e9, help="bytes the copy kernel reads per launch")
    st = sub.add_parser("steps")
    st.add_argument("db")
    st.add_argument("--kernel", required=True)
    st.add_argument("--before", required=True)
    st.add_argument("--count", type=int, default=20)
    o = sub.add_parser("overlap")
    o.add_argument("db")
    o.add_argument("--kernel", required=True)
    v = sub.add_parser("valu")
    v.add_argument("--db", required=True)
    v.add_argument("--kernel", required=True)
    v.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace(a.db))
    elif a.cmd == "counters":
        print(counters(a.dbs))
    elif a.cmd == "steps":
        print(json.dumps(timed_steps(dispatches(a.db), a.kernel, a.before, a.count), indent=1))
    elif a.cmd == "overlap":
        print(json.dumps(overlap_stats(dispatch_spans(a.db, a.kernel)), indent=1))
    elif a.cmd == "valu":
        print(json.dumps(valu(a), indent=1))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    main()
