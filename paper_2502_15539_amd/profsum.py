"""Summaries of rocprofv3 results (rocpd SQLite databases).

    python -m paper_2502_15539_amd.profsum trace DB
        per-kernel calls / total / average duration (markdown)
    python -m paper_2502_15539_amd.profsum counters DB [DB ...]
        mean value of each collected counter per kernel (markdown)
    python -m paper_2502_15539_amd.profsum traffic --fetch DB --write DB \\
            --kernel SUBSTR (--copy SUBSTR --copy-bytes N | --scale-from JSON) --out JSON
        HBM bytes per launch of a kernel from FETCH_SIZE and WRITE_SIZE, each
        scaled by the factor that maps the same counter of a plain copy
        kernel (reading and writing N bytes) onto N, or by the factors of an
        earlier traffic JSON of the same device; the JSON records a hash of
        the kernel sources so that a later change voids it.
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
    if args.scale_from:
        ref = json.load(open(args.scale_from))
        fs, ws = ref["fetch_scale"], ref["write_scale"]
    else:
        if not args.copy or not args.copy_bytes:
            raise SystemExit("traffic needs --copy and --copy-bytes, or --scale-from")
        copy_fetch = _mean(args.fetch, args.copy, "FETCH_SIZE") * 1024.0
        copy_write = _mean(args.write, args.copy, "WRITE_SIZE") * 1024.0
        fs, ws = args.copy_bytes / copy_fetch, args.copy_bytes / copy_write
    k_fetch = _mean(args.fetch, args.kernel, "FETCH_SIZE") * 1024.0
    k_write = _mean(args.write, args.kernel, "WRITE_SIZE") * 1024.0
    res = {"kernel": args.kernel, "fetch_bytes_raw": k_fetch, "write_bytes_raw": k_write,
           "fetch_scale": fs, "write_scale": ws, "fetch_bytes": k_fetch * fs, "write_bytes": k_write * ws,
           "traffic_bytes_per_launch": k_fetch * fs + k_write * ws, "kernel_source_sha256": kernel_source_hash()}
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    return res


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
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--kernel", required=True)
    r.add_argument("--copy")
    r.add_argument("--copy-bytes", type=float)
    r.add_argument("--scale-from", help="take the scale factors of this traffic JSON")
    r.add_argument("--out", required=True)
    v = sub.add_parser("valu")
    v.add_argument("--db", required=True)
    v.add_argument("--kernel", required=True)
    v.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace(a.db))
    elif a.cmd == "counters":
        print(counters(a.dbs))
    elif a.cmd == "valu":
        print(json.dumps(valu(a), indent=1))
    else:
        print(json.dumps(traffic(a), indent=1))


if __name__ == "__main__":
    main()
