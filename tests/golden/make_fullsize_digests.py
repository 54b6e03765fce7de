"""Write tests/golden/fullsize_digests.json from the oracle alone.

The two full benchmark sets -- 10^9 uniform u64 keys (Section 4.1, the
Table 1 setting) and 3*10^8 random strings of length 10..50 (Section 4.2,
the Table 2 setting) -- are built once by the plain single-threaded oracle
at Default parameters (Section 4.1.2: gamma_3, lambda = 3.5, alpha = 0.99,
CacheLineEF; S from the rule of Section 3.1, "Parameter values"). The JSON
keeps the parameters, the seed the build ended on, the eviction count and
SHA-256 digests of the pilot array and of the CacheLineEF bytes, so that a
device construction of the same keys can be compared with the oracle's
byte for byte without building at full size inside a test.

Only ``oracle/`` and the seeded input generators are used. The u64 build
needs about 40 GB of host memory and the string build about 25 GB; run the
two one after the other:

    python tests/golden/make_fullsize_digests.py u64
    python tests/golden/make_fullsize_digests.py bytes
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2502_15539_amd import keygen as K  # noqa: E402

OUT = os.path.join(HERE, "fullsize_digests.json")
SETS = {
    "u64_1e9": {"n": 10**9, "keys": "u64_keys(n, seed=KEY_SEED)",
                "cite": "Section 4.1 / Table 1: 10^9 uniform random 64-bit keys, Default parameters"},
    "bytes_3e8": {"n": 3 * 10**8, "keys": "strings(n, seed=KEY_SEED)",
                  "cite": "Section 4.2 / Table 2: 3*10^8 random strings of length 10..50, Default parameters"},
}


def say(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def sha(a) -> str:
    return hashlib.sha256(memoryview(a).cast("B")).hexdigest()


def record(name, m, secs):
    p = m.params
    return {
        "cite": SETS[name]["cite"],
        "keys": SETS[name]["keys"],
        "n": int(p.n),
        "num_parts": int(p.num_parts),
        "log2_slots": int(p.log2_slots),
        "buckets_per_part": int(p.buckets_per_part),
        "seed": int(p.seed),
        "attempts": int(m.stats.attempts),
        "evictions": int(m.stats.evictions),
        "max_part_evictions": int(m.stats.max_part_evictions),
        "pilots_bytes": int(m.pilots.size),
        "clef_bytes": int(m.clef.size),
        "pilots_sha256": sha(m.pilots),
        "clef_sha256": sha(m.clef),
        "oracle_build_seconds": round(secs, 1),
    }


def main(which: str) -> None:
    n = SETS[which]["n"]
    say(f"{which}: generating {n} keys")
    if which == "u64_1e9":
        keys = K.u64_keys(n, seed=K.KEY_SEED)
        say("oracle build (single thread)")
        t0 = time.time()
        m = O.build_u64(keys, params=O.params_for(n, seed=K.MPHF_SEED))
    else:
        data, off = K.strings(n, seed=K.KEY_SEED)
        say("oracle build (single thread)")
        t0 = time.time()
        m = O.build_bytes(data, off, params=O.params_for(n, seed=K.MPHF_SEED))
    secs = time.time() - t0
    rec = record(which, m, secs)
    say(f"done in {secs:.0f} s: {rec}")
    doc = json.load(open(OUT)) if os.path.exists(OUT) else {
        "_about": "Oracle-built MPHFs of the full benchmark sets: parameters and SHA-256 of the pilot "
                  "array and the CacheLineEF bytes. Written by make_fullsize_digests.py, which calls only "
                  "the oracle and the seeded key generators."}
    doc[which] = rec
    with open(OUT + ".tmp", "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    arg = sys.argv[1] if len(sys.argv) > 1 else ""
    which = {"u64": "u64_1e9", "bytes": "bytes_3e8"}.get(arg)
    if which is None:
        sys.exit("usage: make_fullsize_digests.py u64|bytes")
    main(which)
