"""Autotuner for the query kernels and the multi-MPHF launch.

Knobs (see ptrhash_set_kernel / ptrhash_set_occupancy): the kernel (one key
per lane, or K keys per lane with all K pilot gathers in flight before any is
used: K is the number of loads in flight per lane), the workgroup size, and
an occupancy cap (resident workgroups per compute unit). Each candidate is
timed on the caller's own launch; the winner is cached per workload class --
device name, key kind, pilot-table size class, index width -- in a JSON file
(``$PTRHASH_TUNE_CACHE`` or ``~/.cache/ptrhash_mi355x/tuning.json``) so a
later process skips the sweep.

The persistent multi-MPHF launch (plans, servers, query_multi) has the same
kinds of knobs -- keys per lane, workgroup size, resident workgroups per CU
(here the persistent grid's size) -- tuned by ``tune_multi`` on a plan and
its batches.
"""
from __future__ import annotations

import json
import math
import os

from . import ptrhash as P

DEFAULT_KPL = (1, 2, 4, 8, 16)
DEFAULT_BLOCKS = (64, 128, 256, 512)
DEFAULT_OCCUPANCY = (0, 2, 3, 4, 6, 8)  # resident workgroups per CU; 0 = uncapped
BYTES_KPL = (1, 2, 4, 8)  # string keys hold more registers per key in flight


def cache_path() -> str:
    return os.environ.get("PTRHASH_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ptrhash_mi355x", "tuning.json"))


def workload_class(mphf: P.Mphf, n_q: int, device_name: str) -> str:
    p = mphf.params
    table = p.num_parts * p.buckets_per_part
    kind = "bytes" if p.key_kind == P.KEY_BYTES else "u64"
    return (f"{device_name}|{kind}|table2^{max(0, int(math.log2(table)))}|out{p.index_bits}|"
            f"nq2^{max(0, int(math.log2(max(n_q, 1))))}")


def candidates(kpls=DEFAULT_KPL, blocks=DEFAULT_BLOCKS, occupancy=DEFAULT_OCCUPANCY):
    out = [(P.KERNEL_PLAIN, 1, 256, 0)]
    for k in kpls:
        for b in blocks:
            for o in occupancy:
                out.append((P.KERNEL_PIPELINED, k, b, o))
    return out


def candidates_for(key_kind):
    """The sweep used for a key kind (u64 or byte strings)."""
    return candidates(kpls=BYTES_KPL if key_kind == P.KEY_BYTES else DEFAULT_KPL)


def _time(torch, fn, reps, warmup=1):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def apply(mphf: P.Mphf, choice):
    kern, kpl, blk, occ = choice
    mphf.set_kernel(kern, kpl, blk)
    mphf.set_occupancy(occ)


def sweep(torch, mphf: P.Mphf, run, cands=None, reps=3):
    """Time every candidate on run() (one query launch); returns {choice: ms}."""
    res = {}
    for c in cands or candidates():
        apply(mphf, c)
        res[c] = _time(torch, run, reps)
    return res


def tune(torch, mphf: P.Mphf, run, n_q: int, cands=None, reps=3, use_cache=True):
    """Pick and apply the fastest choice for this workload class; returns
    (choice, timings) -- timings is empty when the cache answered."""
    name = torch.cuda.get_device_name()
    key = workload_class(mphf, n_q, name)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        choice = tuple(cache[key]["choice"])
        apply(mphf, choice)
        return choice, {}
    res = sweep(torch, mphf, run, cands, reps)
    best = min(res, key=res.get)
    apply(mphf, best)
    if use_cache:
        cache[key] = {"choice": list(best), "ms": res[best]}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp"
            json.dump(cache, open(tmp, "w"), indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return best, res


MULTI_KPL = (1, 2, 4, 8)
MULTI_BLOCKS = (64, 128, 256, 512)
MULTI_OCCUPANCY = (0, 2, 4, 8)  # resident workgroups per CU; 0 = as many as fit


def multi_candidates(kpls=MULTI_KPL, blocks=MULTI_BLOCKS, occupancy=MULTI_OCCUPANCY):
    return [(k, b, o) for k in kpls for b in blocks for o in occupancy]


def multi_workload_class(batches, device_name: str) -> str:
    keys = sum(_batch_len(b) for b in batches)
    return (f"{device_name}|multi|batches2^{max(0, int(math.log2(max(len(batches), 1))))}|"
            f"keys2^{max(0, int(math.log2(max(keys, 1))))}")


def _batch_len(b):
    q = b[1]
    return (q[1].numel() - 1) if isinstance(q, tuple) else q.numel()


def tune_multi(torch, plan: P.MultiPlan, batches, cands=None, reps=3, use_cache=True):
    """Pick the multi-MPHF launch shape for a plan and its batches: each
    candidate is set on the plan, the batches set again, and one plan
    launch timed. Applies the winner (the plan then holds these batches) and
    returns (choice, timings); timings is empty when the cache answered."""
    name = torch.cuda.get_device_name()
    key = multi_workload_class(batches, name)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        choice = tuple(cache[key]["choice"])
        plan.set_kernel(*choice)
        plan.set(batches)
        return choice, {}
    res = {}
    for c in cands or multi_candidates():
        plan.set_kernel(*c)
        plan.set(batches)
        res[c] = _time(torch, plan.launch, reps)
    best = min(res, key=res.get)
    plan.set_kernel(*best)
    plan.set(batches)
    if use_cache:
        cache[key] = {"choice": list(best), "ms": res[best]}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp"
            json.dump(cache, open(tmp, "w"), indent=1)
            os.replace(tmp, path)
        except OSError:
            pass
    return best, res
