"""Parity at the full benchmark sizes, in the launch configuration that the
benchmark times.

The oracle cannot build the 10^9-key and 3*10^8-string MPHFs inside a test
(its single-threaded construction takes tens of minutes and about 40 GB),
so tests/golden/fullsize_digests.json holds the SHA-256 of the pilot array
and of the CacheLineEF bytes that the oracle built for exactly these key
sets, written once by tests/golden/make_fullsize_digests.py (which calls
only the oracle and the seeded generators). The device construction here
must reproduce both digests, its seed and its eviction count, so the tables
the GPU queries are the oracle's own. Then:

* parameters equal the oracle's parameter rule;
* the kernel choice is the one the benchmark's autotuner picks, over the same
  candidate list, and the plain one-key-per-lane kernel agrees with it on
  every output;
* all members map bijectively onto [0, n) (a property that holds at any
  size);
* every index of the whole query stream equals the oracle's query of the
  same key, the oracle's loop split over the host's threads; the keys of
  sampled positions (the first and last 2^18 and 2^20 random ones) are also
  regenerated on the host from the seeded generators and must equal the
  device-generated stream;
* non-members: 2^20 of them, every output equal to the oracle's.

4.4*10^9 keys are beyond the oracle's memory here: there the device build
is checked by bijection and sampled oracle parity only.

The 64-MPHF workload runs at its full size too: 4096 requests (24.1 M keys)
in one multi-MPHF launch with the autotuner's shape, and 2000 of them
through the server, every index equal to the oracle's query of the
request's own MPHF.
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import autotune
from paper_2502_15539_amd import keygen as K
from paper_2502_15539_amd import ptrhash as P
from paper_2502_15539_amd import serving

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"
EDGE = 1 << 18
RANDOM = 1 << 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sample_positions(n, seed):
    rng = np.random.default_rng(seed)
    pos = np.concatenate([np.arange(min(EDGE, n)), np.arange(max(0, n - EDGE), n),
                          rng.integers(0, n, RANDOM)])
    return pos.astype(np.uint64)


def oracle_of(built):
    p = built.params
    op = O.params_explicit(p.n, p.num_parts, p.log2_slots, p.buckets_per_part, gamma=p.gamma, seed=p.seed)
    return O.Mphf(op, built.pilots, None, built.remap, None)


def check_params(p, n):
    ref = O.params_for(n)
    assert (p.num_parts, p.log2_slots, p.buckets_per_part) == (ref.num_parts, ref.log2_slots, ref.buckets_per_part)
    assert p.gamma == P.GAMMA_CUBIC and p.remap_kind == P.REMAP_CLEF


def bijective(out, n):
    o = out.long()
    assert int(o.min()) >= 0 and int(o.max()) < n
    seen = torch.zeros(n, dtype=torch.bool, device=out.device)
    seen[o] = True
    return bool(seen.all())


def to_u64(t):
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 else a.view(np.uint32).astype(np.uint64)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_digests.json")


def host_threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def check_golden(name, built):
    """The device build equals the oracle's build of the same set: seed,
    eviction count and SHA-256 of the pilots and of the CacheLineEF bytes."""
    if not os.path.exists(GOLDEN) or name not in json.load(open(GOLDEN)):
        pytest.fail(f"no oracle digest for {name} in {GOLDEN}")
    g = json.load(open(GOLDEN))[name]
    p = built.params
    assert (p.n, p.num_parts, p.log2_slots, p.buckets_per_part) == (g["n"], g["num_parts"], g["log2_slots"],
                                                                    g["buckets_per_part"])
    assert p.seed == g["seed"] and built.info.attempts == g["attempts"]
    assert built.info.evictions == g["evictions"]
    assert hashlib.sha256(memoryview(built.pilots)).hexdigest() == g["pilots_sha256"]
    assert hashlib.sha256(memoryview(built.remap)).hexdigest() == g["clef_sha256"]
    say(f"[fullsize] {name}: device build == oracle build (digests, seed {p.seed}, {g['evictions']} evictions)")


def oracle_whole_u64(m, keys):
    """The oracle's query of every key, in slices over the host's threads."""
    bounds = np.linspace(0, len(keys), host_threads() * 4 + 1).astype(np.int64)
    out = np.empty(len(keys), dtype=np.uint64)

    def run(i):
        lo, hi = int(bounds[i]), int(bounds[i + 1])
        if hi > lo:
            out[lo:hi] = O.query_u64(m, keys[lo:hi], O.REMAP_CLEF)

    with ThreadPoolExecutor(host_threads()) as ex:
        list(ex.map(run, range(len(bounds) - 1)))
    return out


def oracle_whole_bytes(m, data, offs):
    n = len(offs) - 1
    bounds = np.linspace(0, n, host_threads() * 4 + 1).astype(np.int64)
    out = np.empty(n, dtype=np.uint64)

    def run(i):
        lo, hi = int(bounds[i]), int(bounds[i + 1])
        if hi > lo:
            o = offs[lo:hi + 1]
            out[lo:hi] = O.query_bytes(m, data[int(o[0]):int(o[-1]) + 64], o - o[0], O.REMAP_CLEF)

    with ThreadPoolExecutor(host_threads()) as ex:
        list(ex.map(run, range(len(bounds) - 1)))
    return out


def tuned(mphf, run, n_q, key_kind):
    best, _ = autotune.tune(torch, mphf, run, n_q, cands=autotune.candidates_for(key_kind), use_cache=False)
    say(f"[fullsize] tuned choice {best}")
    return best


def test_u64_1e9_default():
    n = 10**9
    say(f"[fullsize] u64 n={n}: device keys + device construction")
    keys = P.gen_u64_keys(torch.empty(n, dtype=torch.int64, device=DEV), K.KEY_SEED)
    built = P.build_u64_device(keys, index_bits=64, placement="device")
    del keys
    torch.cuda.empty_cache()
    check_params(built.params, n)
    check_golden("u64_1e9", built)
    mphf = P.Mphf.from_built(built)
    q = P.gen_query_stream(torch.empty(n, dtype=torch.int64, device=DEV), n, K.KEY_SEED, K.ORDER_SEED)
    out = torch.empty(n, dtype=torch.int64, device=DEV)
    tuned(mphf, lambda: mphf.query_into(q, out), n, P.KEY_U64)
    mphf.query_into(q, out)
    torch.cuda.synchronize()
    say("[fullsize] u64 bijection")
    assert bijective(out, n)

    say("[fullsize] u64 stream keys at sampled positions regenerated on the host")
    pos = sample_positions(n, 11)
    qs = K.query_stream_at(n, pos)
    assert np.array_equal(to_u64(q[torch.from_numpy(pos.astype(np.int64)).to(DEV)]), qs)

    say(f"[fullsize] u64 whole-stream oracle parity ({n} keys, {host_threads()} host threads)")
    t0 = time.time()
    qh = to_u64(q)
    ref = oracle_whole_u64(oracle_of(built), qh)
    got = to_u64(out)
    bad = int(np.count_nonzero(got != ref))
    say(f"[fullsize] oracle over the whole stream in {time.time() - t0:.1f} s: {bad} differences")
    assert bad == 0
    del qh, ref, got

    say("[fullsize] u64 non-members, tuned and plain kernels")
    nm = K.nonmember_keys(RANDOM, seed=31)
    got_nm = to_u64(mphf.query(torch.from_numpy(nm.view(np.int64)).to(DEV)))
    assert np.array_equal(got_nm, O.query_u64(oracle_of(built), nm, O.REMAP_CLEF))

    mphf.set_kernel(P.KERNEL_PLAIN, 1, 256)
    mphf.set_occupancy(0)
    out2 = torch.empty_like(out)
    mphf.query_into(q, out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)


def test_bytes_3e8_default():
    n = 3 * 10**8
    say(f"[fullsize] strings n={n}: device strings + device construction")
    d_data, d_off = P.gen_strings(n, K.KEY_SEED)
    built = P.build_bytes_device(d_data, d_off, index_bits=32, placement="device")
    del d_data, d_off
    torch.cuda.empty_cache()
    check_params(built.params, n)
    check_golden("bytes_3e8", built)
    mphf = P.Mphf.from_built(built)
    qd, qo = P.gen_strings(n, K.KEY_SEED, K.ORDER_SEED, shuffled=True)
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    tuned(mphf, lambda: mphf.query_bytes_into(qd, qo, out, check_end=False), n, P.KEY_BYTES)
    mphf.query_bytes_into(qd, qo, out)
    torch.cuda.synchronize()
    say("[fullsize] strings bijection")
    assert bijective(out, n)

    say("[fullsize] strings at sampled positions regenerated on the host")
    pos = sample_positions(n, 12)
    sd, so = K.string_query_stream_at(n, pos)
    ref = O.query_bytes(oracle_of(built), sd, so, O.REMAP_CLEF)
    got = to_u64(out[torch.from_numpy(pos.astype(np.int64)).to(DEV)])
    assert np.array_equal(got, ref)

    say(f"[fullsize] strings whole-stream oracle parity ({n} strings, {host_threads()} host threads)")
    t0 = time.time()
    hd = qd.cpu().numpy()
    ho = qo.cpu().numpy().view(np.uint64)
    ref = oracle_whole_bytes(oracle_of(built), hd, ho)
    got = to_u64(out)
    bad = int(np.count_nonzero(got != ref))
    say(f"[fullsize] oracle over the whole stream in {time.time() - t0:.1f} s: {bad} differences")
    assert bad == 0
    del hd, ho, ref, got

    say("[fullsize] strings: plain kernel agrees")
    mphf.set_kernel(P.KERNEL_PLAIN, 1, 256)
    mphf.set_occupancy(0)
    out2 = torch.empty_like(out)
    mphf.query_bytes_into(qd, qo, out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)


def test_u64_beyond_2_32_keys():
    """4.4e9 keys: slots, indices and remap values beyond 2^32, 4239 parts.
    Device construction, the 64-bit query, bijection, sampled oracle parity."""
    n = 4_400_000_000
    free, _ = torch.cuda.mem_get_info()
    if free < 200 * 2**30:
        pytest.skip(f"needs ~200 GiB of free device memory, {free / 2**30:.0f} GiB free")
    say(f"[fullsize] u64 n={n}: device keys + device construction")
    keys = P.gen_u64_keys(torch.empty(n, dtype=torch.int64, device=DEV), K.KEY_SEED)
    t0 = time.time()
    built = P.build_u64_device(keys, index_bits=64, placement="device")
    say(f"[fullsize] construction {time.time() - t0:.1f} s, {built.info.evictions} evictions")
    check_params(built.params, n)
    assert built.params.num_parts * (1 << built.params.log2_slots) > 2**32
    torch.cuda.empty_cache()
    mphf = P.Mphf.from_built(built)
    q = P.gen_query_stream(keys, n, K.KEY_SEED, K.ORDER_SEED)  # the key buffer is free again
    out = torch.empty(n, dtype=torch.int64, device=DEV)
    mphf.query_into(q, out)
    torch.cuda.synchronize()
    say("[fullsize] >2^32 bijection")
    assert int(out.min()) >= 0 and int(out.max()) == n - 1
    seen = torch.zeros(n, dtype=torch.bool, device=DEV)
    step = 1 << 30
    for lo in range(0, n, step):
        seen[out[lo:lo + step]] = True
    assert bool(seen.all())
    del seen
    say("[fullsize] >2^32 sampled oracle parity")
    pos = sample_positions(n, 13)
    qs = K.query_stream_at(n, pos)
    idx = torch.from_numpy(pos.astype(np.int64)).to(DEV)
    assert np.array_equal(to_u64(q[idx]), qs)
    got = to_u64(out[idx])
    ref = O.query_u64(oracle_of(built), qs, O.REMAP_CLEF)
    assert np.array_equal(got, ref)
    assert int(ref.max()) >= 2**32  # the sample reaches indices beyond 32 bits


def test_launch_split_beyond_2_31_work_items():
    """2,147,500,000 queries (more than 2^31 work-items with one key per lane
    and 64-thread workgroups) against a 10^5-key MPHF: the library splits the
    batch into launches of at most 2^31 work-items. The stream is the shuffled
    member stream repeated, so every period's indices must equal the first's,
    which equal the oracle's, and the keys around the split equal it too."""
    n, reps = 100_000, 21_475
    n_q = n * reps
    assert n_q > 2**31
    keys = K.u64_keys(n, seed=8)
    m = O.build_u64(keys)
    period = K.query_stream(n, key_seed=8)
    want = O.query_u64(m, period, O.REMAP_CLEF)
    g = P.Mphf().load(*_lib_load_args(m))
    q = torch.from_numpy(period.view(np.int64)).to(DEV).repeat(reps)
    out = torch.empty(n_q, dtype=torch.int32, device=DEV)
    for kern, kpl, blk in [(P.KERNEL_PLAIN, 1, 64), (P.KERNEL_PIPELINED, 1, 64)]:
        say(f"[fullsize] {n_q} queries, kernel {kern} keys/lane {kpl} block {blk}")
        g.set_kernel(kern, kpl, blk)
        out.fill_(-1)
        g.query_into(q, out)
        torch.cuda.synchronize()
        head = out[:n]
        assert np.array_equal(to_u64(head), want)
        assert bool((out.view(reps, n) == head).all())
        split = 2**31
        assert np.array_equal(to_u64(out[split - 8:split + 8]), want[(np.arange(split - 8, split + 8)) % n])
    del q, out


def _lib_load_args(m):
    from .mphf_pairs import lib_params

    return lib_params(m, P.REMAP_CLEF, 32), m.pilots, m.clef


def oracle_of_params(b):
    p = b.params
    if p.reduce_kind == P.REDUCE_MOD:
        op = O.params_single_mod(p.n, S=p.slots, B=p.buckets_per_part, gamma=p.gamma, seed=p.seed)
    else:
        op = O.params_explicit(p.n, p.num_parts, p.log2_slots, p.buckets_per_part, gamma=p.gamma, seed=p.seed)
    return O.Mphf(op, b.pilots, None, b.remap, None)


def test_multi_mphf_fleet_full_size():
    """64 MPHFs (n log-uniform in [1e4, 1e7]), 4096 requests of log-uniform
    sizes in [1, 65536]: one tuned multi-MPHF launch, then 2000 requests
    through the zero-copy server; every index equals the oracle's."""
    say("[fullsize] serving fleet: 64 MPHFs")
    fleet = serving.build_fleet(threads=16, log=say)
    reqs, js = serving.make_requests(fleet, P.multi_max(), with_index=True)
    oracles = [oracle_of_params(b) for _, _, b in fleet]
    want = [O.query_u64(oracles[j], q, O.REMAP_CLEF) for (_, q, _), j in zip(reqs, js)]
    dev = [(m, torch.from_numpy(q.view(np.int64)).to(DEV), torch.empty(len(q), dtype=torch.int32, device=DEV))
           for m, q, _ in reqs]
    say(f"[fullsize] multi launch over {len(dev)} requests, {sum(len(q) for _, q, _ in reqs)} keys")
    plan = P.MultiPlan(len(dev))
    shape, _ = autotune.tune_multi(torch, plan, dev, use_cache=False)
    say(f"[fullsize] multi shape {shape}")
    plan.launch()
    torch.cuda.synchronize()
    for (_, _, o), w in zip(dev, want):
        assert np.array_equal(o.cpu().numpy().view(np.uint32).astype(np.uint64), w)
    plan.close()

    say("[fullsize] 2000 requests through the server")
    srv = P.Server(streams=2, max_batches=1024, slot_keys=1 << 22, zero_copy=1, multi_kernel=shape)
    tickets = [srv.submit(m, q, out) for m, q, out in reqs[:2000]]
    for t in tickets:
        srv.wait(t)
    srv.close()
    for (_, _, out), w in zip(reqs[:2000], want):
        assert np.array_equal(out.astype(np.uint64), w)
