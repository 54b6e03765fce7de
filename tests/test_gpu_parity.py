"""GPU parity: the HIP kernels against the oracle, element by element.

Every MPHF here is built by the oracle; the same parameters, pilots and
remap bytes are loaded into the library, and the GPU indices must equal the
oracle's query bit for bit, for members and non-members, every kernel
variant, both output widths and every remap encoding. At the full
benchmark sizes, where the oracle cannot build, the library's own build is
checked by properties that hold at any size (bijection of the members, range
of non-members, agreement of the kernel variants).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K
from paper_2502_15539_amd import ptrhash as P

from .mphf_pairs import ORACLE_REMAP, load

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"
VARIANTS = [(P.KERNEL_PLAIN, 1, 256), (P.KERNEL_PLAIN, 1, 64), (P.KERNEL_PIPELINED, 1, 256),
            (P.KERNEL_PIPELINED, 2, 128), (P.KERNEL_PIPELINED, 4, 256), (P.KERNEL_PIPELINED, 8, 256),
            (P.KERNEL_PIPELINED, 16, 64), (P.KERNEL_PIPELINED, 4, 1024)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_cache = {}


def oracle_mphf(n, seed=0, **kw):
    key = (n, seed, tuple(sorted(kw.items())))
    if key not in _cache:
        keys = K.u64_keys(n, seed=100 + seed)
        _cache[key] = (keys, O.build_u64(keys, seed=seed, **kw))
    return _cache[key]


def probe_keys(keys, extra=20_000, seed=0):
    rng = np.random.default_rng(seed)
    members = keys[rng.permutation(len(keys))]
    return np.concatenate([members, K.nonmember_keys(extra, seed=seed + 77)])


def gpu_query(mphf, q, index_bits):
    qt = torch.from_numpy(q.view(np.int64)).to(DEV)
    out = mphf.query(qt)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o.view(np.uint64) if index_bits == 64 else o.view(np.uint32).astype(np.uint64)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 1000, 65_537, 1_000_000])
def test_u64_all_variants_clef(n):
    keys, m = oracle_mphf(n)
    q = probe_keys(keys)
    want = O.query_u64(m, q, O.REMAP_CLEF)
    for bits in (32, 64):
        g = load(m, P.REMAP_CLEF, bits)
        for kern, kpl, blk in VARIANTS:
            say(f"[parity] n={n} bits={bits} kernel={kern} kpl={kpl} block={blk} nq={len(q)}")
            g.set_kernel(kern, kpl, blk)
            got = gpu_query(g, q, bits)
            mism = np.nonzero(got != want)[0]
            assert mism.size == 0, f"{mism.size} mismatches, first at {mism[:5]}: {got[mism[:5]]} vs {want[mism[:5]]}"


@pytest.mark.parametrize("remap", [P.REMAP_U32, P.REMAP_NONE])
@pytest.mark.parametrize("n", [1000, 300_001])
def test_u64_other_remaps(n, remap):
    keys, m = oracle_mphf(n)
    q = probe_keys(keys)
    want = O.query_u64(m, q, ORACLE_REMAP[remap])
    g = load(m, remap, 64)
    for kern, kpl, blk in VARIANTS[:1] + VARIANTS[4:6]:
        say(f"[parity] remap={remap} n={n} kernel={kern} kpl={kpl}")
        g.set_kernel(kern, kpl, blk)
        assert np.array_equal(gpu_query(g, q, 64), want)


@pytest.mark.parametrize("lam,gamma", [(3.0, O.GAMMA_LINEAR), (4.0, O.GAMMA_CUBIC)])
def test_u64_fast_and_compact(lam, gamma):
    keys, m = oracle_mphf(200_000, lam=lam, gamma=gamma)
    q = probe_keys(keys)
    for remap in (P.REMAP_CLEF, P.REMAP_U32):
        want = O.query_u64(m, q, ORACLE_REMAP[remap])
        g = load(m, remap, 32)
        say(f"[parity] lambda={lam} gamma={gamma} remap={remap}")
        assert np.array_equal(gpu_query(g, q, 32), want)


def test_u64_reseeded_mphf():
    """An MPHF whose construction needed a new seed queries with that seed."""
    n = 20_000
    keys = K.u64_keys(n, seed=4)
    try:
        m = O.build_u64(keys, params=O.params_explicit(n, 1, 15, 5000, seed=0))
    except O.BuildError:
        pytest.skip("oracle could not build this instance")
    g = load(m, P.REMAP_CLEF, 32)
    q = probe_keys(keys)
    say(f"[parity] reseeded seed={m.params.seed}")
    assert np.array_equal(gpu_query(g, q, 32), O.query_u64(m, q))


@pytest.mark.parametrize("n", [1, 5, 30_000, 200_003])
def test_bytes_parity(n):
    data, off = K.strings(n, seed=31)
    m = O.build_bytes(data, off)
    qd, qo = K.string_query_stream(n, seed=31)
    want = O.query_bytes(m, qd, qo)
    assert np.array_equal(np.sort(want), np.arange(n, dtype=np.uint64))
    g = load(m, P.REMAP_CLEF, 32, key_kind=P.KEY_BYTES)
    dt = torch.from_numpy(qd).to(DEV)
    ot = torch.from_numpy(qo.view(np.int64)).to(DEV)
    for kern, kpl, blk in VARIANTS:
        say(f"[parity-bytes] n={n} kernel={kern} kpl={kpl} block={blk}")
        g.set_kernel(kern, kpl, blk)
        got = g.query_bytes(dt, ot)
        torch.cuda.synchronize()
        got = got.cpu().numpy().view(np.uint32).astype(np.uint64)
        assert np.array_equal(got, want)


def test_bytes_unaligned_and_edge_lengths():
    """Lengths 0..40 at every byte alignment (the kernel reads aligned words
    and shifts), hashed the same as the oracle."""
    strs = [bytes([65 + (i * 7 + j) % 26 for j in range(L)]) for i, L in enumerate(list(range(41)) * 3)]
    strs = list(dict.fromkeys(strs))
    buf = b"".join(strs)
    data = np.frombuffer(buf + b"\0" * 64, dtype=np.uint8).copy()
    off = np.concatenate([[0], np.cumsum([len(s) for s in strs])]).astype(np.uint64)
    m = O.build_bytes(data, off)
    want = O.query_bytes(m, data, off)
    g = load(m, P.REMAP_CLEF, 64, key_kind=P.KEY_BYTES)
    say(f"[parity-bytes] edge lengths n={len(strs)}")
    got = g.query_bytes(torch.from_numpy(data).to(DEV), torch.from_numpy(off.view(np.int64)).to(DEV))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)


def test_empty_query_and_errors():
    keys, m = oracle_mphf(1000)
    g = load(m, P.REMAP_CLEF, 32)
    empty = torch.empty(0, dtype=torch.int64, device=DEV)
    out = torch.empty(0, dtype=torch.int32, device=DEV)
    g.query_into(empty, out)  # no launch
    with pytest.raises(P.PtrHashError) as e:
        g.query_bytes(torch.zeros(64, dtype=torch.uint8, device=DEV), torch.zeros(2, dtype=torch.int64, device=DEV))
    assert e.value.code == P.E_STATE
    torch.cuda.synchronize()


def test_overlapping_buffers_are_refused():
    """keys/out (u64), data/offsets/out (bytes) and the batches of one
    multi-MPHF launch must not overlap: E_INVAL before any launch, while
    buffers that only touch are taken."""
    keys, m = oracle_mphf(1000)
    g = load(m, P.REMAP_CLEF, 32)
    want = O.query_u64(m, keys)
    buf = torch.zeros(4096, dtype=torch.int64, device=DEV)
    buf[:1000] = torch.from_numpy(keys.view(np.int64)).to(DEV)
    k = buf[:1000]
    for lo, hi in [(0, 500), (500, 1000), (999, 1499)]:  # int32 out overlapping the keys' bytes
        with pytest.raises(P.PtrHashError) as e:
            g.query_into(k, buf[lo:hi].view(torch.int32))
        assert e.value.code == P.E_INVAL
    out = buf[1000:1500].view(torch.int32)  # starts where the keys end
    g.query_into(k, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32).astype(np.uint64), want)

    data, off = K.strings(100, seed=5)
    mb = O.build_bytes(data, off)
    gb = load(mb, P.REMAP_CLEF, 32, key_kind=P.KEY_BYTES)
    d = torch.from_numpy(data).to(DEV)
    o = torch.from_numpy(off.view(np.int64)).to(DEV)
    with pytest.raises(P.PtrHashError) as e:
        gb.query_bytes_into(d, o, d[:400].view(torch.int32))
    assert e.value.code == P.E_INVAL
    with pytest.raises(P.PtrHashError) as e:
        gb.query_bytes_into(d, o, o[:50].view(torch.int32))
    assert e.value.code == P.E_INVAL

    k2 = buf[2000:3000]
    k2.copy_(k)
    o1 = torch.empty(1000, dtype=torch.int32, device=DEV)
    with pytest.raises(P.PtrHashError) as e:  # two batches writing the same indices
        P.query_multi([(g, k, o1), (g, k2, o1)])
    assert e.value.code == P.E_INVAL
    with pytest.raises(P.PtrHashError) as e:  # one batch's out inside another batch's keys
        P.query_multi([(g, k, o1), (g, k2, k[:500].view(torch.int32))])
    assert e.value.code == P.E_INVAL
    o2 = torch.empty(1000, dtype=torch.int32, device=DEV)
    P.query_multi([(g, k, o1), (g, k2, o2)])  # two batches reading the same keys is fine
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    assert np.array_equal(o1.cpu().numpy().view(np.uint32).astype(np.uint64), want)


def test_bad_string_offsets_are_not_read():
    """The offsets live on the device, so the kernel checks them: a key whose
    end precedes its start, or ends past data_len - 16, is not read and gets
    an index of all ones; every other key keeps its index. The binding
    refuses a data tensor shorter than the last offset plus 64 bytes."""
    n = 1000
    data, off = K.strings(n, seed=3)
    m = O.build_bytes(data, off)
    want = O.query_bytes(m, data, off)
    g = load(m, P.REMAP_CLEF, 32, key_kind=P.KEY_BYTES)
    d = torch.from_numpy(data).to(DEV)
    bad_off = off.copy()
    bad_off[11] = bad_off[10] - 1  # key 10 ends before it starts; key 11 then starts after... its own start
    bad_off[n] = len(data) + 4096  # the last key ends far past the buffer
    o = torch.from_numpy(bad_off.view(np.int64)).to(DEV)
    with pytest.raises(ValueError):
        g.query_bytes(d, o)
    for kern, kpl, blk in [(P.KERNEL_PLAIN, 1, 256), (P.KERNEL_PIPELINED, 4, 256)]:
        say(f"[parity-bytes] bad offsets kernel={kern} kpl={kpl}")
        g.set_kernel(kern, kpl, blk)
        out = torch.empty(n, dtype=torch.int32, device=DEV)
        g.query_bytes_into(d, o, out, check_end=False)
        got = out.cpu().numpy().view(np.uint32).astype(np.uint64)
        assert got[10] == 0xFFFFFFFF and got[n - 1] == 0xFFFFFFFF
        keep = np.ones(n, dtype=bool)
        keep[[10, 11, n - 1]] = False  # key 11 now spans [off[10] - 1, off[12]): another string
        assert np.array_equal(got[keep], want[keep])
        want11 = O.query_bytes(m, data, np.array([bad_off[11], off[12]], dtype=np.uint64))
        assert got[11] == want11[0]
    # the same keys in a multi-MPHF batch, with a data_len below the padding refused
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    P.query_multi([(g, (d, o), out)])
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32).astype(np.uint64)
    assert got[10] == 0xFFFFFFFF and got[n - 1] == 0xFFFFFFFF
    assert np.array_equal(got[keep], want[keep])
    with pytest.raises(P.PtrHashError) as e:
        P.query_multi([(g, (d[:32], o), out)])
    assert e.value.code == P.E_INVAL


def test_device_generators_match_host():
    n = 1_000_003
    say("[gen] device generators vs host")
    k = P.gen_u64_keys(torch.empty(n, dtype=torch.int64, device=DEV), K.KEY_SEED)
    q = P.gen_query_stream(torch.empty(n, dtype=torch.int64, device=DEV), n, K.KEY_SEED, K.ORDER_SEED)
    torch.cuda.synchronize()
    assert np.array_equal(k.cpu().numpy().view(np.uint64), K.u64_keys(n))
    assert np.array_equal(q.cpu().numpy().view(np.uint64), K.query_stream(n))
    part = P.gen_query_stream(torch.empty(1000, dtype=torch.int64, device=DEV), n, K.KEY_SEED, K.ORDER_SEED,
                              start=5000)
    torch.cuda.synchronize()
    assert np.array_equal(part.cpu().numpy().view(np.uint64), K.query_stream(n, start=5000, count=1000))


def bijection_on_device(out, n):
    seen = torch.zeros(n, dtype=torch.bool, device=out.device)
    assert int(out.min()) >= 0 and int(out.max()) < n
    seen[out.long()] = True
    return bool(seen.all())


@pytest.mark.parametrize("n", [10**8])
def test_full_size_properties(n):
    """Library-built MPHF at the 10^8-key workload: all members map
    bijectively onto [0, n), every kernel variant agrees, non-members stay
    below n."""
    say(f"[full] n={n}: host keys + library build")
    keys = K.u64_keys(n)
    b = P.build_u64(keys, index_bits=32)
    del keys
    g = P.Mphf.from_built(b)
    q = P.gen_query_stream(torch.empty(n, dtype=torch.int64, device=DEV), n, K.KEY_SEED, K.ORDER_SEED)
    ref = None
    for kern, kpl, blk in [(P.KERNEL_PLAIN, 1, 256), (P.KERNEL_PIPELINED, 4, 256), (P.KERNEL_PIPELINED, 8, 512)]:
        say(f"[full] n={n} kernel={kern} kpl={kpl} block={blk}")
        g.set_kernel(kern, kpl, blk)
        out = g.query(q)
        torch.cuda.synchronize()
        if ref is None:
            assert bijection_on_device(out, n)
            ref = out
        else:
            assert torch.equal(out, ref)
    nm = torch.from_numpy(K.nonmember_keys(1_000_000).view(np.int64)).to(DEV)
    o = g.query(nm)
    torch.cuda.synchronize()
    assert int(o.long().max()) < n


def test_device_string_generator_matches_host():
    n = 5000
    say("[gen] device strings vs host")
    d, o = P.gen_strings(n, 7)
    hd, ho = K.strings(n, seed=7)
    assert np.array_equal(o.cpu().numpy().view(np.uint64), ho)
    assert np.array_equal(d.cpu().numpy()[: int(ho[-1])], hd[: int(ho[-1])])
    qd, qo = P.gen_strings(n, 7, K.ORDER_SEED, shuffled=True)
    hqd, hqo = K.string_query_stream(n, seed=7, order_seed=K.ORDER_SEED)
    assert np.array_equal(qo.cpu().numpy().view(np.uint64), hqo)
    assert np.array_equal(qd.cpu().numpy()[: int(hqo[-1])], hqd[: int(hqo[-1])])


def test_occupancy_cap_and_autotuner(tmp_path, monkeypatch):
    """Occupancy caps change only speed, never indices; the autotuner
    applies its winner and answers the next call from its cache."""
    from paper_2502_15539_amd import autotune

    keys, m = oracle_mphf(65_537)
    q = probe_keys(keys)
    want = O.query_u64(m, q)
    g = load(m, P.REMAP_CLEF, 32)
    for occ in (1, 2, 4, 0):
        g.set_kernel(P.KERNEL_PIPELINED, 4, 256)
        eff = g.set_occupancy(occ)
        say(f"[tune] occupancy {occ} -> {eff}")
        assert np.array_equal(gpu_query(g, q, 32), want)
    monkeypatch.setenv("PTRHASH_TUNE_CACHE", str(tmp_path / "tune.json"))
    qt = torch.from_numpy(q.view(np.int64)).to(DEV)
    out = torch.empty(len(q), dtype=torch.int32, device=DEV)
    cands = autotune.candidates(kpls=(1, 4), blocks=(256,), occupancy=(0, 2))
    best, res = autotune.tune(torch, g, lambda: g.query_into(qt, out), len(q), cands=cands, reps=1)
    assert best in res and len(res) == len(cands)
    best2, res2 = autotune.tune(torch, g, lambda: g.query_into(qt, out), len(q), cands=cands, reps=1)
    assert best2 == best and res2 == {}
    g.query_into(qt, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32).astype(np.uint64), want)


@pytest.mark.parametrize("n", [1, 3, 1000, 12_345, 100_000])
def test_single_part_mod_reduce_parity(n):
    keys = K.u64_keys(n, seed=55)
    m = O.build_u64(keys, params=O.params_single_mod(n))
    q = probe_keys(keys)
    for remap in (P.REMAP_CLEF, P.REMAP_U32, P.REMAP_NONE):
        want = O.query_u64(m, q, ORACLE_REMAP[remap])
        g = load(m, remap, 32)
        for kern, kpl, blk in VARIANTS[:1] + VARIANTS[4:6]:
            say(f"[parity] single-part mod n={n} remap={remap} kernel={kern} kpl={kpl}")
            g.set_kernel(kern, kpl, blk)
            assert np.array_equal(gpu_query(g, q, 32), want)


@pytest.mark.parametrize("n", [1, 2, 1000, 250_000, 2_000_000])
def test_device_front_half_build_equals_oracle(n):
    """Hash + radix sort on the device, pilot search on the host: the same
    pilots and remap bytes as the oracle's construction."""
    keys = K.u64_keys(n, seed=321)
    say(f"[build-device] n={n}")
    kt = torch.from_numpy(keys.view(np.int64)).to(DEV)
    b = P.build_u64_device(kt, threads=8, placement="host")
    assert b.placement == "host"
    m = O.build_u64(keys)
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)
    assert b.params.seed == m.params.seed


def test_device_front_half_rejects_duplicates():
    keys = K.u64_keys(5000, seed=3)
    keys[4000] = keys[12]
    with pytest.raises(P.PtrHashError) as e:
        P.build_u64_device(torch.from_numpy(keys.view(np.int64)).to(DEV), placement="host")
    assert e.value.code == P.E_DUPLICATE


@pytest.mark.parametrize("n", [7, 30_000])
def test_bytes_hash128_parity(n):
    data, off = K.strings(n, seed=41)
    o = O.params_for(n)
    o.hash_bits = 128
    m = O.build_bytes(data, off, params=o)
    qd, qo = K.string_query_stream(n, seed=41)
    want = O.query_bytes(m, qd, qo)
    g = load(m, P.REMAP_CLEF, 32, key_kind=P.KEY_BYTES)
    assert g.params.hash_bits == 128
    dt = torch.from_numpy(qd).to(DEV)
    ot = torch.from_numpy(qo.view(np.int64)).to(DEV)
    for kern, kpl, blk in VARIANTS[:1] + VARIANTS[3:6]:
        say(f"[parity-bytes128] n={n} kernel={kern} kpl={kpl}")
        g.set_kernel(kern, kpl, blk)
        got = g.query_bytes(dt, ot)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().view(np.uint32).astype(np.uint64), want)
