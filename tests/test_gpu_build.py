"""Construction with the pilot search on the device.

The oracle builds the same keys with the same parameters; the device build
must give the same seed, the same pilots and the same remap bytes. Beyond
the oracle's reach (10^8 keys) the device search must equal the library's
host search byte for byte.
"""
import os
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K
from paper_2502_15539_amd import ptrhash as P

from .mphf_pairs import lib_params

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(keys):
    return torch.from_numpy(keys.view(np.int64)).to(DEV)


def same(b, m, remap_kind=P.REMAP_CLEF):
    assert b.placement == "device"
    assert b.params.seed == m.params.seed
    assert np.array_equal(b.pilots, m.pilots)
    want = m.clef if remap_kind == P.REMAP_CLEF else m.F.astype(np.uint32).view(np.uint8)
    assert np.array_equal(b.remap, want)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 1000, 40_000, 250_000, 2_000_000])
def test_device_search_equals_oracle_default(n):
    keys = K.u64_keys(n, seed=1000 + n % 97)
    say(f"[gpu-build] default n={n}")
    b = P.build_u64_device(dev(keys), placement="device")
    m = O.build_u64(keys)
    assert (b.params.num_parts, b.params.log2_slots, b.params.buckets_per_part) == \
        (m.params.num_parts, m.params.log2_slots, m.params.buckets_per_part)
    same(b, m)
    assert b.info.max_bucket_size == m.stats.max_bucket_size


@pytest.mark.parametrize("preset,lam,gamma,remap", [(P.PRESET_FAST, 3.0, O.GAMMA_LINEAR, P.REMAP_U32),
                                                    (P.PRESET_COMPACT, 4.0, O.GAMMA_CUBIC, P.REMAP_CLEF)])
def test_device_search_equals_oracle_presets(preset, lam, gamma, remap):
    n = 300_000
    keys = K.u64_keys(n, seed=77)
    say(f"[gpu-build] preset={preset} n={n}")
    b = P.build_u64_device(dev(keys), placement="device", preset=preset, index_bits=32)
    m = O.build_u64(keys, lam=lam, gamma=gamma)
    assert b.params.remap_kind == remap
    same(b, m, remap)


@pytest.mark.parametrize("n", [1, 3, 1000, 77_777])
def test_device_search_single_part_mod(n):
    keys = K.u64_keys(n, seed=55)
    say(f"[gpu-build] single-part mod n={n}")
    p = P.params_default(n, P.PRESET_DEFAULT | P.PRESET_SINGLE_MOD)
    b = P.build_u64_device(dev(keys), params=p, placement="device")
    m = O.build_u64(keys, params=O.params_single_mod(n))
    same(b, m)


def test_device_search_reseeds_like_oracle():
    """Little slack (lambda = 4 with S = 2^15 for 20000 keys) makes
    attempts fail; the device must step through the seeds like the oracle."""
    n = 20_000
    keys = K.u64_keys(n, seed=4)
    o = O.params_explicit(n, 1, 15, 5000, seed=0)
    try:
        m = O.build_u64(keys, params=o)
    except O.BuildError:
        pytest.skip("oracle could not build this instance")
    p = lib_params(m)
    p.seed = 0
    p.index_bits = 32
    say(f"[gpu-build] reseed n={n}")
    b = P.build_u64_device(dev(keys), params=p, placement="device")
    same(b, m)
    assert b.info.attempts == m.stats.attempts


# oracle attempts: 1, 1, 2, 3, 5, 9, and all 16 seeds failing
@pytest.mark.parametrize("n,P_,log2,lam,kseed", [(20_000, 1, 15, 4.0, 4), (250_000, 1, 18, 3.5, 8),
                                                  (30_000, 4, 13, 4.5, 20), (60_000, 8, 13, 4.5, 39),
                                                  (30_000, 4, 13, 4.5, 33), (30_500, 4, 13, 4.5, 39),
                                                  (30_000, 4, 13, 4.5, 38)])
@pytest.mark.parametrize("stuck_ms", ["0", None])
def test_side_by_side_seeds_equal_oracle(n, P_, log2, lam, kseed, stuck_ms, monkeypatch):
    """With every search counted as stuck at once (PTRHASH_SPECULATE_MS=0)
    up to four seeds are searched side by side and later ones cancelled when
    an earlier one succeeds; without it, one seed after the other. Either
    way the result must be the oracle's (same seed, pilots, remap and number
    of attempts), whether seed 0 succeeds, several fail, or all do."""
    if stuck_ms is None:
        monkeypatch.delenv("PTRHASH_SPECULATE_MS", raising=False)  # one seed after the other
    else:
        monkeypatch.setenv("PTRHASH_SPECULATE_MS", stuck_ms)
    keys = K.u64_keys(n, seed=kseed)
    B = int(np.ceil(0.99 * (1 << log2) / lam))
    o = O.params_explicit(n, P_, log2, B, seed=0)
    say(f"[gpu-build] side by side n={n} P={P_} S=2^{log2} lambda={lam}")
    try:
        m = O.build_u64(keys, params=o)
    except O.BuildError:
        q = P.params_default(n)
        q.num_parts, q.log2_slots, q.buckets_per_part, q.remap_len, q.seed = P_, log2, B, o.remap_len, 0
        with pytest.raises(P.PtrHashError) as e:
            P.build_u64_device(dev(keys), params=q, placement="device")
        assert e.value.code == P.E_BUILD
        return
    p = lib_params(m)
    p.seed = 0
    b = P.build_u64_device(dev(keys), params=p, placement="device")
    same(b, m)
    assert b.info.attempts == m.stats.attempts
    say(f"[gpu-build] attempts {b.info.attempts}")


@pytest.mark.parametrize("helpers", ["0", "1", "2", "6", "7"])
def test_device_search_helper_counts_equal_oracle(helpers, monkeypatch):
    """Every count of look-ahead wavefronts (the default is 7; 0 runs the
    placing wavefront alone) gives the oracle's pilots: at the default
    parameters, with Compact's heavy evictions at S = 2^13, and with a
    failing seed."""
    monkeypatch.setenv("PTRHASH_SEARCH_HELPERS", helpers)
    say(f"[gpu-build] look-ahead wavefronts {helpers}")
    keys = K.u64_keys(600_000, seed=91)
    b = P.build_u64_device(dev(keys), placement="device")
    same(b, O.build_u64(keys))
    for n, P_, log2, lam, kseed in [(30_000, 4, 13, 4.5, 20), (20_000, 1, 15, 4.0, 4)]:
        keys = K.u64_keys(n, seed=kseed)
        B = int(np.ceil(0.99 * (1 << log2) / lam))
        m = O.build_u64(keys, params=O.params_explicit(n, P_, log2, B, seed=0))
        p = lib_params(m)
        p.seed = 0
        b = P.build_u64_device(dev(keys), params=p, placement="device")
        same(b, m)
        assert b.info.attempts == m.stats.attempts


@pytest.mark.parametrize("parts,lam", [(1, 3.5), (2, 3.5), (2, 4.0)])
def test_device_search_equals_oracle_at_full_part_size(parts, lam):
    """S = 2^20 slots per part, the part size the parameter rule of Section
    3.1 ("Parameter values") gives every set beyond about 5*10^7 keys, so the
    geometry every benchmark MPHF is built with: a 128 KiB taken-slot
    bitvector that fills the workgroup's LDS. n = floor(0.99 * P * S) keys
    (alpha = 0.99) and B = ceil(0.99 * S / lambda), Default (lambda = 3.5)
    and Compact (lambda = 4.0): same seed, pilots, remap bytes and eviction
    count as the oracle."""
    log2 = 20
    n = int(0.99 * parts * (1 << log2))
    B = int(np.ceil(0.99 * (1 << log2) / lam))
    keys = K.u64_keys(n, seed=2020 + parts)
    say(f"[gpu-build] S=2^20 P={parts} lambda={lam} n={n}")
    m = O.build_u64(keys, params=O.params_explicit(n, parts, log2, B, seed=0))
    p = lib_params(m, P.REMAP_CLEF, 32)
    p.seed = 0
    b = P.build_u64_device(dev(keys), params=p, placement="device")
    same(b, m)
    assert b.info.attempts == m.stats.attempts
    assert b.info.evictions == m.stats.evictions
    assert b.info.max_part_evictions == m.stats.max_part_evictions


def test_device_string_search_equals_oracle_at_full_part_size():
    """Byte keys at S = 2^20 (two parts, alpha = 0.99, Default lambda)."""
    log2, parts = 20, 2
    n = int(0.99 * parts * (1 << log2))
    B = int(np.ceil(0.99 * (1 << log2) / 3.5))
    data, off = K.strings(n, seed=2022)
    say(f"[gpu-build] strings S=2^20 P={parts} n={n}")
    m = O.build_bytes(data, off, params=O.params_explicit(n, parts, log2, B, seed=0))
    p = lib_params(m, P.REMAP_CLEF, 32, P.KEY_BYTES)
    p.seed = 0
    b = P.build_bytes_device(*dev_strings(data, off), params=p, placement="device")
    same(b, m)
    assert b.info.evictions == m.stats.evictions


def test_device_search_errors():
    keys = K.u64_keys(5000, seed=3)
    keys[4000] = keys[12]
    say("[gpu-build] duplicates")
    with pytest.raises(P.PtrHashError) as e:
        P.build_u64_device(dev(keys), placement="device")
    assert e.value.code == P.E_DUPLICATE
    # S = 2^21 needs 256 KiB of LDS per part: outside the device search
    n = 300_000
    o = O.params_explicit(n, 1, 21, 150_000)
    p = P.params_default(n)
    p.num_parts, p.log2_slots, p.buckets_per_part, p.remap_len = 1, 21, 150_000, o.remap_len
    with pytest.raises(P.PtrHashError) as e:
        P.build_u64_device(dev(K.u64_keys(n)), params=p, placement="device")
    assert e.value.code == P.E_RANGE
    b = P.build_u64_device(dev(K.u64_keys(n)), params=p, placement="auto")
    assert b.placement == "host"


def test_device_search_bucket_limit_falls_back_to_host():
    """One bucket of 2100 keys (over the device search's 2048-key limit):
    the device search refuses it with E_RANGE before any launch, and the
    automatic placement builds it on the host, equal to the oracle."""
    n = 2100
    keys = K.u64_keys(n, seed=21)
    m = O.build_u64(keys, params=O.params_explicit(n, 1, 20, 1))
    q = lib_params(m, P.REMAP_CLEF, 32)
    say(f"[gpu-build] one bucket of {n} keys")
    with pytest.raises(P.PtrHashError) as e:
        P.build_u64_device(dev(keys), params=q, placement="device")
    assert e.value.code == P.E_RANGE
    b = P.build_u64_device(dev(keys), params=q, placement="auto")
    assert b.placement == "host" and b.info.max_bucket_size == n
    assert b.params.seed == m.params.seed
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)


def test_device_search_equals_host_search_1e8():
    n = 10**8
    say(f"[gpu-build] n={n}: device keys, device search vs host search")
    keys = P.gen_u64_keys(torch.empty(n, dtype=torch.int64, device=DEV), K.KEY_SEED)
    t0 = time.time()
    bd = P.build_u64_device(keys, placement="device")
    t1 = time.time()
    bh = P.build_u64_device(keys, placement="host", threads=min(16, os.cpu_count() or 1))
    t2 = time.time()
    say(f"[gpu-build] device {t1 - t0:.2f} s, host search {t2 - t1:.2f} s, evictions {bd.info.evictions}")
    assert bd.placement == "device" and bh.placement == "host"
    assert bd.params.seed == bh.params.seed
    assert bd.info.evictions == bh.info.evictions
    assert np.array_equal(bd.pilots, bh.pilots) and np.array_equal(bd.remap, bh.remap)


def dev_strings(data, off):
    return torch.from_numpy(data).to(DEV), torch.from_numpy(off.view(np.int64)).to(DEV)


@pytest.mark.parametrize("n", [1, 7, 1000, 30_000, 300_000])
def test_device_string_build_equals_oracle(n):
    data, off = K.strings(n, seed=61 + n % 13)
    say(f"[gpu-build] strings n={n}")
    b = P.build_bytes_device(*dev_strings(data, off), placement="device", index_bits=32)
    m = O.build_bytes(data, off)
    same(b, m)


@pytest.mark.parametrize("n", [1, 7, 1000, 30_000, 300_000])
def test_device_string_build_hash128_equals_oracle(n):
    """128-bit string hashes (what the parameter rule takes beyond 2^32 keys):
    part and bucket from the high half, the slot from the low half."""
    data, off = K.strings(n, seed=71 + n % 11)
    say(f"[gpu-build] strings n={n}, 128-bit hashes")
    p = P.params_default(n, key_kind=P.KEY_BYTES, index_bits=32)
    p.hash_bits = 128
    b = P.build_bytes_device(*dev_strings(data, off), params=p, placement="device")
    o = O.params_for(n)
    o.hash_bits = 128
    m = O.build_bytes(data, off, params=o)
    same(b, m)
    # and the query of the members, through the 128-bit query kernel, is the oracle's
    g = P.Mphf.from_built(b)
    got = g.query_bytes(*dev_strings(data, off))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint32).astype(np.uint64), O.query_bytes(m, data, off))


def test_device_string_build_errors_and_host_agreement():
    n = 3_000_000
    data, off = K.strings(n, seed=9)
    d, o = dev_strings(data, off)
    say(f"[gpu-build] strings n={n}: device vs host construction")
    bd = P.build_bytes_device(d, o, placement="device")
    bh = P.build_bytes(data, off, threads=min(16, os.cpu_count() or 1))
    assert bd.params.seed == bh.params.seed
    assert np.array_equal(bd.pilots, bh.pilots) and np.array_equal(bd.remap, bh.remap)
    # a repeated string
    data2, off2 = K.strings(5000, seed=3)
    lens = np.diff(off2.astype(np.int64))
    same_len = np.nonzero(lens == lens[10])[0]
    j = int(same_len[same_len != 10][0])
    data2[off2[j]:off2[j + 1]] = data2[off2[10]:off2[11]]
    with pytest.raises(P.PtrHashError) as e:
        P.build_bytes_device(*dev_strings(data2, off2), placement="device")
    assert e.value.code == P.E_DUPLICATE
    # offsets checked on the device before any string is read
    data3, off3 = K.strings(5000, seed=4)
    bad = off3.copy()
    bad[100] = bad[99] - 1
    with pytest.raises(P.PtrHashError) as e:
        P.build_bytes_device(*dev_strings(data3, bad), placement="device")
    assert e.value.code == P.E_INVAL
    d3, o3 = dev_strings(data3, off3)
    with pytest.raises(P.PtrHashError) as e:  # the last string ends less than 16 bytes before the buffer does
        P.build_bytes_device(d3[: int(off3[-1]) + 8], o3, placement="device")
    assert e.value.code == P.E_INVAL
    # 128-bit string hashes: the device build equals the host build
    p = P.params_default(1000, key_kind=P.KEY_BYTES)
    p.hash_bits = 128
    d3, o3 = dev_strings(*K.strings(1000, seed=5))
    bd = P.build_bytes_device(d3, o3, params=p.copy(), placement="device")
    bh = P.build_bytes_device(d3, o3, params=p.copy(), placement="host")
    assert bd.placement == "device" and bh.placement == "host"
    assert bd.params.seed == bh.params.seed
    assert np.array_equal(bd.pilots, bh.pilots) and np.array_equal(bd.remap, bh.remap)
