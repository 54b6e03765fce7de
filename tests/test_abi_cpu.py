"""Host-side checks of the C-ABI library that need no GPU: every declared
symbol is exported, the parameter rule agrees with the oracle's, argument
validation, and the host construction reproduces the oracle's construction
byte for byte (same pilots, same remap table)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K
from paper_2502_15539_amd import ptrhash as P

from .mphf_pairs import lib_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "ptrhash.h")).read()
    return sorted(set(re.findall(r"PTRHASH_API\s+[\w\s\*]+?\b(ptrhash_\w+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert len(syms) >= 15
    L = C.CDLL(P.LIB_PATH)
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    assert set(syms) <= set(P._SIGS), set(syms) - set(P._SIGS)


@pytest.mark.parametrize("n", [1, 2, 3, 10, 1000, 80000, 217000, 10**6, 12_345_678, 10**8, 3 * 10**8, 10**9,
                               10**10])
@pytest.mark.parametrize("preset,lam,gamma", [(P.PRESET_DEFAULT, 3.5, 0), (P.PRESET_FAST, 3.0, 1),
                                              (P.PRESET_COMPACT, 4.0, 0)])
def test_params_match_oracle(n, preset, lam, gamma):
    if preset == P.PRESET_FAST and n > 2**32:
        with pytest.raises(P.PtrHashError) as e:  # u32 remap entries cannot hold indices >= 2^32
            P.params_default(n, preset, index_bits=64)
        assert e.value.code == P.E_RANGE
        return
    p = P.params_default(n, preset, index_bits=64)
    o = O.params_for(n, 0.99, lam, gamma=gamma)
    assert (p.num_parts, p.log2_slots, p.buckets_per_part, p.remap_len, p.gamma) == (
        o.num_parts, o.log2_slots, o.buckets_per_part, o.remap_len, o.gamma)


def test_index_bits_default_and_range():
    assert P.params_default(10**6).index_bits == 32
    assert P.params_default(5 * 10**9).index_bits == 64
    with pytest.raises(P.PtrHashError) as e:
        P.params_default(5 * 10**9, index_bits=32)
    assert e.value.code == P.E_RANGE


def test_remap_bytes():
    p = P.params_default(10**9)
    assert P.remap_bytes(p) == -(-p.remap_len // 44) * 64
    pf = P.params_default(10**6, P.PRESET_FAST)
    assert P.remap_bytes(pf) == 4 * pf.remap_len


def test_load_rejects_bad_params_without_touching_the_device():
    good = P.params_default(1000)
    pilots = np.zeros(good.num_parts * good.buckets_per_part, dtype=np.uint8)
    remap = np.zeros(P.remap_bytes(good), dtype=np.uint8)
    cases = {
        "remap_len": dict(remap_len=good.remap_len + 1),
        "n0": dict(n=0),
        "parts0": dict(num_parts=0),
        "buckets0": dict(buckets_per_part=0),
        "gamma": dict(gamma=7),
        "remap_kind": dict(remap_kind=9),
        "index_bits": dict(index_bits=16),
        "key_kind": dict(key_kind=3),
        "small": dict(log2_slots=2),
    }
    for name, change in cases.items():
        p = good.copy()
        for k, v in change.items():
            setattr(p, k, v)
        m = P.Mphf()
        with pytest.raises(P.PtrHashError) as e:
            m.load(p, pilots, remap)
        assert e.value.code in (P.E_INVAL, P.E_RANGE), name
    m = P.Mphf()
    with pytest.raises(P.PtrHashError) as e:
        m.load(good, pilots, None)  # CacheLineEF bytes needed
    assert e.value.code == P.E_INVAL


def test_query_needs_loaded_handle():
    m = P.Mphf()
    with pytest.raises(P.PtrHashError) as e:
        P._check(P.lib().ptrhash_query(m.handle, None, 10, None, None), "q")
    assert e.value.code == P.E_STATE
    with pytest.raises(P.PtrHashError) as e:
        m.set_kernel(P.KERNEL_PIPELINED, 3, 256)
    assert e.value.code == P.E_INVAL
    with pytest.raises(P.PtrHashError):
        m.set_kernel(P.KERNEL_PIPELINED, 4, 100)
    assert P.lib().ptrhash_destroy(None) == P.OK


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 0), (7, 3), (1000, 0), (4097, 9), (250_000, 1), (1_000_000, 0),
                                    (3_000_000, 5)])
def test_builder_equals_oracle_default(n, seed):
    keys = K.u64_keys(n, seed=100 + seed)
    b = P.build_u64(keys, seed=seed)
    m = O.build_u64(keys, seed=seed)
    assert b.params.seed == m.params.seed
    assert np.array_equal(b.pilots, m.pilots)
    assert np.array_equal(b.remap, m.clef)
    assert b.info.evictions == m.stats.evictions


@pytest.mark.parametrize("preset,lam,gamma", [(P.PRESET_FAST, 3.0, O.GAMMA_LINEAR),
                                              (P.PRESET_COMPACT, 4.0, O.GAMMA_CUBIC)])
def test_builder_equals_oracle_presets(preset, lam, gamma):
    n = 400_000
    keys = K.u64_keys(n, seed=21)
    b = P.build_u64(keys, preset=preset)
    m = O.build_u64(keys, lam=lam, gamma=gamma)
    assert np.array_equal(b.pilots, m.pilots)
    if preset == P.PRESET_FAST:
        assert np.array_equal(b.remap.view(np.uint32), m.F.astype(np.uint32))
    else:
        assert np.array_equal(b.remap, m.clef)


def test_builder_equals_oracle_strings():
    data, off = K.strings(60_000, seed=13)
    b = P.build_bytes(data, off)
    m = O.build_bytes(data, off)
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)


def test_builder_reseeds_like_oracle():
    """Explicit parameters with little slack force failed attempts; both
    constructions must reseed the same way and agree on the result."""
    n = 20_000
    keys = K.u64_keys(n, seed=4)
    o = O.params_explicit(n, 1, 15, 5000, seed=0)  # S = 32768, lambda = 4
    try:
        m = O.build_u64(keys, params=o)
    except O.BuildError:
        pytest.skip("oracle could not build this instance")
    p = lib_params(m)
    p.seed = 0
    p.index_bits = 32
    b = P.build_u64(keys, params=p)
    assert b.params.seed == m.params.seed
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)


def test_builder_errors():
    keys = K.u64_keys(1000)
    keys[10] = keys[11]
    with pytest.raises(P.PtrHashError) as e:
        P.build_u64(keys)
    assert e.value.code == P.E_DUPLICATE
    p = P.params_default(1000)
    with pytest.raises(P.PtrHashError) as e:
        P.build_u64(K.u64_keys(999), params=p)
    assert e.value.code == P.E_INVAL


@pytest.mark.parametrize("n", [1, 2, 3, 100, 5000, 77_777, 129_000])
def test_single_mod_params_and_builder_match_oracle(n):
    p = P.params_default(n, P.PRESET_DEFAULT | P.PRESET_SINGLE_MOD)
    o = O.params_single_mod(n)
    assert p.reduce_kind == P.REDUCE_MOD and p.num_parts == 1
    assert (p.slots, p.buckets_per_part, p.remap_len) == (o.slots_per_part, o.buckets_per_part, o.remap_len)
    keys = K.u64_keys(n, seed=17)
    b = P.build_u64(keys, params=p)
    m = O.build_u64(keys, params=o)
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)


def test_single_mod_flag_keeps_multi_part_rule():
    p = P.params_default(10**6, P.PRESET_DEFAULT | P.PRESET_SINGLE_MOD)
    assert p.reduce_kind == P.REDUCE_POW2 and p.num_parts == 4


def test_hash128_builder_equals_oracle():
    data, off = K.strings(50_000, seed=19)
    o = O.params_for(50_000)
    o.hash_bits = 128
    m = O.build_bytes(data, off, params=o)
    p = P.params_default(50_000, key_kind=P.KEY_BYTES)
    assert p.hash_bits == 64
    p.hash_bits = 128
    b = P.build_bytes(data, off, params=p)
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)


def test_hash128_params_rule():
    assert P.params_default(5 * 10**9, key_kind=P.KEY_BYTES).hash_bits == 128
    assert P.params_default(10**9, key_kind=P.KEY_BYTES).hash_bits == 64
    p = P.params_default(1000)
    p.hash_bits = 128  # only byte keys take 128-bit hashing
    m = P.Mphf()
    with pytest.raises(P.PtrHashError) as e:
        m.load(p, np.zeros(p.num_parts * p.buckets_per_part, np.uint8), np.zeros(P.remap_bytes(p), np.uint8))
    assert e.value.code == P.E_INVAL


def test_device_build_rejects_bad_arguments_before_any_device_call():
    import ctypes as C

    p = P.params_default(1000)
    pil = np.zeros(p.num_parts * p.buckets_per_part, dtype=np.uint8)
    rm = np.zeros(P.remap_bytes(p), dtype=np.uint8)
    f = P.lib().ptrhash_build_u64_gpu
    # NULL keys
    assert f(None, 1000, C.byref(p), pil.ctypes.data, rm.ctypes.data, None, None) == P.E_INVAL
    # n disagrees with params->n (checked before the keys are touched)
    assert f(C.c_void_p(16), 999, C.byref(p), pil.ctypes.data, rm.ctypes.data, None, None) == P.E_INVAL
    # byte-key params
    q = P.params_default(1000, key_kind=P.KEY_BYTES)
    assert f(C.c_void_p(16), 1000, C.byref(q), pil.ctypes.data, rm.ctypes.data, None, None) == P.E_INVAL
    assert b"key_kind" in P.lib().ptrhash_last_error()


def test_multi_launch_shape_validation_without_device():
    f = P.lib().ptrhash_set_multi_kernel
    for bad in [(3, 256, 0), (16, 256, 0), (4, 32, 0), (4, 1088, 0), (4, 100, 0), (4, 256, -1), (4, 256, 65)]:
        assert f(*bad) == P.E_INVAL, bad
    assert f(4, 256, 0) == P.OK  # the initial default
    with pytest.raises(P.PtrHashError) as e:
        P.Server(multi_kernel=(5, 256, 0))
    assert e.value.code == P.E_INVAL


def test_device_string_build_rejects_bad_arguments_before_any_device_call():
    import ctypes as C

    p = P.params_default(1000, key_kind=P.KEY_BYTES)
    pil = np.zeros(p.num_parts * p.buckets_per_part, dtype=np.uint8)
    rm = np.zeros(P.remap_bytes(p), dtype=np.uint8)
    f = P.lib().ptrhash_build_bytes_gpu
    assert f(None, 1 << 20, C.c_void_p(64), 1000, C.byref(p), pil.ctypes.data, rm.ctypes.data, None,
             None) == P.E_INVAL
    assert f(C.c_void_p(67), 1 << 20, C.c_void_p(64), 1000, C.byref(p), pil.ctypes.data, rm.ctypes.data, None,
             None) == P.E_INVAL  # unaligned data
    assert f(C.c_void_p(64), 63, C.c_void_p(64), 1000, C.byref(p), pil.ctypes.data, rm.ctypes.data, None,
             None) == P.E_INVAL  # no room for the padding
    q = P.params_default(1000)  # u64-key params
    assert f(C.c_void_p(64), 1 << 20, C.c_void_p(64), 1000, C.byref(q), pil.ctypes.data, rm.ctypes.data, None,
             None) == P.E_INVAL


def test_host_string_build_checks_offsets_before_reading():
    """Decreasing offsets, or strings that end past data_len, are refused
    with E_INVAL before any string is read."""
    data, off = K.strings(1000, seed=2)
    ok = P.build_bytes(data, off)
    assert ok.params.n == 1000
    bad = off.copy()
    bad[500] = bad[499] - 1
    with pytest.raises(P.PtrHashError) as e:
        P.build_bytes(data, bad)
    assert e.value.code == P.E_INVAL
    with pytest.raises(P.PtrHashError) as e:
        P.build_bytes(data[: int(off[-1]) - 1], off)
    assert e.value.code == P.E_INVAL


def test_builder_equals_oracle_one_huge_bucket():
    """All 2100 keys in one bucket (one part of 2^20 slots): the host search
    places it like the oracle (the device search stops at 2048 keys)."""
    n = 2100
    keys = K.u64_keys(n, seed=21)
    m = O.build_u64(keys, params=O.params_explicit(n, 1, 20, 1))
    b = P.build_u64(keys, params=lib_params(m, P.REMAP_CLEF, 32), threads=2)
    assert b.info.max_bucket_size == n == m.stats.max_bucket_size
    assert b.params.seed == m.params.seed
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)


def test_probe_arguments_checked_before_any_device_call():
    """The benchmark probes refuse bad arguments on the host: a scatter whose
    in and out overlap or whose size is out of range, and a single-launch
    probe of 2^32 or more work-items (grid times block)."""
    L = P.lib()
    a = np.zeros(512, dtype=np.uint64)
    b = np.zeros(512, dtype=np.uint64)
    pa, pb = C.c_void_p(a.ctypes.data), C.c_void_p(b.ctypes.data)
    assert L.ptrhash_bench_scatter(pa, 8, C.c_void_p(a.ctypes.data + 8 * 100), None) == P.E_INVAL
    assert L.ptrhash_bench_scatter(pa, 7, pb, None) == P.E_INVAL
    assert L.ptrhash_bench_scatter(pa, 35, pb, None) == P.E_INVAL
    assert L.ptrhash_bench_scatter(None, 8, pb, None) == P.E_INVAL
    for kpl, block in [(1, 64), (1, 1024), (2, 256)]:
        n_q = (2**32 // block + 1) * block * kpl  # one workgroup past 2^32 work-items
        assert L.ptrhash_bench_copy(pa, n_q, pb, kpl, block, None) == P.E_RANGE
        assert L.ptrhash_bench_gather(pa, n_q, pa, 256, pb, kpl, block, 0, None) == P.E_RANGE


def test_query_entry_points_need_a_loaded_handle_first():
    """Queries on an empty handle fail with E_STATE whatever the buffers
    (the overlap and padding checks need the loaded index width)."""
    h = C.c_void_p()
    assert P.lib().ptrhash_create(C.byref(h)) == P.OK
    a = np.zeros(128, dtype=np.uint64)
    pa = C.c_void_p(a.ctypes.data)
    assert P.lib().ptrhash_query(h, pa, 10, pa, None) == P.E_STATE
    assert P.lib().ptrhash_query_bytes(h, pa, 8, pa, 10, pa, None) == P.E_STATE
    assert P.lib().ptrhash_bench_gather_buckets(h, pa, 10, pa, 1, 256, 0, None) == P.E_STATE
    assert P.lib().ptrhash_destroy(h) == P.OK
