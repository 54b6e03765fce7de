"""The seeded input generators: slices and position lookups agree with the
whole stream, keys are distinct, the shuffle is a permutation, and string
lengths and bytes follow the stated recipe."""
import numpy as np

from paper_2502_15539_amd import keygen as K


def test_permutation_is_bijection():
    for n in (1, 2, 3, 1000, 65537):
        p = K.Permutation(n, seed=5)(np.arange(n, dtype=np.uint64))
        assert np.array_equal(np.sort(p), np.arange(n, dtype=np.uint64))


def test_keys_distinct_and_slices_agree():
    n = 200_000
    keys = K.u64_keys(n)
    assert len(np.unique(keys)) == n
    assert np.array_equal(K.u64_keys(n, start=1234, count=999), keys[1234:1234 + 999])


def test_query_stream_is_shuffled_member_set():
    n = 100_000
    q = K.query_stream(n)
    assert np.array_equal(np.sort(q), np.sort(K.u64_keys(n)))
    assert not np.array_equal(q, K.u64_keys(n))
    assert np.array_equal(K.query_stream(n, start=777, count=100), q[777:877])
    pos = np.array([0, 5, n - 1, 31337, 4242], dtype=np.uint64)
    assert np.array_equal(K.query_stream_at(n, pos), q[pos.astype(np.int64)])


def test_strings_recipe_and_lookups():
    d, o = K.strings(3000, seed=9)
    lens = np.diff(o.astype(np.int64))
    assert lens.min() >= K.STR_MIN and lens.max() <= K.STR_MAX
    body = d[: int(o[-1])]
    assert body.min() >= 0x20 and body.max() <= 0x7E
    assert np.all(d[int(o[-1]):] == 0) and len(d) - int(o[-1]) == K.STR_PAD
    da, oa = K.strings_at(np.arange(3000), seed=9)
    assert np.array_equal(da, d) and np.array_equal(oa, o)
    ds, os_ = K.strings(100, seed=9, start=1500)
    db, ob = K.strings_at(np.arange(1500, 1600), seed=9)
    assert np.array_equal(ds, db) and np.array_equal(os_, ob)


def test_string_query_stream_lookup():
    qd, qo = K.string_query_stream(4000, seed=3, order_seed=4)
    pos = np.array([0, 17, 3999, 2500, 17], dtype=np.uint64)
    d, o = K.string_query_stream_at(4000, pos, seed=3, order_seed=4)
    for j, i in enumerate(pos.astype(np.int64)):
        assert bytes(qd[qo[i]:qo[i + 1]]) == bytes(d[o[j]:o[j + 1]])
