"""The multi-MPHF entry point that allocates nothing
(ptrhash_query_multi_noalloc) against ptrhash_query_multi, through the C
ABI: two calls in a row on one stream, the second with fewer batches and
fewer keys than the first, each equal to the allocating entry point's
indices and to the oracle's, bit for bit; the second call leaves the
outputs of the first call's other batches alone."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K
from paper_2502_15539_amd import ptrhash as P

from .mphf_pairs import load

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fleet():
    """Two u64-key MPHFs (32- and 64-bit indices) and one byte-key MPHF."""
    out = []
    for j, (n, bits) in enumerate([(5_000, 32), (120_000, 64)]):
        keys = K.u64_keys(n, seed=900 + j)
        m = O.build_u64(keys)
        out.append(("u64", keys, m, load(m, P.REMAP_CLEF, bits), bits))
    data, off = K.strings(30_000, seed=905)
    m = O.build_bytes(data, off)
    out.append(("bytes", (data, off), m, load(m, P.REMAP_CLEF, 32, key_kind=P.KEY_BYTES), 32))
    return out


def batch(rng, item, size):
    kind, keys, m, g, bits = item
    dt = torch.int64 if bits == 64 else torch.int32
    if kind == "u64":
        q = keys[rng.integers(0, len(keys), size=size)]
        want = O.query_u64(m, q)
        src = torch.from_numpy(q.view(np.int64)).to(DEV)
    else:
        data, off = keys
        pick = rng.integers(0, len(off) - 1, size=size)
        parts = [data[int(off[i]):int(off[i + 1])] for i in pick]
        lens = np.array([len(p) for p in parts], dtype=np.uint64)
        qo = np.zeros(size + 1, dtype=np.uint64)
        qo[1:] = np.cumsum(lens)
        qd = np.zeros(int(qo[-1]) + 64, dtype=np.uint8)
        if size:
            qd[:int(qo[-1])] = np.concatenate(parts)
        want = O.query_bytes(m, qd, qo)
        src = (torch.from_numpy(qd).to(DEV), torch.from_numpy(qo.view(np.int64)).to(DEV))
    return g, src, torch.full((size,), -7, dtype=dt, device=DEV), want


def host(t):
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 else a.view(np.uint32).astype(np.uint64)


def test_noalloc_equals_query_multi_on_two_calls():
    rng = np.random.default_rng(17)
    items = fleet()
    sizes1 = [0, 1, 3, 64, 65, 1000, 70_000] + [int(x) for x in rng.integers(1, 5000, size=33)]
    first = [batch(rng, items[i % 3], s) for i, s in enumerate(sizes1)]
    second = [batch(rng, items[(i + 1) % 3], s) for i, s in enumerate([2, 500, 9_000, 0, 77])]
    assert sum(len(w) for *_, w in second) < sum(len(w) for *_, w in first)

    for name, batches in (("first", first), ("second", second)):
        say(f"[noalloc] {name} call: {len(batches)} batches, {sum(len(w) for *_, w in batches)} keys")
        ref = [torch.full_like(o, -7) for _, _, o, _ in batches]
        P.query_multi([(g, src, r) for (g, src, _, _), r in zip(batches, ref)])
        P.query_multi_noalloc([(g, src, o) for g, src, o, _ in batches])
        torch.cuda.synchronize()
        for (_, _, o, want), r in zip(batches, ref):
            assert torch.equal(o, r)
            assert np.array_equal(host(o), want)
        if name == "first":
            for _, _, o, _ in first:  # the second call must not write these again
                o.fill_(-7)
    torch.cuda.synchronize()
    for _, _, o, _ in first:
        assert bool((o == -7).all())


def test_noalloc_limits():
    items = fleet()
    rng = np.random.default_rng(5)
    g, src, o, want = batch(rng, items[0], 10)
    with pytest.raises(P.PtrHashError) as e:
        P.query_multi_noalloc([(g, src, o)] * 257)
    assert e.value.code == P.E_RANGE
    with pytest.raises(P.PtrHashError) as e:  # two batches writing the same indices
        P.query_multi_noalloc([(g, src, o), (g, src, o)])
    assert e.value.code == P.E_INVAL
    P.query_multi_noalloc([])
    P.query_multi_noalloc([(g, src, o)] + [(g, src[:0], o[:0])] * 255)  # 256 batches, most of them empty
    torch.cuda.synchronize()
    assert np.array_equal(host(o), want)
