"""GPU parity of the many-MPHF launch (row A8): each batch of a persistent
multi-batch launch equals the oracle's query of its own MPHF, for mixes of
sizes, key kinds and output widths, and a captured HIP graph of a plan
replays correctly over rewritten batch tables."""
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


_pool = None


def pool():
    """A dozen oracle-built MPHFs of uneven sizes: u64 (u32 and u64 outputs,
    CacheLineEF / u32 / no remap) and byte keys."""
    global _pool
    if _pool is None:
        rng = np.random.default_rng(5)
        items = []
        for j, n in enumerate([1, 17, 1000, 4096, 10_000, 33_333, 100_000, 250_000]):
            keys = K.u64_keys(n, seed=500 + j)
            m = O.build_u64(keys, seed=j % 3)
            remap = [P.REMAP_CLEF, P.REMAP_U32, P.REMAP_NONE][j % 3]
            bits = 64 if j % 2 else 32
            items.append(("u64", keys, m, load(m, remap, bits), remap, bits))
        for j, n in enumerate([3, 2000, 40_000]):
            data, off = K.strings(n, seed=900 + j)
            m = O.build_bytes(data, off)
            items.append(("bytes", (data, off), m, load(m, P.REMAP_CLEF, 32, key_kind=P.KEY_BYTES), P.REMAP_CLEF, 32))
        _pool = (items, rng)
    return _pool


def make_batch(item, rng, size):
    kind, keys, m, g, remap, bits = item
    if kind == "u64":
        nk = len(keys)
        idx = rng.integers(0, nk, size=size)
        q = keys[idx] if size else keys[:0]
        if size > 4:
            q = q.copy()
            q[::5] = K.nonmember_keys(len(q[::5]), seed=int(rng.integers(1 << 30)))
        want = O.query_u64(m, q, {P.REMAP_CLEF: O.REMAP_CLEF, P.REMAP_U32: O.REMAP_PLAIN,
                                  P.REMAP_NONE: O.REMAP_NONE}[remap])
        qt = torch.from_numpy(q.view(np.int64).copy()).to(DEV)
        dt = torch.int64 if bits == 64 else torch.int32
        return g, qt, torch.full((size,), -1, dtype=dt, device=DEV), want
    data, off = keys
    nk = len(off) - 1
    idx = rng.integers(0, nk, size=size)
    strs = [data[off[i]:off[i + 1]].tobytes() for i in idx]
    buf = np.frombuffer(b"".join(strs) + b"\0" * 64, dtype=np.uint8).copy()
    offs = np.concatenate([[0], np.cumsum([len(x) for x in strs])]).astype(np.uint64)
    want = O.query_bytes(m, buf, offs)
    pair = (torch.from_numpy(buf).to(DEV), torch.from_numpy(offs.view(np.int64)).to(DEV))
    return g, pair, torch.full((size,), -1, dtype=torch.int32, device=DEV), want


def host(out, bits):
    o = out.cpu().numpy()
    return o.view(np.uint64) if out.dtype == torch.int64 else o.view(np.uint32).astype(np.uint64)


def test_multi_matches_oracle_mixed_batches():
    items, rng = pool()
    for rep in range(3):
        sizes = [int(x) for x in np.exp(rng.uniform(0, np.log(70_000), size=40)).astype(int)]
        sizes[0] = 0
        sizes[1] = 1
        batches, wants = [], []
        for s in sizes:
            it = items[int(rng.integers(len(items)))]
            g, q, out, want = make_batch(it, rng, s)
            batches.append((g, q, out))
            wants.append(want)
        say(f"[multi] rep={rep} batches={len(batches)} keys={sum(sizes)}")
        P.query_multi(batches)
        torch.cuda.synchronize()
        for (g, q, out), want in zip(batches, wants):
            assert np.array_equal(host(out, 0), want)


def test_multi_equals_single_calls_many_launches():
    """Back-to-back multi launches (ring reuse) equal single queries."""
    items, rng = pool()
    u64_items = [it for it in items if it[0] == "u64"]
    outs = []
    for launch in range(20):
        batches = []
        for b in range(8):
            it = u64_items[(launch + b) % len(u64_items)]
            g, q, out, want = make_batch(it, rng, int(rng.integers(1, 5000)))
            batches.append((g, q, out, want))
        P.query_multi([(g, q, o) for g, q, o, _ in batches])
        outs.extend(batches)
    torch.cuda.synchronize()
    say(f"[multi] ring reuse: {len(outs)} batches")
    for g, q, out, want in outs:
        assert np.array_equal(host(out, 0), want)


def test_multi_errors():
    items, rng = pool()
    g = items[2][3]
    q = torch.zeros(10, dtype=torch.int64, device=DEV)
    with pytest.raises(P.PtrHashError) as e:
        P.query_multi([(P.Mphf(), q, q)])
    assert e.value.code == P.E_STATE
    with pytest.raises(P.PtrHashError) as e:
        P.query_multi([(g, q, None)])
    assert e.value.code == P.E_INVAL
    o = torch.zeros(10, dtype=torch.int64 if g.index_bytes == 8 else torch.int32, device=DEV)
    plan = P.MultiPlan(2)
    with pytest.raises(P.PtrHashError) as e:
        plan.set([(g, q, o)] * 3)
    assert e.value.code == P.E_RANGE
    # an output of the wrong width or length is refused before any launch
    wrong = torch.zeros(10, dtype=torch.int32 if g.index_bytes == 8 else torch.int64, device=DEV)
    with pytest.raises(ValueError):
        P.query_multi([(g, q, wrong)])
    with pytest.raises(ValueError):
        P.query_multi([(g, q, o[:5])])
    P.query_multi([])  # nothing to do


def test_plan_graph_capture_and_replay():
    """Capture one plan launch; rewrite its batches between replays (with
    eager work and syncs in between) and check every replay."""
    items, rng = pool()
    plan = P.MultiPlan(16)
    stream = torch.cuda.Stream()
    u64_items = [it for it in items if it[0] == "u64"]

    def fresh():
        bs = []
        for b in range(int(rng.integers(1, 16))):
            it = u64_items[int(rng.integers(len(u64_items)))]
            bs.append(make_batch(it, rng, int(rng.integers(0, 20_000))))
        return bs

    first = fresh()
    plan.set([(g, q, o) for g, q, o, _ in first])
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        plan.launch(stream)
    torch.cuda.synchronize()
    for rep in range(6):
        bs = first if rep == 0 else fresh()
        plan.set([(g, q, o) for g, q, o, _ in bs])
        say(f"[graph] replay {rep} batches={len(bs)}")
        graph.replay()
        torch.cuda.synchronize()
        for g, q, out, want in bs:
            assert np.array_equal(host(out, 0), want)
        # eager work between replays
        x = torch.arange(1000, device=DEV).sum()
        assert int(x) == 499500
    plan.close()


@pytest.mark.parametrize("kpl,block,bpc", [(1, 64, 0), (2, 128, 2), (4, 256, 0), (8, 512, 1), (1, 1024, 0),
                                           (8, 64, 8)])
def test_plan_launch_shapes_match_oracle(kpl, block, bpc):
    """Every launch shape the autotuner may pick gives the oracle's indices."""
    items, rng = pool()
    plan = P.MultiPlan(64)
    plan.set_kernel(kpl, block, bpc)
    batches, wants = [], []
    for s in [0, 1, 5, 63, 64, 65, 1000, 4097, 30_000]:
        g, q, out, want = make_batch(items[int(rng.integers(len(items)))], rng, s)
        batches.append((g, q, out))
        wants.append(want)
    plan.set(batches)
    say(f"[multi] shape kpl={kpl} block={block} bpc={bpc}")
    plan.launch()
    torch.cuda.synchronize()
    for (g, q, out), want in zip(batches, wants):
        assert np.array_equal(host(out, 0), want)
    plan.close()


def test_plan_shape_change_needs_new_set_and_default_applies():
    items, rng = pool()
    g, q, out, want = make_batch(items[3], rng, 3000)
    plan = P.MultiPlan(4)
    plan.set([(g, q, out)])
    plan.set_kernel(2, 128, 0)
    with pytest.raises(P.PtrHashError) as e:
        plan.launch()
    assert e.value.code == P.E_STATE
    with pytest.raises(P.PtrHashError) as e:
        plan.set_kernel(3, 128, 0)
    assert e.value.code == P.E_INVAL
    plan.set([(g, q, out)])
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(host(out, 0), want)
    plan.close()
    # the process default reaches query_multi
    P.set_multi_kernel(8, 128, 2)
    try:
        g, q, out, want = make_batch(items[5], rng, 7777)
        P.query_multi([(g, q, out)])
        torch.cuda.synchronize()
        assert np.array_equal(host(out, 0), want)
    finally:
        P.set_multi_kernel(4, 256, 0)


def test_multi_autotuner(tmp_path, monkeypatch):
    from paper_2502_15539_amd import autotune

    monkeypatch.setenv("PTRHASH_TUNE_CACHE", str(tmp_path / "tune.json"))
    items, rng = pool()
    u64_items = [it for it in items if it[0] == "u64"]
    bs = [make_batch(u64_items[i % len(u64_items)], rng, int(rng.integers(1, 20_000))) for i in range(24)]
    batches = [(g, q, o) for g, q, o, _ in bs]
    plan = P.MultiPlan(64)
    cands = autotune.multi_candidates(kpls=(1, 4), blocks=(128, 256), occupancy=(0, 2))
    say(f"[multi] tuning {len(cands)} shapes")
    best, res = autotune.tune_multi(torch, plan, batches, cands=cands, reps=1)
    assert best in res and len(res) == len(cands)
    best2, res2 = autotune.tune_multi(torch, plan, batches, cands=cands, reps=1)
    assert best2 == best and res2 == {}
    for _, _, o, _ in bs:
        o.fill_(-1)
    plan.launch()
    torch.cuda.synchronize()
    for g, q, out, want in bs:
        assert np.array_equal(host(out, 0), want)
    plan.close()


@pytest.mark.parametrize("shape", [(4, 64, 0), (1, 256, 2), (8, 128, 0)])
def test_tile_split_over_dies_and_batch_search(shape):
    """The multi launch gives each of the 8 dies a contiguous range of the
    tiles (split by estimated work, so some ranges may be empty) and finds a
    tile's batch with rounds of 64 parallel reads. Tile
    totals around multiples of 8 and below 8, and batch counts around
    powers of 64 (1, 2, 63, 64, 65, 130, 4096), each batch equal to the
    oracle's query of its MPHF, interleaved MPHFs included (the table groups
    batches by MPHF)."""
    items, _ = pool()
    rng = np.random.default_rng(77)
    plan = P.MultiPlan(4096)
    plan.set_kernel(*shape)
    tile = shape[0] * shape[1]
    cases = [[tile * t] for t in (1, 3, 7, 8, 9, 15, 16, 17)]
    cases += [[1] * c for c in (2, 63, 64, 65, 130)]
    cases += [[int(x) for x in rng.integers(1, 200, size=4096)]]
    for sizes in cases:
        batches = [make_batch(items[(i * 7) % len(items)], rng, s) for i, s in enumerate(sizes)]
        say(f"[multi] shape {shape}: {len(sizes)} batches, {sum(sizes)} keys")
        plan.set([(g, src, out) for g, src, out, _ in batches])
        plan.launch()
        torch.cuda.synchronize()
        for g, src, out, want in batches:
            assert np.array_equal(host(out, 0), want)
    plan.close()


_packed = None


def packed_pool():
    """MPHFs whose slot >= n share is about one half (n = 130,000 just past
    one part of 2^17 slots, so two parts), with each remap kind, and a byte
    key one."""
    global _packed
    if _packed is None:
        items = []
        keys = K.u64_keys(130_000, seed=4242)
        m = O.build_u64(keys)
        frac = float(np.mean(O.query_u64(m, keys, O.REMAP_NONE) >= m.params.n))
        for remap, bits in [(P.REMAP_CLEF, 32), (P.REMAP_U32, 64)]:
            items.append(("u64", keys, m, load(m, remap, bits), remap, bits))
        data, off = K.strings(130_000, seed=4343)
        mb = O.build_bytes(data, off)
        items.append(("bytes", (data, off), mb, load(mb, P.REMAP_CLEF, 32, key_kind=P.KEY_BYTES), P.REMAP_CLEF, 32))
        _packed = (items, frac)
    return _packed


@pytest.mark.parametrize("shape", [(8, 64, 0), (8, 256, 0), (1, 64, 0), (2, 128, 4)])
def test_packed_remap_decode_over_several_rounds(shape):
    """The multi launch decodes a wavefront's remap entries packed onto its
    lanes, 64 per round. With about half of the keys remapped and 8 keys per
    lane, a wavefront has about 256 entries to decode (four rounds, the last
    one partial); with 1 key per lane, about 32 (one partial round). Every
    index equals the oracle's, members and non-members, for both remap
    encodings and byte keys."""
    items, frac = packed_pool()
    say(f"[multi] packed remap: slot >= n share {frac:.3f}, shape {shape}")
    assert frac > 0.3
    rng = np.random.default_rng(91)
    plan = P.MultiPlan(64)
    plan.set_kernel(*shape)
    sizes = [130_000, 1, 63, 64, 65, 4097, 20_000]
    batches = [make_batch(items[i % len(items)], rng, s) for i, s in enumerate(sizes)]
    plan.set([(g, src, out) for g, src, out, _ in batches])
    plan.launch()
    torch.cuda.synchronize()
    for g, src, out, want in batches:
        assert np.array_equal(host(out, 0), want)
    plan.close()
