"""GPU tests of the serving core (row A8): every request's indices are the
same alone and in a mix of concurrent requests (tolerance: exact), equal
the oracle's, and no request is lost or duplicated, also when admission is
squeezed by a tiny per-launch memory budget."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K
from paper_2502_15539_amd import ptrhash as P

from .mphf_pairs import load

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_fleet = None


def fleet():
    global _fleet
    if _fleet is None:
        items = []
        for j, n in enumerate([10, 1000, 12_345, 50_000, 100_000, 300_000]):
            keys = K.u64_keys(n, seed=700 + j)
            m = O.build_u64(keys, seed=j)
            bits = 64 if j % 2 else 32
            items.append((keys, m, load(m, P.REMAP_CLEF, bits), bits))
        _fleet = items
    return _fleet


def requests(rng, count, max_size):
    items = fleet()
    reqs = []
    for _ in range(count):
        keys, m, g, bits = items[int(rng.integers(len(items)))]
        size = int(np.exp(rng.uniform(0, np.log(max_size))))
        q = keys[rng.integers(0, len(keys), size=size)].copy()
        if size > 3:
            q[::3] = K.nonmember_keys(len(q[::3]), seed=int(rng.integers(1 << 30)))
        want = O.query_u64(m, q)
        out = np.zeros(size, dtype=np.uint64 if bits == 64 else np.uint32)
        reqs.append((g, q, out, want))
    return reqs


@pytest.mark.parametrize("zero_copy,shape", [(1, None), (0, None), (1, (1, 128, 2)), (0, (8, 512, 0))])
def test_alone_equals_mix_equals_oracle(zero_copy, shape):
    rng = np.random.default_rng(3)
    reqs = requests(rng, 120, 20_000)
    srv = P.Server(streams=2, max_batches=64, slot_keys=1 << 16, zero_copy=zero_copy, multi_kernel=shape)
    say(f"[serve] alone: {len(reqs)} requests")
    alone = []
    for g, q, out, want in reqs:
        srv.wait(srv.submit(g, q, out))
        alone.append(out.copy())
        out[:] = 0
    say("[serve] mix")
    tickets = [srv.submit(g, q, out) for g, q, out, _ in reqs]
    for t in tickets:
        srv.wait(t)
    for (g, q, out, want), a in zip(reqs, alone):
        assert np.array_equal(a.astype(np.uint64), want)
        assert np.array_equal(out, a)
    st = srv.stats()
    assert st["completed"] == 2 * len(reqs)
    assert st["launches"] < 2 * len(reqs)  # the mix was batched
    srv.close()


@pytest.mark.parametrize("zero_copy", [1, 0])
def test_replay_tiny_budget_no_loss(zero_copy):
    """slot_keys of 3000 and 3 requests per launch force many launches and a
    long queue; every request is delivered once and correctly."""
    rng = np.random.default_rng(4)
    reqs = requests(rng, 400, 3000)
    srv = P.Server(streams=2, max_batches=3, slot_keys=3000, max_queued_keys=1 << 30, zero_copy=zero_copy)
    arrivals = np.cumsum(rng.exponential(20.0, size=len(reqs)))
    say(f"[serve] replay {len(reqs)} requests, tiny budget")
    span = srv.replay([(g, q, out, t) for (g, q, out, _), t in zip(reqs, arrivals)])
    st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["keys"] == sum(len(q) for _, q, _, _ in reqs)
    assert st["launches"] >= len(reqs) / 3
    for g, q, out, want in reqs:
        assert np.array_equal(out.astype(np.uint64), want)
    assert span > 0 and st["p99_us"] >= st["p50_us"] > 0
    srv.close()


def test_server_errors():
    keys, m, g, bits = fleet()[1]
    odt = np.uint64 if bits == 64 else np.uint32
    srv = P.Server(streams=1, max_batches=4, slot_keys=100)
    big = np.zeros(101, dtype=np.uint64)
    out = np.zeros(101, dtype=odt)
    with pytest.raises(P.PtrHashError) as e:
        srv.submit(g, big, out)
    assert e.value.code == P.E_RANGE
    t = srv.submit(g, np.zeros(0, dtype=np.uint64), np.zeros(0, dtype=odt))
    assert srv.wait(t) == 0.0
    with pytest.raises(P.PtrHashError) as e:
        srv.wait(t)  # collected already
    assert e.value.code == P.E_INVAL
    with pytest.raises(P.PtrHashError) as e:
        srv.submit(P.Mphf(), big[:5], out[:5])  # not loaded
    assert e.value.code == P.E_STATE
    srv.close()
    with pytest.raises(P.PtrHashError) as e:
        P.Server(streams=1, max_batches=4, slot_keys=100, multi_kernel=(4, 100, 0))
    assert e.value.code == P.E_INVAL


@pytest.mark.parametrize("zero_copy", [1, 0])
def test_mapped_requests_in_place(zero_copy):
    """Requests whose keys and outputs live in mapped pinned memory are
    served in place, alone or mixed with copied requests; a plain numpy
    buffer is refused for the mapped path."""
    rng = np.random.default_rng(8)
    reqs = requests(rng, 80, 20_000)
    total = sum(len(q) * 8 + len(o) * o.itemsize + 16 for _, q, o, _ in reqs)
    buf = P.HostBuffer(total)
    mapped = []
    off = 0
    for g, q, out, want in reqs:
        k = buf.view(off, len(q), np.uint64)
        k[:] = q
        off += len(q) * 8
        o = buf.view(off, len(out), out.dtype)
        o[:] = 0
        off += (len(out) * out.itemsize + 7) // 8 * 8
        mapped.append((g, k, o, want))
    srv = P.Server(streams=2, max_batches=64, slot_keys=1 << 16, zero_copy=zero_copy)
    say(f"[serve] mapped requests zero_copy={zero_copy}")
    tickets = []
    for i, ((g, k, o, _), (_, q, out, _)) in enumerate(zip(mapped, reqs)):
        tickets.append(srv.submit_mapped(g, k, o) if i % 2 == 0 else srv.submit(g, q, out))
    for t in tickets:
        srv.wait(t)
    for i, ((g, k, o, want), (_, q, out, _)) in enumerate(zip(mapped, reqs)):
        got = o if i % 2 == 0 else out
        assert np.array_equal(got.astype(np.uint64), want)
    # replay with every request mapped
    for _, _, o, _ in mapped:
        o[:] = 0
    span = srv.replay([(g, k, o, 0.0) for g, k, o, _ in mapped], mapped=True)
    assert span > 0
    for g, k, o, want in mapped:
        assert np.array_equal(o.astype(np.uint64), want)
    with pytest.raises(P.PtrHashError) as e:
        g, q, out, _ = reqs[1]
        srv.submit_mapped(g, q, out)
    assert e.value.code == P.E_INVAL
    srv.close()
    buf.close()


@pytest.mark.parametrize("zero_copy", [1, 0])
def test_loaded_replay_overlaps_launches(zero_copy):
    """A saturating Poisson replay (mean gap 2 us, sizes log-uniform up to
    65536 keys) over four launch slots: several slots are busy at once, the
    launches overlap on the device (each launch's start and done events on
    its stream), and every request's indices equal its result alone."""
    rng = np.random.default_rng(12)
    reqs = requests(rng, 600, 65_536)
    srv = P.Server(streams=4, max_batches=16, slot_keys=1 << 17, max_queued_keys=1 << 30, zero_copy=zero_copy)
    say(f"[serve] overlap: {len(reqs)} requests alone, zero_copy={zero_copy}")
    alone = []
    for g, q, out, want in reqs:
        srv.wait(srv.submit(g, q, out))
        assert np.array_equal(out.astype(np.uint64), want)
        alone.append(out.copy())
        out[:] = 0
    srv.reset_stats()
    arrivals = np.cumsum(rng.exponential(2.0, size=len(reqs)))
    say("[serve] overlap: loaded replay")
    srv.replay([(g, q, out, t) for (g, q, out, _), t in zip(reqs, arrivals)])
    st = srv.stats()
    say(f"[serve] overlap: launches {st['launches']} slots busy at most {st['slots_busy_max']}, on the device at "
        f"most {st['overlap_max']} at once, {st['overlap_mean']:.2f} on average")
    for (_, _, out, _), a in zip(reqs, alone):
        assert np.array_equal(out, a)
    assert st["completed"] == len(reqs)
    assert st["slots_busy_max"] >= 2
    assert st["overlap_max"] >= 2 and st["overlap_mean"] > 1.0
    srv.close()
