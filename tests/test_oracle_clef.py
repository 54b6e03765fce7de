"""Pins of the oracle's CacheLineEF (Section 3.4, eq. clef, "Lookup",
"Limitations"): round trips, the byte layout of the fields the paper lists,
select against its definition, and the span limit."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

L = O.lib()
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_space.json")))
RNG = np.random.default_rng(7)


def nondecreasing(n, max_step, start=0):
    steps = RNG.integers(0, max_step + 1, size=n)
    return (start + np.cumsum(steps)).astype(np.uint64)


def select_def(word: int, r: int) -> int:
    """Smallest b such that bits 0..b of word hold r+1 ones."""
    for b in range(128):
        if (word & ((2 << b) - 1)).bit_count() == r + 1:
            return b
    return 128


def test_select128_definition():
    for _ in range(300):
        bits = RNG.choice(128, size=int(RNG.integers(1, 129)), replace=False)
        word = sum(1 << int(b) for b in bits)
        lo, hi = word & ((1 << 64) - 1), word >> 64
        for r in range(len(bits)):
            assert L.orc_select128(lo, hi, r) == select_def(word, r)


@pytest.mark.parametrize("n", [0, 1, 2, 43, 44, 45, 87, 88, 89, 1000, 100_000])
def test_round_trip(n):
    F = nondecreasing(n, 450, start=int(RNG.integers(0, 1 << 39)))
    enc = O.clef_encode(F)
    assert enc.size == -(-n // 44) * 64
    for i in range(n) if n <= 1000 else RNG.integers(0, n, 5000):
        assert O.clef_get(enc, int(i)) == int(F[i])


def test_field_layout():
    """Offset floor(v_0/2^8) as 32 bits, 128 bits with 44 ones at
    i + high(v_i) - high(v_0), then the 44 low bytes (eq. clef)."""
    F = nondecreasing(44 * 3 + 5, 300, start=123456789)
    enc = O.clef_encode(F)
    for c in range(4):
        line = enc[64 * c: 64 * c + 64]
        vals = F[44 * c: 44 * c + 44]
        off = int(vals[0]) >> 8
        assert int.from_bytes(line[0:4].tobytes(), "little") == off
        word = int.from_bytes(line[4:20].tobytes(), "little")
        assert word.bit_count() == len(vals)
        for i, v in enumerate(vals):
            assert (word >> (i + (int(v) >> 8) - off)) & 1
            assert line[20 + i] == int(v) & 0xFF
        assert not line[20 + len(vals):].any()  # partial chunk: zero tail


def test_span_limit():
    """A line spans (128-44)*2^8 = 21504 plus the last partial block of
    256: the 44th value may sit at high part 84 above v_0 but not 85."""
    span = GOLD["clef"]["span"]
    ok = np.zeros(44, dtype=np.uint64)
    ok[-1] = 84 * 256 + 255
    enc = O.clef_encode(ok)
    assert O.clef_get(enc, 43) == 84 * 256 + 255
    assert 84 * 256 == span
    bad = ok.copy()
    bad[-1] = 85 * 256
    with pytest.raises(O.BuildError) as e:
        O.clef_encode(bad)
    assert e.value.code == O.ECLEF_RANGE


def test_offset_limit_40_bits():
    ok = np.array([(1 << 40) - 1], dtype=np.uint64)
    assert O.clef_get(O.clef_encode(ok), 0) == (1 << 40) - 1
    with pytest.raises(O.BuildError):
        O.clef_encode(np.array([1 << 40], dtype=np.uint64))


def test_rejects_decreasing():
    with pytest.raises(O.BuildError):
        O.clef_encode(np.array([5, 4], dtype=np.uint64))


def test_constant_runs():
    """Repeated values (the remap's copied predecessors) encode fine."""
    F = np.repeat(np.array([7, 7, 900, 20000], dtype=np.uint64), [30, 20, 40, 3])
    enc = O.clef_encode(F)
    assert [O.clef_get(enc, i) for i in range(len(F))] == F.tolist()
