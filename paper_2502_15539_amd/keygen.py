"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers; it holds none of the hash-function
arithmetic that it feeds. Every generator is counter based, so any slice of a
stream can be produced on its own (``start``/``count``) and the same slice is
bit-identical no matter how the work is split.

Generators
----------
* ``splitmix64(seed, idx)``: the SplitMix64 generator of Steele, Lea and Flood
  (OOPSLA 2014, "Fast splittable pseudorandom number generators"); output
  number ``idx`` of the stream whose state starts at ``seed`` is the mixer
  applied to ``seed + (idx + 1) * 0x9e3779b97f4a7c15``. The mixer is a
  bijection of 64-bit words, so distinct indices give distinct keys.
* ``u64_keys``: the key set of size n = outputs 0..n-1 of one stream
  (uniform, distinct 64-bit integers, as in the paper's integer-key runs,
  Section 4.1).
* ``permutation``: a seeded bijection of [0, n) built from a 4-round
  balanced Feistel network on ceil(log2 n) bits (rounded up to even) with
  cycle walking; used to query the members in a shuffled order.
* ``query_stream``: member keys in that shuffled order.
* ``strings``: random strings of length uniform in [10, 50] over printable
  ASCII, packed back to back with u64 offsets (the string workload of
  Section 4.2, Table 2), plus at least 64 bytes of zero tail padding.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

#: Seeds used by the benchmark and the tests (keys, query order, MPHF).
KEY_SEED = 1
ORDER_SEED = 2
MPHF_SEED = 0

_CHUNK = 1 << 22


def _threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixer, in place on a uint64 array."""
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """Output ``idx`` (uint64 array) of the SplitMix64 stream seeded ``seed``."""
    with np.errstate(over="ignore"):
        z = np.asarray(idx, dtype=np.uint64) + np.uint64(1)
        z *= GOLDEN
        z += np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        return _mix(z)


def _parallel_fill(out: np.ndarray, fn, start: int) -> np.ndarray:
    """Fill ``out[j] = fn(start + j)`` chunk by chunk on a thread pool."""
    n = out.shape[0]
    if n <= _CHUNK:
        out[:] = fn(np.arange(start, start + n, dtype=np.uint64))
        return out

    def work(lo):
        hi = min(n, lo + _CHUNK)
        out[lo:hi] = fn(np.arange(start + lo, start + hi, dtype=np.uint64))

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(0, n, _CHUNK)))
    return out


def u64_keys(n: int, seed: int = KEY_SEED, start: int = 0, count: int | None = None) -> np.ndarray:
    """Keys ``start .. start+count`` of the n-key set (distinct uniform u64)."""
    count = n - start if count is None else count
    out = np.empty(count, dtype=np.uint64)
    return _parallel_fill(out, lambda i: splitmix64(seed, i), start)


def nonmember_keys(count: int, seed: int = 12345) -> np.ndarray:
    """Uniform u64 keys from an unrelated stream (members only by chance)."""
    return u64_keys(count, seed=seed ^ 0x5DEECE66D)


class Permutation:
    """Seeded bijection of [0, n): 4-round Feistel on 2h bits + cycle walking."""

    ROUNDS = 4

    def __init__(self, n: int, seed: int = ORDER_SEED):
        if n < 1:
            raise ValueError("permutation of an empty range")
        self.n = int(n)
        bits = max(2, int(n - 1).bit_length())
        bits += bits & 1
        self.half = bits // 2
        self.mask = np.uint64((1 << self.half) - 1)
        self.keys = splitmix64(seed, np.arange(self.ROUNDS, dtype=np.uint64))

    def _round(self, x: np.ndarray) -> np.ndarray:
        h = np.uint64(self.half)
        left = x >> h
        right = x & self.mask
        with np.errstate(over="ignore"):
            for r in range(self.ROUNDS):
                f = _mix(right ^ self.keys[r]) & self.mask
                left, right = right, left ^ f
        return (left << h) | right

    def __call__(self, idx: np.ndarray) -> np.ndarray:
        x = self._round(np.asarray(idx, dtype=np.uint64).copy())
        n = np.uint64(self.n)
        bad = x >= n
        while bad.any():
            x[bad] = self._round(x[bad])
            bad = x >= n
        return x


def query_stream(n: int, key_seed: int = KEY_SEED, order_seed: int = ORDER_SEED,
                 start: int = 0, count: int | None = None) -> np.ndarray:
    """Members of the n-key set in a seeded shuffled order (slice of it)."""
    count = n - start if count is None else count
    perm = Permutation(n, order_seed)
    out = np.empty(count, dtype=np.uint64)
    return _parallel_fill(out, lambda i: splitmix64(key_seed, perm(i)), start)


def query_stream_at(n: int, positions: np.ndarray, key_seed: int = KEY_SEED,
                    order_seed: int = ORDER_SEED) -> np.ndarray:
    """Entries at arbitrary ``positions`` of the shuffled member stream."""
    return splitmix64(key_seed, Permutation(n, order_seed)(np.asarray(positions, dtype=np.uint64)))


STR_MIN, STR_MAX = 10, 50
STR_PAD = 64


def string_lengths(count: int, seed: int, start: int = 0) -> np.ndarray:
    return string_lengths_at(np.arange(start, start + count, dtype=np.uint64), seed)


def string_lengths_at(indices: np.ndarray, seed: int) -> np.ndarray:
    r = splitmix64(seed, np.asarray(indices, dtype=np.uint64))
    return (np.uint64(STR_MIN) + r % np.uint64(STR_MAX - STR_MIN + 1)).astype(np.int64)


def strings(count: int, seed: int = KEY_SEED, start: int = 0):
    """Strings ``start .. start+count`` of the random-string stream.

    Returns ``(data, offsets)``: ``data`` is uint8, strings packed back to
    back followed by ``STR_PAD`` zero bytes; ``offsets`` is uint64 of length
    count+1 with string j = data[offsets[j]:offsets[j+1]]. String i's bytes
    depend only on (seed, i), so slices of the stream agree with the whole.
    """
    lens = string_lengths(count, seed, start)
    offsets = np.zeros(count + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    data = np.zeros(total + STR_PAD, dtype=np.uint8)
    # byte j of string i comes from output (i * 64 + j) of a second stream:
    # 64 > STR_MAX, so every byte has its own counter.
    bseed = seed ^ 0x2545F4914F6CDD1D
    step = 1 << 20

    def work(lo):
        hi = min(count, lo + step)
        l = lens[lo:hi]
        o = offsets[lo:hi].astype(np.int64)
        tot = int(l.sum())
        owner = np.repeat(np.arange(lo, hi, dtype=np.int64), l)
        pos_in = np.arange(tot, dtype=np.int64) - np.repeat(o - o[0], l)
        ctr = (owner + start).astype(np.uint64) * np.uint64(64) + pos_in.astype(np.uint64)
        r = splitmix64(bseed, ctr)
        data[o[0]:o[0] + tot] = (np.uint64(0x20) + (r & np.uint64(0xFF)) % np.uint64(95)).astype(np.uint8)

    chunks = range(0, count, step)
    if count > step:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, chunks))
    else:
        for lo in chunks:
            work(lo)
    return data, offsets


def strings_at(indices: np.ndarray, seed: int = KEY_SEED):
    """Strings with arbitrary indices of the random-string stream, packed in
    the given order (same layout as ``strings``)."""
    idx = np.asarray(indices, dtype=np.uint64)
    lens = string_lengths_at(idx, seed)
    offsets = np.zeros(len(idx) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    owner = np.repeat(idx, lens)
    pos_in = np.arange(total, dtype=np.int64) - np.repeat(offsets[:-1].astype(np.int64), lens)
    r = splitmix64(seed ^ 0x2545F4914F6CDD1D, owner * np.uint64(64) + pos_in.astype(np.uint64))
    data = np.zeros(total + STR_PAD, dtype=np.uint8)
    data[:total] = (np.uint64(0x20) + (r & np.uint64(0xFF)) % np.uint64(95)).astype(np.uint8)
    return data, offsets


def string_query_stream_at(count: int, positions: np.ndarray, seed: int = KEY_SEED,
                           order_seed: int = ORDER_SEED):
    """Entries at arbitrary ``positions`` of the shuffled string stream."""
    return strings_at(Permutation(count, order_seed)(np.asarray(positions, dtype=np.uint64)), seed)


def string_query_stream(count: int, seed: int = KEY_SEED, order_seed: int = ORDER_SEED):
    """All ``count`` strings of the set, repacked in a seeded shuffled order."""
    data, offsets = strings(count, seed)
    perm = Permutation(count, order_seed)(np.arange(count, dtype=np.uint64)).astype(np.int64)
    lens = (offsets[1:] - offsets[:-1]).astype(np.int64)
    qlens = lens[perm]
    qoff = np.zeros(count + 1, dtype=np.uint64)
    np.cumsum(qlens, out=qoff[1:])
    src = np.repeat(offsets[:-1].astype(np.int64)[perm], qlens)
    within = np.arange(int(qoff[-1]), dtype=np.int64) - np.repeat(qoff[:-1].astype(np.int64), qlens)
    qdata = np.zeros(int(qoff[-1]) + STR_PAD, dtype=np.uint8)
    qdata[: int(qoff[-1])] = data[src + within]
    return qdata, qoff
