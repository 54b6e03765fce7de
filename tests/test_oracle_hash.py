"""Pins of the oracle's hash, part, bucket and slot functions (Section 3.1,
eq. partbucket, eq. slot, Section 3.3) against closed forms, special
values and exact rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K

L = O.lib()
M64 = (1 << 64) - 1
C = 0x517CC1B727220A95
RNG = np.random.default_rng(2024)


def rand_u64(k):
    return [int(x) for x in RNG.integers(0, 1 << 63, size=k, dtype=np.uint64) * 2 + RNG.integers(0, 2, size=k).astype(np.uint64)]


def test_hi_lo_match_exact_product():
    vals = rand_u64(200) + [0, 1, M64, 1 << 63, C]
    for a, b in zip(vals, vals[::-1]):
        prod = a * b  # exact 128-bit product
        assert L.orc_hi(a, b) == prod >> 64
        assert L.orc_lo(a, b) == prod & M64


def test_fxhash_is_invertible():
    """h(k) = C*k mod 2^64 has the inverse C^-1 (C odd)."""
    cinv = pow(C, -1, 1 << 64)
    for k in rand_u64(500) + [0, 1, M64]:
        h = L.orc_hash_u64(k)
        assert (h * cinv) & M64 == k
    assert L.orc_hash_u64(1) == C


@pytest.mark.parametrize("P", [1, 2, 3, 4, 97, 964, 12345])
def test_part_is_fastrange(P):
    """part = floor(P*h/2^64): the first hash of part j is ceil(j*2^64/P)."""
    p = O.params_explicit(1, P, 0, 1)
    for j in range(min(P, 50)):
        first = -((-j << 64) // P)
        assert L.orc_part(p, first) == j
        if first:
            assert L.orc_part(p, first - 1) == j - 1
    assert L.orc_part(p, M64) == P - 1
    assert L.orc_part(p, 0) == 0


def gamma3_exact(x: Fraction) -> Fraction:
    """gamma_3(x) = (255/256)*(x^2+x^3)/2 + x/256 in exact arithmetic."""
    return Fraction(255, 256) * (x * x + x * x * x) / 2 + x / 256


def test_gamma3_fixed_point_matches_real_function():
    xs = rand_u64(400) + [0, 1, 255, 256, 1 << 32, 1 << 63, M64 - 1, M64]
    for x in xs:
        g = L.orc_gamma(O.GAMMA_CUBIC, x)
        exact = gamma3_exact(Fraction(x, 1 << 64)) * (1 << 64)
        assert abs(g - exact) <= 4, (x, g, float(exact))
        assert g <= x


def test_gamma_special_cases():
    assert L.orc_gamma(O.GAMMA_CUBIC, 0) == 0
    for x in rand_u64(50):
        assert L.orc_gamma(O.GAMMA_LINEAR, x) == x
    # slope 1/256 at 0: for tiny x the cubic part vanishes
    assert L.orc_gamma(O.GAMMA_CUBIC, 256 * 1000) == 1000


def test_gamma3_monotone():
    xs = sorted(rand_u64(2000))
    gs = [L.orc_gamma(O.GAMMA_CUBIC, x) for x in xs]
    assert all(a <= b for a, b in zip(gs, gs[1:]))


@pytest.mark.parametrize("gamma", [O.GAMMA_CUBIC, O.GAMMA_LINEAR])
def test_bucket_matches_definition(gamma):
    """bucket = part*B + floor(B * gamma(x)), x = frac(P*h/2^64) (eq. partbucket)."""
    P, B = 97, 296598
    p = O.params_explicit(10**8, P, 20, B, gamma=gamma)
    for h in rand_u64(400):
        part = (P * h) >> 64
        x = Fraction((P * h) & M64, 1 << 64)
        gx = gamma3_exact(x) if gamma == O.GAMMA_CUBIC else x
        want = B * gx
        got = L.orc_bucket(p, h)
        assert part * B <= got < (part + 1) * B
        local = got - part * B
        if abs(want - round(want)) > Fraction(16 * B, 1 << 64):
            assert local == int(want)
        else:
            assert local in (int(want) - 1, int(want))


def test_reduce_special_values():
    """reduce(x, S) = hi(C*x) mod S: hi(C*(2^64-1)) = C-1, hi(C*2^k) = C>>(64-k)."""
    for lg in (1, 4, 18, 20, 30):
        S = 1 << lg
        assert L.orc_reduce(0, S) == 0
        assert L.orc_reduce(M64, S) == (C - 1) & (S - 1)
        for k in (1, 7, 33, 63):
            assert L.orc_reduce(1 << k, S) == (C >> (64 - k)) & (S - 1)
        for x in rand_u64(100):
            assert L.orc_reduce(x, S) < S


def test_pilot_hash_is_fx_of_pilot_xor_seed():
    cinv = pow(C, -1, 1 << 64)
    for seed in (0, 1, 0xDEADBEEF, M64):
        for pl in (0, 1, 17, 255):
            assert (L.orc_hp(seed, pl) * cinv) & M64 == pl ^ seed


def test_slot_layout():
    """slot = part*S + reduce(...), inside the key's own part."""
    p = O.params_explicit(10**6, 4, 18, 74150, seed=3)
    S = p.slots_per_part
    for h in rand_u64(300):
        part = L.orc_part(p, h)
        for pl in (0, 200):
            s = L.orc_slot(p, h, pl)
            assert part * S <= s < (part + 1) * S
            assert s - part * S == L.orc_reduce(h ^ L.orc_hp(3, pl), S)
    # the pilot changes the slot
    moved = sum(L.orc_slot(p, h, 0) != L.orc_slot(p, h, 1) for h in rand_u64(200))
    assert moved > 190


def fmix_inverse(h):
    """Inverse of MurmurHash3's fmix64: undo each invertible step."""
    h ^= h >> 33
    h = (h * pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)) & M64
    h ^= h >> 33
    h = (h * pow(0xFF51AFD7ED558CCD, -1, 1 << 64)) & M64
    h ^= h >> 33
    return h


def test_fmix64_bijective():
    for k in rand_u64(300) + [0, 1, M64]:
        assert fmix_inverse(L.orc_fmix64(k)) == k


def test_bytes_hash_structure():
    """Undoing the final mix and then each absorbed word (inverse mixer)
    leads back to the initial state seed ^ len*C."""
    for s in (b"", b"a", b"abcdefgh", b"0123456789", b"x" * 50):
        seed = 0x1234
        st = fmix_inverse(O.hash_bytes(seed, s))
        words = [int.from_bytes(s[i:i + 8].ljust(8, b"\0"), "little") for i in range(0, len(s), 8)]
        for w in reversed(words):
            st = fmix_inverse(st) ^ w
        assert st == seed ^ ((len(s) * C) & M64)


def test_bytes_hash_sensitivity():
    base = b"the quick brown fox jumps over"
    h0 = O.hash_bytes(0, base)
    for i in range(len(base)):
        mod = bytearray(base)
        mod[i] ^= 1
        assert O.hash_bytes(0, bytes(mod)) != h0
    assert O.hash_bytes(0, b"ab") != O.hash_bytes(0, b"ab\0")
    assert O.hash_bytes(0, base) != O.hash_bytes(1, base)


def test_bytes_hash_collision_free_and_uniform():
    data, off = K.strings(200_000, seed=5)
    hs = np.array([O.hash_bytes(0, data[off[i]:off[i + 1]].tobytes()) for i in range(len(off) - 1)], dtype=np.uint64)
    assert len(np.unique(hs)) == len(hs)
    # chi-square of the top 8 bits over 256 cells
    cnt = np.bincount((hs >> np.uint64(56)).astype(np.int64), minlength=256)
    e = len(hs) / 256
    chi2 = float(((cnt - e) ** 2 / e).sum())
    assert chi2 < 400  # 255 dof: mean 255, sd 22.6
