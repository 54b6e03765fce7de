"""Pins of the oracle's hash-evict decisions (Section 3.1 "Construction",
Section 3.2 "Hash-evict", Section 4.1.2) on instances built by hand.

The rule the paper gives, and that every construction here must follow:

* buckets are taken largest first (reading: equal sizes by bucket id);
* a bucket takes the smallest pilot in [0, 256) whose slots are free (and,
  reading, pairwise distinct);
* if there is none, it takes the pilot whose colliding buckets weigh least,
  a bucket of size s weighing s^2 (reading: weights add per colliding key;
  ties go to the smallest pilot), never evicting one of the 16 buckets
  placed most recently; the colliding buckets are evicted and queued again;
* a part fails once it has made more than 10*S evictions.

Hashes are chosen first and keys derived from them through C^-1 mod 2^64,
so that every bucket and every pilot-0 slot is placed at will: one part
(P = 1) and the linear bucket function put hash h in bucket hi(B*h), and
for a wanted slot s under pilot p the hash is y xor h_p(p) with y the
smallest integer whose product hi(C*y) ends in the bits of s. Each filler
bucket gets its own pilot-0 slots, so the search places it with pilot 0 and
no eviction, and the part reaches a known state before the bucket under
test. The expected decision is then read off the designed state, and each
instance is chosen so that the plausible mistakes (cost s instead of s^2,
8 or 32 recent buckets instead of 16, the last tying pilot instead of the
first, a wrong scan order, a wrong eviction cap) give another answer; the
oracle's placement records (``build_u64_traced``) show which it made.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K

L = O.lib()
C = 0x517CC1B727220A95
M64 = (1 << 64) - 1
CINV = pow(C, -1, 1 << 64)


def hp(p, seed=0):
    return (C * (p ^ seed)) & M64


def slot_of(h, p, k, seed=0):
    """reduce(h xor h_p(p), 2^k) = hi(C * (h xor h_p)) & (2^k - 1) (eq. slot)."""
    return ((C * (h ^ hp(p, seed))) >> 64) & ((1 << k) - 1)


def bucket_of(h, B):
    """One part, linear bucket function: hi(B * h) (eq. partbucket)."""
    return (B * h) >> 64


def hash_for(rng, b, B, s, p, k):
    """A hash in bucket b whose slot under pilot p is s."""
    for _ in range(1000):
        lo = -(-(b << 64) // B)
        hi_ = -(-((b + 1) << 64) // B) - 1
        target = lo + int(rng.integers(0, hi_ - lo + 1, dtype=np.uint64))
        y0 = target ^ hp(p)
        z = ((C * y0) >> 64) & ~((1 << k) - 1) | s
        if z >= C:
            continue
        y = -(-(z << 64) // C)  # hi(C*y) == z
        if y > M64:
            continue
        h = y ^ hp(p)
        if bucket_of(h, B) == b:
            assert slot_of(h, p, k) == s
            return h
    raise AssertionError("no hash found")


def random_hash_in(rng, b, B):
    lo = -(-(b << 64) // B)
    hi_ = -(-((b + 1) << 64) // B) - 1
    return lo + int(rng.integers(0, hi_ - lo + 1, dtype=np.uint64))


def keys_of(hashes):
    return np.array([(CINV * h) & M64 for h in hashes], dtype=np.uint64)


class Instance:
    """One part of 2^k slots; filler buckets with designed pilot-0 slots,
    then the bucket under test (largest id among the smallest size)."""

    def __init__(self, k, sizes, slots, w_hashes, seed=0):
        self.k = k
        self.S = 1 << k
        self.sizes = sizes            # bucket id -> size (the test bucket last)
        self.slots = slots            # filler bucket id -> its pilot-0 slots
        self.B = len(sizes)
        self.w = self.B - 1
        rng = np.random.default_rng(seed)
        hashes = []
        for b, ss in slots.items():
            assert len(ss) == sizes[b]
            hashes += [hash_for(rng, b, self.B, s, 0, k) for s in ss]
        hashes += list(w_hashes)
        self.hashes = hashes
        self.n = len(hashes)
        assert self.n <= self.S
        taken = [s for ss in slots.values() for s in ss]
        assert len(set(taken)) == len(taken)
        self.owner = {s: b for b, ss in slots.items() for s in ss}
        # fillers in placement order: size descending, then id
        self.order = sorted(slots, key=lambda b: (-sizes[b], b))
        self.rank = {b: len(self.order) - i for i, b in enumerate(self.order)}  # 1 = most recent

    def params(self):
        return O.params_explicit(self.n, 1, self.k, self.B, gamma=O.GAMMA_LINEAR, seed=0)

    def w_slots(self, p):
        return [slot_of(h, p, self.k) for h in self.hashes[-self.sizes[self.w]:]]

    def choice(self, weight=lambda s: s * s, recent=16, last_tie=False):
        """The pilot the rule (or a mutated rule) gives the test bucket."""
        best, best_p = None, None
        free_p = None
        for p in range(256):
            ss = self.w_slots(p)
            if len(set(ss)) != len(ss):
                continue
            owners = [self.owner.get(s) for s in ss]
            if all(o is None for o in owners):
                free_p = p if free_p is None else free_p
                continue
            if any(o is not None and self.rank[o] <= recent for o in owners):
                continue
            cost = sum(weight(self.sizes[o]) for o in owners if o is not None)
            if best is None or cost < best or (last_tie and cost == best):
                best, best_p = cost, p
        return ("free", free_p) if free_p is not None else ("evict", best_p)

    def build(self, **kw):
        return O.build_u64_traced(keys_of(self.hashes), self.params(), **kw)

    def check_fillers(self, recs):
        """The designed state: every filler placed in order with pilot 0."""
        first = recs[:len(self.order)]
        assert [r["bucket"] for r in first] == self.order
        assert all(r["pilot"] == 0 and r["evicted"] == 0 for r in first)
        return recs[len(self.order)]


def layout(rng, S, fixed, n_huge, huge_size, small):
    """Slots for the fillers: `fixed` maps bucket -> slots it must hold; the
    others get random free slots. Bucket ids: huge fillers first, then the
    `small` list of (bucket id, size)."""
    used = {s for ss in fixed.values() for s in ss}
    free_pool = [s for s in rng.permutation(S).tolist() if s not in used]
    slots = {}
    for b in range(n_huge):
        slots[b] = [free_pool.pop() for _ in range(huge_size)]
    for b, size in small:
        ss = list(fixed.get(b, []))
        while len(ss) < size:
            ss.append(free_pool.pop())
        slots[b] = ss
    return slots, free_pool


# ---- (a) the smallest free pilot ----

def test_smallest_pilot_with_distinct_slots():
    """A lone bucket of two keys whose slots coincide under pilots 0, 1 and 2
    takes pilot 3: the first pilot, in increasing order, whose slots are
    pairwise distinct."""
    k, B = 4, 4
    rng = np.random.default_rng(5)
    h1 = random_hash_in(rng, 0, B)
    for _ in range(200_000):
        h2 = random_hash_in(rng, 0, B)
        same = [slot_of(h1, p, k) == slot_of(h2, p, k) for p in range(5)]
        if same[:3] == [True, True, True] and not same[3]:
            break
    else:
        raise AssertionError("no instance")
    p = O.params_explicit(2, 1, k, B, gamma=O.GAMMA_LINEAR)
    rc, pilots, recs, _ = O.build_u64_traced(keys_of([h1, h2]), p)
    assert rc == O.OK
    assert recs[0]["bucket"] == 0 and recs[0]["pilot"] == 3
    assert pilots[0] == 3


def test_smallest_pilot_with_free_slots_and_order():
    """Bucket 1 (two keys) is placed before bucket 0 (one key) although its
    id is larger: it keeps pilot 0, whose slots bucket 0's key also reaches
    under pilots 0..4. Bucket 0 then takes pilot 5, the first whose slot is
    free. Placing by id, or scanning pilots in another order, gives other
    pilots."""
    k, B = 4, 2
    rng = np.random.default_rng(6)
    for _ in range(100_000):
        a, b = random_hash_in(rng, 1, B), random_hash_in(rng, 1, B)
        sa, sb = slot_of(a, 0, k), slot_of(b, 0, k)
        if sa == sb:
            continue
        c = random_hash_in(rng, 0, B)
        cs = [slot_of(c, p, k) for p in range(8)]
        if all(s in (sa, sb) for s in cs[:5]) and cs[5] not in (sa, sb):
            break
    else:
        raise AssertionError("no instance")
    p = O.params_explicit(3, 1, k, B, gamma=O.GAMMA_LINEAR)
    rc, pilots, recs, _ = O.build_u64_traced(keys_of([a, b, c]), p)
    assert rc == O.OK
    assert [(r["bucket"], r["pilot"]) for r in recs] == [(1, 0), (0, 5)]


def replay_smallest_free(keys, p):
    """Placement of an eviction-free build, replayed from the rule: per part,
    buckets by (size desc, id asc), each taking the smallest pilot whose
    slots are free and distinct."""
    P, S, B, seed = p.num_parts, p.slots_per_part, p.buckets_per_part, p.seed
    k = S.bit_length() - 1
    members = {}
    for key in keys:
        h = (C * int(key)) & M64
        part, x = (P * h) >> 64, (P * h) & M64
        x2 = (x * x) >> 64
        x3 = (x2 * x) >> 64
        y = (x2 >> 1) + (x3 >> 1)
        g = y - (y >> 8) + (x >> 8)
        members.setdefault(part * B + ((B * g) >> 64), []).append(h)
    pilots = np.zeros(P * B, dtype=np.uint8)
    for part in range(P):
        taken = set()
        ids = [b for b in range(B) if part * B + b in members]
        for b in sorted(ids, key=lambda b: (-len(members[part * B + b]), b)):
            hs = members[part * B + b]
            for pl in range(256):
                ss = [slot_of(h, pl, k, seed) for h in hs]
                if len(set(ss)) == len(ss) and not taken.intersection(ss):
                    taken.update(ss)
                    pilots[part * B + b] = pl
                    break
            else:
                raise AssertionError("replay found no free pilot")
    return pilots


@pytest.mark.parametrize("n,P,k,lam,seed", [(3000, 1, 13, 3.5, 0), (5000, 3, 12, 3.0, 4), (800, 2, 11, 2.0, 9)])
def test_eviction_free_builds_take_smallest_free_pilots(n, P, k, lam, seed):
    """Builds at load <= 0.61 make no evictions; every pilot is the smallest
    free one given the buckets placed before it."""
    keys = K.u64_keys(n, seed=100 + seed)
    B = math.ceil((1 << k) * n / (P << k) / lam)
    p = O.params_explicit(n, P, k, B, gamma=O.GAMMA_CUBIC, seed=seed)
    m = O.build_u64(keys, params=p, max_attempts=1)
    assert m.stats.evictions == 0
    assert np.array_equal(m.pilots, replay_smallest_free(keys, m.params))


# ---- (b) eviction cost s^2, smallest tying pilot; (c) 16 recent buckets ----

K12 = 12          # S = 4096 slots
HUGE, HUGE_SIZE = 62, 64


def make_eviction_instance(seed, design):
    """Search test-bucket hashes for which `design` returns a layout; see the
    tests for the designs."""
    rng = np.random.default_rng(seed)
    for _ in range(400):
        inst = design(rng)
        if inst is not None:
            return inst
    raise AssertionError("no instance found")


def test_eviction_weight_is_size_squared():
    """The test bucket W (two keys) finds no free pilot. Under pilot p1 one
    key hits bucket A (three keys) and the other a free slot: weight 9
    (s^2) or 3 (s). Under pilot p2 its keys hit buckets Y and Z (two keys
    each): weight 8 (s^2) or 4 (s). Every other pilot hits a 64-key bucket.
    The s^2 rule takes p2 and evicts two buckets; weighing by s would take
    p1."""
    S = 1 << K12
    a_id, y_id, z_id = HUGE, HUGE + 1, HUGE + 2
    spacers = list(range(HUGE + 3, HUGE + 3 + 17))  # 17 later two-key buckets: A, Y, Z not recent
    w_id = spacers[-1] + 1
    sizes = [HUGE_SIZE] * HUGE + [3, 2, 2] + [2] * len(spacers) + [2]

    def design(rng):
        w = [random_hash_in(rng, w_id, w_id + 1), random_hash_in(rng, w_id, w_id + 1)]
        p1, p2 = sorted(rng.choice(256, 2, replace=False).tolist())
        if rng.integers(2):
            p1, p2 = p2, p1
        s1 = [slot_of(w[0], p, K12) for p in (p1, p2)]
        s2 = [slot_of(w[1], p, K12) for p in (p1, p2)]
        need = [s1[0], s2[0], s1[1], s2[1]]
        if len(set(need)) != 4:
            return None
        fixed = {a_id: [s1[0]], y_id: [s1[1]], z_id: [s2[1]]}
        slots, free = layout(rng, S, {**fixed, -1: [s2[0]]}, HUGE, HUGE_SIZE,
                             [(a_id, 3), (y_id, 2), (z_id, 2)] + [(b, 2) for b in spacers])
        free.append(s2[0])
        inst = Instance(K12, sizes, slots, w)
        assert inst.n <= S
        if inst.choice() != ("evict", p2) or inst.choice(weight=lambda s: s) != ("evict", p1):
            return None
        return inst, p1, p2

    inst, p1, p2 = make_eviction_instance(21, design)
    rc, _, recs, _ = inst.build(eviction_factor=0, max_attempts=1)
    w = inst.check_fillers(recs)
    assert w["bucket"] == inst.w
    assert w["pilot"] == p2 and w["evicted"] == 2
    assert p1 != p2


def test_eviction_ties_take_the_smallest_pilot():
    """Two pilots of W each hit one two-key bucket and a free slot (weight 4);
    every other pilot costs more. The smaller of the two is taken."""
    S = 1 << K12
    q_ids = [HUGE, HUGE + 1]
    spacers = list(range(HUGE + 2, HUGE + 2 + 17))
    w_id = spacers[-1] + 1
    sizes = [HUGE_SIZE] * HUGE + [2, 2] + [2] * len(spacers) + [2]

    def design(rng):
        w = [random_hash_in(rng, w_id, w_id + 1), random_hash_in(rng, w_id, w_id + 1)]
        p1, p2 = sorted(rng.choice(256, 2, replace=False).tolist())
        a = [slot_of(w[0], p1, K12), slot_of(w[1], p1, K12), slot_of(w[0], p2, K12), slot_of(w[1], p2, K12)]
        if len(set(a)) != 4:
            return None
        slots, free = layout(rng, S, {q_ids[0]: [a[0]], q_ids[1]: [a[2]], -1: [a[1], a[3]]}, HUGE, HUGE_SIZE,
                             [(q_ids[0], 2), (q_ids[1], 2)] + [(b, 2) for b in spacers])
        inst = Instance(K12, sizes, slots, w)
        if inst.choice() != ("evict", p1) or inst.choice(last_tie=True) != ("evict", p2):
            return None
        return inst, p1, p2

    inst, p1, p2 = make_eviction_instance(22, design)
    rc, _, recs, _ = inst.build(eviction_factor=0, max_attempts=1)
    w = inst.check_fillers(recs)
    assert (w["bucket"], w["pilot"], w["evicted"]) == (inst.w, p1, 1)


def test_sixteen_most_recent_buckets_are_never_evicted():
    """W's cheapest pilots hit two-key buckets placed 12th (R) and 20th (Q)
    most recently, each with a free slot for W's other key (weight 4);
    a third pilot hits a three-key bucket A placed long before (weight 9).
    Pilot p_R < p_Q. Excluding the 16 most recent placements leaves p_Q;
    excluding 8 would take p_R, excluding 32 would take p_A (A is placed
    33rd most recently), and no exclusion would take p_R."""
    S = 1 << K12
    a_id = HUGE
    twos = list(range(HUGE + 1, HUGE + 1 + 32))  # placed in this order; ranks 32 .. 1
    q_id, r_id = twos[12], twos[20]              # ranks 20 and 12
    w_id = twos[-1] + 1
    sizes = [HUGE_SIZE] * HUGE + [3] + [2] * len(twos) + [2]

    def design(rng):
        w = [random_hash_in(rng, w_id, w_id + 1), random_hash_in(rng, w_id, w_id + 1)]
        pr, pq, pa = sorted(rng.choice(256, 3, replace=False).tolist())
        if rng.integers(2):
            pa, pq = pq, pa  # p_A on either side of p_Q
        pr, pq = min(pr, pq), max(pr, pq)
        s = {p: (slot_of(w[0], p, K12), slot_of(w[1], p, K12)) for p in (pr, pq, pa)}
        flat = [x for v in s.values() for x in v]
        if len(set(flat)) != 6:
            return None
        fixed = {r_id: [s[pr][0]], q_id: [s[pq][0]], a_id: [s[pa][0]], -1: [s[pr][1], s[pq][1], s[pa][1]]}
        slots, free = layout(rng, S, fixed, HUGE, HUGE_SIZE, [(a_id, 3)] + [(b, 2) for b in twos])
        inst = Instance(K12, sizes, slots, w)
        if inst.rank[r_id] != 12 or inst.rank[q_id] != 20 or inst.rank[a_id] != 33:
            return None
        want = inst.choice()
        if want != ("evict", pq):
            return None
        if inst.choice(recent=8) != ("evict", pr) or inst.choice(recent=32) != ("evict", pa):
            return None
        if inst.choice(recent=0) != ("evict", pr):
            return None
        return inst, pq

    inst, pq = make_eviction_instance(23, design)
    rc, _, recs, _ = inst.build(eviction_factor=0, max_attempts=1)
    w = inst.check_fillers(recs)
    assert (w["bucket"], w["pilot"], w["evicted"]) == (inst.w, pq, 1)


def test_evicted_buckets_are_queued_again():
    """W evicts Y and Z (two keys each). Both go back on the queue and are
    placed again, Y first (same size, smaller id), each with the smallest
    pilot free in the part as W left it; then the build is complete."""
    S = 1 << K12
    a_id, y_id, z_id = HUGE, HUGE + 1, HUGE + 2
    spacers = list(range(HUGE + 3, HUGE + 3 + 17))
    w_id = spacers[-1] + 1
    sizes = [HUGE_SIZE] * HUGE + [3, 2, 2] + [2] * len(spacers) + [2]

    def smallest_free(hs, owner):
        for p in range(256):
            ss = [slot_of(h, p, K12) for h in hs]
            if len(set(ss)) == len(ss) and all(s not in owner for s in ss):
                return p, ss
        return None, None

    def design(rng):
        w = [random_hash_in(rng, w_id, w_id + 1), random_hash_in(rng, w_id, w_id + 1)]
        p2 = int(rng.integers(256))
        s = [slot_of(w[0], p2, K12), slot_of(w[1], p2, K12)]
        if s[0] == s[1]:
            return None
        slots, free = layout(rng, S, {y_id: [s[0]], z_id: [s[1]]}, HUGE, HUGE_SIZE,
                             [(a_id, 3), (y_id, 2), (z_id, 2)] + [(b, 2) for b in spacers])
        inst = Instance(K12, sizes, slots, w)
        if inst.choice() != ("evict", p2):
            return None
        owner = {x: b for x, b in inst.owner.items() if b not in (y_id, z_id)}
        owner.update({x: w_id for x in s})
        hy = [h for h in inst.hashes if bucket_of(h, inst.B) == y_id]
        hz = [h for h in inst.hashes if bucket_of(h, inst.B) == z_id]
        py, sy = smallest_free(hy, owner)
        if py is None:
            return None
        owner.update({x: y_id for x in sy})
        pz, _ = smallest_free(hz, owner)
        if pz is None:
            return None
        return inst, p2, py, pz

    inst, p2, py, pz = make_eviction_instance(24, design)
    rc, pilots, recs, st = inst.build(eviction_factor=1, max_attempts=1)
    w = inst.check_fillers(recs)
    assert (w["pilot"], w["evicted"]) == (p2, 2)
    i = len(inst.order) + 1
    assert [(r["bucket"], r["pilot"], r["evicted"]) for r in recs[i:]] == [(y_id, py, 0), (z_id, pz, 0)]
    assert rc == O.OK and st.evictions == 2
    assert (pilots[w_id], pilots[y_id], pilots[z_id]) == (p2, py, pz)
    slots = set()
    for h in inst.hashes:
        slots.add(slot_of(h, int(pilots[bucket_of(h, inst.B)]), K12))
    assert len(slots) == inst.n


# ---- the eviction cap (Section 4.1.2: a part fails after 10*S evictions) ----

def test_part_fails_right_after_ten_S_evictions():
    """gamma_1 at lambda = 4.0 (Fig. bucket-fn-plot's failing case) on a part
    of S = 2^11 slots: the search keeps evicting and stops at the first
    placement that takes the part's eviction count past 10*S, not before."""
    k = 11
    S = 1 << k
    n = int(0.99 * S)
    p = O.params_explicit(n, 1, k, math.ceil(0.99 * S / 4.0), gamma=O.GAMMA_LINEAR, seed=0)
    rc, _, recs, st = O.build_u64_traced(K.u64_keys(n, seed=7), p, eviction_factor=10, max_attempts=1,
                                         cap=1 << 22)
    assert rc == O.EBUILD_FAILED
    last = recs[-1]
    assert last["part_evictions"] > 10 * S
    assert last["part_evictions"] - last["evicted"] <= 10 * S
    assert all(r["part_evictions"] <= 10 * S for r in recs[:-1])
    # the same keys and cap with gamma_3 build (Fig. bucket-fn-plot)
    p3 = O.params_explicit(n, 1, k, math.ceil(0.99 * S / 4.0), gamma=O.GAMMA_CUBIC, seed=0)
    rc3, _, recs3, st3 = O.build_u64_traced(K.u64_keys(n, seed=7), p3, eviction_factor=10, max_attempts=1,
                                            cap=1 << 22)
    assert rc3 == O.OK and st3.evictions < S
