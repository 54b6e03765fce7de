"""Randomised agreement of the library's constructions with the oracle.

Hypothesis draws key-set sizes, bucket functions, lambda, alpha-derived
geometry (including explicit slot counts that force evictions and
reseeding) and seeds; the library's host construction must give the
oracle's exact seed, pilots and remap bytes. The GPU variant (marked gpu)
does the same with the device construction and checks the query of every
member and some non-members.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import oracle as O
from paper_2502_15539_amd import keygen as K
from paper_2502_15539_amd import ptrhash as P

from .mphf_pairs import ORACLE_REMAP

cases = st.tuples(
    st.integers(min_value=1, max_value=60_000),       # n
    st.sampled_from([O.GAMMA_CUBIC, O.GAMMA_LINEAR]),  # bucket function
    st.sampled_from([3.0, 3.5, 4.0]),                  # lambda
    st.integers(min_value=0, max_value=2**32),         # MPHF seed
    st.integers(min_value=0, max_value=2**20),         # key-set seed
    st.sampled_from([0, 1, 2]),                        # 0: the rule; 1: tight explicit S; 2: several parts
)


def oracle_case(n, gamma, lam, seed, kseed, shape):
    keys = K.u64_keys(n, seed=kseed)
    if shape == 0:
        p = O.params_for(n, lam=lam, gamma=gamma, seed=seed)
    elif shape == 1:  # one part, S the power of two just above n (load up to 1)
        log2 = max(1, int(n - 1).bit_length())
        B = max(1, int(np.ceil(0.99 * (1 << log2) / lam)))
        p = O.params_explicit(n, 1, log2, B, gamma=gamma, seed=seed)
    else:  # several parts of 2^12 slots at load ~0.9
        log2 = 12
        P_ = max(1, int(np.ceil(n / (0.9 * (1 << log2)))))
        B = max(1, int(np.ceil(0.99 * (1 << log2) / lam)))
        p = O.params_explicit(n, P_, log2, B, gamma=gamma, seed=seed)
    try:
        m = O.build_u64(keys, params=p)
    except O.BuildError:
        return keys, p, None
    return keys, p, m


def lib_from(p, remap=P.REMAP_CLEF):
    q = P.Params()
    q.n, q.num_parts, q.log2_slots, q.buckets_per_part = p.n, p.num_parts, p.log2_slots, p.buckets_per_part
    q.seed, q.gamma, q.remap_kind, q.remap_len = p.seed, p.gamma, remap, p.remap_len
    q.key_kind, q.index_bits, q.hash_bits = P.KEY_U64, 64, 64
    return q


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cases)
def test_host_construction_equals_oracle(case):
    keys, p, m = oracle_case(*case)
    q = lib_from(p)
    if m is None:  # the oracle gave up after 16 seeds: so must the library
        with pytest.raises(P.PtrHashError) as e:
            P.build_u64(keys, params=q, threads=4)
        assert e.value.code == P.E_BUILD
        return
    b = P.build_u64(keys, params=q, threads=4)
    assert b.params.seed == m.params.seed
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)
    assert b.info.evictions == m.stats.evictions


@pytest.mark.gpu
@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(cases)
def test_device_construction_and_query_equal_oracle(case):
    torch = pytest.importorskip("torch")
    keys, p, m = oracle_case(*case)
    q = lib_from(p)
    kt = torch.from_numpy(keys.view(np.int64)).to("cuda")
    print(f"[random] case={case}", flush=True)
    if m is None:
        with pytest.raises(P.PtrHashError) as e:
            P.build_u64_device(kt, params=q, placement="device")
        assert e.value.code == P.E_BUILD
        return
    b = P.build_u64_device(kt, params=q, placement="device")
    assert b.params.seed == m.params.seed
    assert np.array_equal(b.pilots, m.pilots) and np.array_equal(b.remap, m.clef)
    g = P.Mphf.from_built(b)
    probe = np.concatenate([keys, K.nonmember_keys(2000, seed=case[4] + 1)])
    out = g.query(torch.from_numpy(probe.view(np.int64)).to("cuda"))
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, O.query_u64(m, probe, ORACLE_REMAP[P.REMAP_CLEF]))
