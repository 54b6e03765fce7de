"""Pins of the oracle's parameter rule and space accounting against the
figures the paper prints (Table 1, Table 2, Section 3.4) and against the
closed form of the rule (Section 3.1, "Parameter values")."""
import json
import math
import os

import pytest

from oracle import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_space.json")))
TOL = 0.006  # the paper prints two decimals


def clef_bits(p):
    return 8 * O.lib().orc_clef_bytes(p.remap_len) / p.n


def pilot_bits(p):
    return 8 * p.num_parts * p.buckets_per_part / p.n


def vec_bits(p):
    return 32 * p.remap_len / p.n


@pytest.mark.parametrize("row", GOLD["table1_n1e9_S2p18"]["rows"], ids=lambda r: r["preset"])
def test_table1_space(row):
    t = GOLD["table1_n1e9_S2p18"]
    p = O.params_for(t["n"], 0.99, row["lambda"], log2_slots=t["log2_slots"])
    assert abs(pilot_bits(p) - row["pilots"]) <= TOL
    assert abs(vec_bits(p) - row["vec_u32"]) <= TOL
    assert abs(clef_bits(p) - row["clef"]) <= TOL


@pytest.mark.parametrize("row", GOLD["table2_n3e8_formula_S"]["rows"], ids=lambda r: r["preset"])
def test_table2_total_space(row):
    t = GOLD["table2_n3e8_formula_S"]
    p = O.params_for(t["n"], 0.99, row["lambda"])
    remap = clef_bits(p) if row["remap"] == "clef" else vec_bits(p)
    assert abs(pilot_bits(p) + remap - row["total"]) <= TOL


def test_clef_bits_per_value():
    c = GOLD["clef"]
    # 10 * 44 values take 10 lines of 64 bytes
    p_bits = 8 * O.lib().orc_clef_bytes(10 * c["values_per_line"]) / (10 * c["values_per_line"])
    assert abs(p_bits - c["bits_per_value"]) < 0.05


@pytest.mark.parametrize("n", [1, 2, 3, 10, 1000, 80000, 217000, 10**6, 10**8, 10**9, 3 * 10**8, 10**12])
def test_rule_closed_form(n):
    alpha, lam = 0.99, 3.5
    p = O.params_for(n, alpha, lam)
    S, P, B = p.slots_per_part, p.num_parts, p.buckets_per_part
    assert S & (S - 1) == 0 and S == 1 << p.log2_slots
    assert P * S >= n and p.remap_len == P * S - n
    assert P == math.ceil(n / (alpha * S))
    assert B == math.ceil(alpha * S / lam)
    K = max(80000.0, 80000.0 * math.log(n / 80000.0))
    if P > 1:
        # smallest power of two with alpha*S >= K (Section 3.1)
        assert alpha * S >= K and alpha * (S // 2) < K
    else:
        # single part: smallest power of two holding n/alpha slots
        assert S >= n / alpha and (S == 1 or S // 2 < n / alpha)


def test_config_integers():
    """The four single-MPHF workloads: parts, slots, buckets, remap length."""
    want = {
        10**6: (4, 18, 74150, 48576),
        10**8: (97, 20, 296598, 1711872),
        10**9: (964, 20, 296598, 10827264),
        3 * 10**8: (289, 20, 296598, 3038464),
    }
    for n, (P, l2, B, R) in want.items():
        p = O.params_for(n)
        assert (p.num_parts, p.log2_slots, p.buckets_per_part, p.remap_len) == (P, l2, B, R)


def test_pilot_space_tends_to_8_over_lambda():
    """8-bit pilots per bucket of expected size lambda/alpha*alpha: 8*P*B/n -> 8/lambda."""
    for lam in (3.0, 3.5, 4.0):
        p = O.params_for(10**12, 0.99, lam)
        assert abs(pilot_bits(p) - 8 / lam) < 0.01


def test_invalid_params():
    with pytest.raises(ValueError):
        O.params_for(0)
    with pytest.raises(ValueError):
        O.params_for(10, alpha=1.5)
    with pytest.raises(ValueError):
        O.params_explicit(100, 1, 4, 5)  # P*S = 16 < n
