"""Test helpers: hand an oracle-built MPHF to the HIP library unchanged.

The oracle's parameters, pilots and remap tables are copied field by field
into the library's load call; nothing computed by the library flows back
into the oracle.
"""
import numpy as np

from oracle import oracle as O
from paper_2502_15539_amd import ptrhash as P

REMAPS = {"clef": P.REMAP_CLEF, "u32": P.REMAP_U32, "none": P.REMAP_NONE}
ORACLE_REMAP = {P.REMAP_CLEF: O.REMAP_CLEF, P.REMAP_U32: O.REMAP_PLAIN, P.REMAP_NONE: O.REMAP_NONE}


def lib_params(m: O.Mphf, remap_kind=P.REMAP_CLEF, index_bits=64, key_kind=P.KEY_U64) -> P.Params:
    o = m.params
    p = P.Params()
    p.n = o.n
    p.num_parts = o.num_parts
    p.log2_slots = o.log2_slots
    p.buckets_per_part = o.buckets_per_part
    p.seed = o.seed
    p.gamma = o.gamma
    p.remap_kind = remap_kind
    p.remap_len = o.remap_len
    p.key_kind = key_kind
    p.index_bits = index_bits
    p.hash_bits = 128 if o.hash_bits == 128 else 64
    if o.reduce_kind == O.REDUCE_MOD:
        p.reduce_kind = P.REDUCE_MOD
        p.slots = o.slots_per_part
        p.log2_slots = 0
    return p


def lib_remap(m: O.Mphf, remap_kind):
    if remap_kind == P.REMAP_CLEF:
        return m.clef
    if remap_kind == P.REMAP_U32:
        return m.F.astype(np.uint32).view(np.uint8)
    return None


def load(m: O.Mphf, remap_kind=P.REMAP_CLEF, index_bits=64, key_kind=P.KEY_U64) -> P.Mphf:
    return P.Mphf().load(lib_params(m, remap_kind, index_bits, key_kind), m.pilots, lib_remap(m, remap_kind))
