"""ctypes binding of the PtrHash CPU oracle -- TEST INFRASTRUCTURE ONLY.

Loaded by the tests, the smoke check and the benchmark's CPU-baseline leg;
the HIP library never imports it. ``build()`` compiles the C source with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ptrhash_oracle.c")
LIB = os.path.join(HERE, "libptrhash_oracle.so")

GAMMA_CUBIC, GAMMA_LINEAR = 0, 1
REMAP_CLEF, REMAP_PLAIN, REMAP_NONE = 0, 1, 2
REDUCE_POW2, REDUCE_MOD = 0, 1
OK, EINVAL, EDUPLICATE, EPART_OVERFLOW, EBUILD_FAILED, ECLEF_RANGE, ENOMEM = range(7)

#: Default parameters (Section 4.1.2, "Recommended parameters": Default).
ALPHA, LAMBDA = 0.99, 3.5


def build() -> str:
    """Compile the oracle into a shared library next to its source."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", SRC, "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_uint64),
        ("num_parts", C.c_uint64),
        ("slots_per_part", C.c_uint64),
        ("log2_slots", C.c_uint32),
        ("buckets_per_part", C.c_uint32),
        ("seed", C.c_uint64),
        ("gamma", C.c_int32),
        ("reduce_kind", C.c_int32),
        ("remap_len", C.c_uint64),
        ("hash_bits", C.c_int32),
        ("pad2_", C.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("pad")}


class BuildCfg(C.Structure):
    _fields_ = [("eviction_factor", C.c_uint32), ("max_attempts", C.c_uint32)]


class BuildStats(C.Structure):
    _fields_ = [
        ("attempts", C.c_uint64),
        ("evictions", C.c_uint64),
        ("max_part_evictions", C.c_uint64),
        ("placements", C.c_uint64),
        ("max_bucket_size", C.c_uint64),
    ]


class TraceRec(C.Structure):
    _fields_ = [
        ("part", C.c_uint64),
        ("bucket", C.c_uint32),
        ("pilot", C.c_uint32),
        ("evicted", C.c_uint32),
        ("attempt", C.c_uint32),
        ("part_evictions", C.c_uint64),
    ]


class Trace(C.Structure):
    _fields_ = [("rec", C.POINTER(TraceRec)), ("cap", C.c_uint64), ("len", C.c_uint64), ("total", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        u64, P = C.c_uint64, C.POINTER
        sig = {
            "orc_hi": (u64, [u64, u64]),
            "orc_lo": (u64, [u64, u64]),
            "orc_params_for": (C.c_int, [u64, C.c_double, C.c_double, C.c_int32, C.c_uint32, u64, P(Params)]),
            "orc_params_explicit": (C.c_int, [u64, u64, C.c_uint32, C.c_uint32, C.c_int32, u64, P(Params)]),
            "orc_params_single_mod": (C.c_int, [u64, u64, C.c_uint32, C.c_int32, u64, P(Params)]),
            "orc_params_for_single_mod": (C.c_int, [u64, C.c_double, C.c_double, C.c_int32, u64, P(Params)]),
            "orc_reduce_mod": (u64, [u64, u64]),
            "orc_hash_u64": (u64, [u64]),
            "orc_fmix64": (u64, [u64]),
            "orc_hash_bytes": (u64, [u64, C.c_void_p, u64]),
            "orc_hash_bytes128": (None, [u64, C.c_void_p, u64, P(u64), P(u64)]),
            "orc_slot2": (u64, [P(Params), u64, u64, C.c_uint32]),
            "orc_query_hash2": (u64, [P(Params), C.c_void_p, C.c_int32, C.c_void_p, u64, u64]),
            "orc_part": (u64, [P(Params), u64]),
            "orc_rel": (u64, [P(Params), u64]),
            "orc_gamma": (u64, [C.c_int32, u64]),
            "orc_bucket": (u64, [P(Params), u64]),
            "orc_hp": (u64, [u64, C.c_uint32]),
            "orc_reduce": (u64, [u64, u64]),
            "orc_slot": (u64, [P(Params), u64, C.c_uint32]),
            "orc_build_u64": (C.c_int, [P(Params), C.c_void_p, P(BuildCfg), C.c_void_p, C.c_void_p, P(BuildStats)]),
            "orc_build_u64_traced": (C.c_int, [P(Params), C.c_void_p, P(BuildCfg), C.c_void_p, C.c_void_p,
                                               P(BuildStats), P(Trace)]),
            "orc_build_bytes": (C.c_int, [P(Params), C.c_void_p, C.c_void_p, P(BuildCfg), C.c_void_p, C.c_void_p,
                                          P(BuildStats)]),
            "orc_clef_bytes": (u64, [u64]),
            "orc_clef_encode": (C.c_int, [C.c_void_p, u64, C.c_void_p]),
            "orc_clef_get": (u64, [C.c_void_p, u64]),
            "orc_select128": (C.c_uint32, [u64, u64, C.c_uint32]),
            "orc_query_hash": (u64, [P(Params), C.c_void_p, C.c_int32, C.c_void_p, u64]),
            "orc_query_u64": (C.c_int, [P(Params), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, u64, C.c_void_p]),
            "orc_query_bytes": (C.c_int, [P(Params), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, u64,
                                          C.c_void_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a is not None and a.size else None


def params_for(n, alpha=ALPHA, lam=LAMBDA, gamma=GAMMA_CUBIC, log2_slots=0, seed=0) -> Params:
    p = Params()
    rc = lib().orc_params_for(int(n), float(alpha), float(lam), int(gamma), int(log2_slots), int(seed), C.byref(p))
    if rc:
        raise ValueError(f"orc_params_for(n={n}) -> {rc}")
    return p


def params_explicit(n, P, log2_slots, B, gamma=GAMMA_CUBIC, seed=0) -> Params:
    p = Params()
    rc = lib().orc_params_explicit(int(n), int(P), int(log2_slots), int(B), int(gamma), int(seed), C.byref(p))
    if rc:
        raise ValueError(f"orc_params_explicit -> {rc}")
    return p


def params_single_mod(n, S=None, B=None, alpha=ALPHA, lam=LAMBDA, gamma=GAMMA_CUBIC, seed=0) -> Params:
    """Single part with reduce = x mod S; S and B from the rule unless given."""
    p = Params()
    if S is None:
        rc = lib().orc_params_for_single_mod(int(n), float(alpha), float(lam), int(gamma), int(seed), C.byref(p))
    else:
        rc = lib().orc_params_single_mod(int(n), int(S), int(B), int(gamma), int(seed), C.byref(p))
    if rc:
        raise ValueError(f"single-part mod params(n={n}) -> {rc}")
    return p


class BuildError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


@dataclass
class Mphf:
    """An MPHF built by the oracle: parameters, pilots, plain remap F and
    its CacheLineEF encoding."""

    params: Params
    pilots: np.ndarray  # u8[P*B]
    F: np.ndarray       # u64[P*S - n]
    clef: np.ndarray    # u8[ceil(len/44)*64]
    stats: BuildStats

    @property
    def n(self):
        return self.params.n


def _cfg(eviction_factor, max_attempts):
    cfg = BuildCfg()
    cfg.eviction_factor = eviction_factor
    cfg.max_attempts = max_attempts
    return cfg


def _finish(p, pilots, F, st, rc):
    if rc != OK:
        raise BuildError(rc, f"oracle construction failed with code {rc}")
    clef = np.zeros(lib().orc_clef_bytes(p.remap_len), dtype=np.uint8)
    rc = lib().orc_clef_encode(_ptr(F), p.remap_len, _ptr(clef))
    if rc != OK:
        raise BuildError(rc, f"CacheLineEF encoding failed with code {rc}")
    return Mphf(p, pilots, F, clef, st)


def build_u64(keys: np.ndarray, params: Params | None = None, eviction_factor=10, max_attempts=16, **kw) -> Mphf:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    p = params if params is not None else params_for(len(keys), **kw)
    p = Params.from_buffer_copy(p)
    assert p.n == len(keys)
    pilots = np.zeros(p.num_parts * p.buckets_per_part, dtype=np.uint8)
    F = np.zeros(p.remap_len, dtype=np.uint64)
    st = BuildStats()
    rc = lib().orc_build_u64(C.byref(p), _ptr(keys), C.byref(_cfg(eviction_factor, max_attempts)), _ptr(pilots),
                             _ptr(F), C.byref(st))
    return _finish(p, pilots, F, st, rc)


def build_u64_traced(keys: np.ndarray, params: Params, eviction_factor=10, max_attempts=16, cap=1 << 20):
    """Build like ``build_u64`` and also return the search's placement
    records. Never raises on a failed build: returns ``(rc, pilots, records,
    stats)`` with ``records`` a list of dicts (part, bucket, pilot, evicted,
    attempt, part_evictions) in placement order."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    p = Params.from_buffer_copy(params)
    assert p.n == len(keys)
    pilots = np.zeros(p.num_parts * p.buckets_per_part, dtype=np.uint8)
    F = np.zeros(max(1, p.remap_len), dtype=np.uint64)
    st = BuildStats()
    buf = (TraceRec * cap)()
    tr = Trace(C.cast(buf, C.POINTER(TraceRec)), cap, 0, 0)
    rc = lib().orc_build_u64_traced(C.byref(p), _ptr(keys), C.byref(_cfg(eviction_factor, max_attempts)),
                                    _ptr(pilots), _ptr(F), C.byref(st), C.byref(tr))
    recs = [{f: getattr(buf[i], f) for f, _ in TraceRec._fields_} for i in range(tr.len)]
    return rc, pilots, recs, st


def build_bytes(data: np.ndarray, offsets: np.ndarray, params: Params | None = None, eviction_factor=10,
                max_attempts=16, **kw) -> Mphf:
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(offsets) - 1
    p = params if params is not None else params_for(n, **kw)
    p = Params.from_buffer_copy(p)
    pilots = np.zeros(p.num_parts * p.buckets_per_part, dtype=np.uint8)
    F = np.zeros(p.remap_len, dtype=np.uint64)
    st = BuildStats()
    rc = lib().orc_build_bytes(C.byref(p), _ptr(data), _ptr(offsets), C.byref(_cfg(eviction_factor, max_attempts)),
                               _ptr(pilots), _ptr(F), C.byref(st))
    return _finish(p, pilots, F, st, rc)


def _remap_ptr(m: Mphf, kind):
    if kind == REMAP_CLEF:
        return _ptr(m.clef)
    if kind == REMAP_PLAIN:
        return _ptr(m.F)
    return None


def query_u64(m: Mphf, keys: np.ndarray, remap=REMAP_CLEF) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(len(keys), dtype=np.uint64)
    rc = lib().orc_query_u64(C.byref(m.params), _ptr(m.pilots), remap, _remap_ptr(m, remap), _ptr(keys), len(keys),
                             _ptr(out))
    if rc:
        raise ValueError(f"orc_query_u64 -> {rc}")
    return out


def query_bytes(m: Mphf, data: np.ndarray, offsets: np.ndarray, remap=REMAP_CLEF) -> np.ndarray:
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(offsets) - 1
    out = np.zeros(n, dtype=np.uint64)
    rc = lib().orc_query_bytes(C.byref(m.params), _ptr(m.pilots), remap, _remap_ptr(m, remap), _ptr(data),
                               _ptr(offsets), n, _ptr(out))
    if rc:
        raise ValueError(f"orc_query_bytes -> {rc}")
    return out


def clef_encode(F: np.ndarray) -> np.ndarray:
    F = np.ascontiguousarray(F, dtype=np.uint64)
    out = np.zeros(lib().orc_clef_bytes(len(F)), dtype=np.uint8)
    rc = lib().orc_clef_encode(_ptr(F), len(F), _ptr(out))
    if rc:
        raise BuildError(rc, f"orc_clef_encode -> {rc}")
    return out


def clef_get(clef: np.ndarray, i: int) -> int:
    return lib().orc_clef_get(_ptr(clef), int(i))


def hash_bytes(seed: int, s: bytes) -> int:
    buf = np.frombuffer(s, dtype=np.uint8) if s else np.zeros(1, dtype=np.uint8)
    return lib().orc_hash_bytes(int(seed), _ptr(buf), len(s))
