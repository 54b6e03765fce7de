"""Python binding of the C ABI in include/ptrhash.h (argument marshalling only).

Every query runs in the HIP kernels of ``libptrhash_hip.so``; there is no
fallback. If the library is missing, :func:`lib` raises. Torch is used only
to hold device memory and to name the stream a launch goes on.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptrhash_hip.so")

OK, E_INVAL, E_STATE, E_RANGE, E_NOMEM, E_HIP, E_DUPLICATE, E_BUILD, E_REMAP_RANGE = range(9)
GAMMA_CUBIC, GAMMA_LINEAR = 0, 1
REMAP_CLEF, REMAP_U32, REMAP_NONE = 0, 1, 2
KEY_U64, KEY_BYTES = 0, 1
PRESET_DEFAULT, PRESET_FAST, PRESET_COMPACT = 0, 1, 2
PRESET_SINGLE_MOD = 0x100
REDUCE_POW2, REDUCE_MOD = 0, 1
KERNEL_PLAIN, KERNEL_PIPELINED = 0, 1


class PtrHashError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_uint64),
        ("num_parts", C.c_uint64),
        ("log2_slots", C.c_uint32),
        ("buckets_per_part", C.c_uint32),
        ("seed", C.c_uint64),
        ("gamma", C.c_uint32),
        ("remap_kind", C.c_uint32),
        ("remap_len", C.c_uint64),
        ("key_kind", C.c_uint32),
        ("index_bits", C.c_uint32),
        ("reduce_kind", C.c_uint32),
        ("hash_bits", C.c_uint32),
        ("slots", C.c_uint64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}

    @property
    def slots_per_part(self) -> int:
        return self.slots if self.reduce_kind == REDUCE_MOD else 1 << self.log2_slots

    def copy(self) -> "Params":
        return Params.from_buffer_copy(self)


class QueryDesc(C.Structure):
    _fields_ = [
        ("handle", C.c_void_p),
        ("keys", C.c_void_p),
        ("data", C.c_void_p),
        ("data_len", C.c_uint64),
        ("offsets", C.c_void_p),
        ("n_q", C.c_uint64),
        ("out", C.c_void_p),
    ]


class ServerConfig(C.Structure):
    _fields_ = [("streams", C.c_int), ("max_batches", C.c_int), ("slot_keys", C.c_uint64),
                ("max_queued_keys", C.c_uint64), ("copy_threads", C.c_int), ("zero_copy", C.c_int),
                ("keys_per_lane", C.c_int), ("block", C.c_int), ("blocks_per_cu", C.c_int)]


class ServerMetrics(C.Structure):
    _fields_ = [("completed", C.c_uint64), ("launches", C.c_uint64), ("keys", C.c_uint64), ("queued", C.c_uint64),
                ("p50_us", C.c_double), ("p99_us", C.c_double), ("max_us", C.c_double),
                ("wait_p50_us", C.c_double), ("wait_p99_us", C.c_double), ("slots_busy_max", C.c_uint64),
                ("overlap_max", C.c_uint64), ("overlap_mean", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerRequest(C.Structure):
    _fields_ = [("handle", C.c_void_p), ("keys", C.c_void_p), ("n_q", C.c_uint64), ("out", C.c_void_p),
                ("arrival_us", C.c_double), ("mapped", C.c_uint32), ("pad_", C.c_uint32)]


class BuildInfo(C.Structure):
    _fields_ = [
        ("attempts", C.c_uint64),
        ("evictions", C.c_uint64),
        ("max_part_evictions", C.c_uint64),
        ("max_bucket_size", C.c_uint64),
    ]


_lib = None
_SIGS = {
    "ptrhash_create": (C.c_int, [C.POINTER(C.c_void_p)]),
    "ptrhash_destroy": (C.c_int, [C.c_void_p]),
    "ptrhash_params_default": (C.c_int, [C.c_uint64, C.c_int, C.c_uint32, C.c_uint32, C.c_uint64, C.POINTER(Params)]),
    "ptrhash_remap_bytes": (C.c_uint64, [C.POINTER(Params)]),
    "ptrhash_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Params)]),
    "ptrhash_get_params": (C.c_int, [C.c_void_p, C.POINTER(Params)]),
    "ptrhash_query": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "ptrhash_query_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p,
                                      C.c_void_p]),
    "ptrhash_set_kernel": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "ptrhash_last_error": (C.c_char_p, []),
    "ptrhash_set_occupancy": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "ptrhash_build_u64": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_int,
                                    C.POINTER(BuildInfo)]),
    "ptrhash_build_u64_device": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Params), C.c_void_p, C.c_void_p,
                                           C.c_int, C.POINTER(BuildInfo), C.c_void_p]),
    "ptrhash_build_u64_gpu": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Params), C.c_void_p, C.c_void_p,
                                        C.POINTER(BuildInfo), C.c_void_p]),
    "ptrhash_build_bytes_gpu": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.POINTER(Params), C.c_void_p,
                                          C.c_void_p, C.POINTER(BuildInfo), C.c_void_p]),
    "ptrhash_build_bytes": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.POINTER(Params), C.c_void_p,
                                      C.c_void_p,
                                      C.c_int, C.POINTER(BuildInfo)]),
    "ptrhash_bench_gather": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p, C.c_int, C.c_int,
                                       C.c_int, C.c_void_p]),
    "ptrhash_server_submit_mapped": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                               C.POINTER(C.c_uint64)]),
    "ptrhash_host_alloc": (C.c_int, [C.c_uint64, C.POINTER(C.c_void_p)]),
    "ptrhash_host_free": (C.c_int, [C.c_void_p]),
    "ptrhash_multi_plan_set_kernel": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "ptrhash_set_multi_kernel": (C.c_int, [C.c_int, C.c_int, C.c_int]),
    "ptrhash_bench_gather_pair": (C.c_int, [C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint32,
                                            C.c_uint32, C.c_void_p]),
    "ptrhash_bench_gather_pure": (C.c_int, [C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint32,
                                            C.c_void_p]),
    "ptrhash_bench_copy": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "ptrhash_bench_gather_buckets": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_int, C.c_int,
                                               C.c_int, C.c_void_p]),
    "ptrhash_bench_gather_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p,
                                             C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "ptrhash_bench_scatter": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "ptrhash_multi_plan_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "ptrhash_multi_plan_destroy": (C.c_int, [C.c_void_p]),
    "ptrhash_multi_plan_set": (C.c_int, [C.c_void_p, C.POINTER(QueryDesc), C.c_int]),
    "ptrhash_multi_plan_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ptrhash_query_multi": (C.c_int, [C.POINTER(QueryDesc), C.c_int, C.c_void_p]),
    "ptrhash_multi_max": (C.c_int, []),
    "ptrhash_query_multi_noalloc": (C.c_int, [C.POINTER(QueryDesc), C.c_int, C.c_void_p]),
    "ptrhash_server_default_config": (C.c_int, [C.POINTER(ServerConfig)]),
    "ptrhash_server_create": (C.c_int, [C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]),
    "ptrhash_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                        C.POINTER(C.c_uint64)]),
    "ptrhash_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_double)]),
    "ptrhash_server_replay": (C.c_int, [C.c_void_p, C.POINTER(ServerRequest), C.c_uint64, C.POINTER(C.c_double)]),
    "ptrhash_server_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerMetrics)]),
    "ptrhash_server_reset_stats": (C.c_int, [C.c_void_p]),
    "ptrhash_server_destroy": (C.c_int, [C.c_void_p]),
    "ptrhash_gen_string_lengths": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, C.c_uint64, C.c_uint64,
                                             C.c_void_p, C.c_void_p]),
    "ptrhash_gen_string_bytes": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, C.c_uint64, C.c_uint64,
                                           C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptrhash_gen_u64_keys": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p]),
    "ptrhash_gen_query_stream": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p,
                                           C.c_void_p]),
}


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_15539_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != OK:
        raise PtrHashError(rc, where, lib().ptrhash_last_error().decode())


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None and a.size else None


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _device_tensor(t, name: str, itemsize: int, count: int):
    """A contiguous device tensor with at least count elements of itemsize
    bytes: the kernels write and read exactly that much, so a smaller or
    wider buffer is refused here rather than overrun on the device."""
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.element_size() != itemsize:
        raise ValueError(f"{name} must have {itemsize}-byte elements, not {t.element_size()}")
    if t.numel() < count:
        raise ValueError(f"{name} holds {t.numel()} elements, {count} are needed")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    """A HIP stream handle: explicit int, a torch stream, or torch's current one."""
    if isinstance(stream, int):
        return C.c_void_p(stream)
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def params_default(n: int, preset: int = PRESET_DEFAULT, key_kind: int = KEY_U64, index_bits: int = 0,
                   seed: int = 0) -> Params:
    p = Params()
    _check(lib().ptrhash_params_default(int(n), int(preset), int(key_kind), int(index_bits), int(seed), C.byref(p)),
           "ptrhash_params_default")
    return p


def remap_bytes(p: Params) -> int:
    return int(lib().ptrhash_remap_bytes(C.byref(p)))


@dataclass
class Built:
    """Host arrays of a built MPHF, ready for :meth:`Mphf.load`."""

    params: Params
    pilots: np.ndarray
    remap: np.ndarray
    info: BuildInfo
    placement: str = "host"  # where the pilot search ran

    @property
    def bits_per_key(self) -> float:
        return 8.0 * (self.pilots.size + self.remap.size) / self.params.n


def build_u64(keys: np.ndarray, params: Params | None = None, threads: int = 0, **kw) -> Built:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    p = (params if params is not None else params_default(len(keys), **kw)).copy()
    pilots = np.zeros(p.num_parts * p.buckets_per_part, dtype=np.uint8)
    remap = np.zeros(remap_bytes(p), dtype=np.uint8)
    info = BuildInfo()
    _check(lib().ptrhash_build_u64(_np_ptr(keys), len(keys), C.byref(p), _np_ptr(pilots), _np_ptr(remap),
                                   int(threads), C.byref(info)), "ptrhash_build_u64")
    return Built(p, pilots, remap, info)


def build_u64_device(keys, params: Params | None = None, threads: int = 0, stream=None, placement: str = "auto",
                     **kw) -> Built:
    """Build from u64 keys in device memory (a cuda int64/uint64 tensor).

    placement: "device" runs the pilot search on the GPU too
    (ptrhash_build_u64_gpu); "host" hashes and sorts on the GPU and searches
    on host threads (ptrhash_build_u64_device); "auto" takes the device
    search unless the parameters are outside its limits (E_RANGE). Every
    choice gives the same MPHF; ``Built.placement`` says which ran."""
    if placement not in ("auto", "device", "host"):
        raise ValueError("placement must be 'auto', 'device' or 'host'")
    n = keys.numel()
    p0 = (params if params is not None else params_default(n, **kw)).copy()
    pilots = np.zeros(p0.num_parts * p0.buckets_per_part, dtype=np.uint8)
    remap = np.zeros(remap_bytes(p0), dtype=np.uint8)
    info = BuildInfo()
    if placement != "host":
        p = p0.copy()
        rc = lib().ptrhash_build_u64_gpu(_device_tensor(keys, "keys", 8, n), n, C.byref(p), _np_ptr(pilots), _np_ptr(remap),
                                         C.byref(info), _stream(stream))
        if rc == 0:
            return Built(p, pilots, remap, info, "device")
        if placement == "device" or rc != E_RANGE:
            _check(rc, "ptrhash_build_u64_gpu")
    p = p0.copy()
    _check(lib().ptrhash_build_u64_device(_device_tensor(keys, "keys", 8, n), n, C.byref(p), _np_ptr(pilots), _np_ptr(remap),
                                          int(threads), C.byref(info), _stream(stream)), "ptrhash_build_u64_device")
    return Built(p, pilots, remap, info, "host")


def build_bytes(data: np.ndarray, offsets: np.ndarray, params: Params | None = None, threads: int = 0,
                **kw) -> Built:
    data = np.ascontiguousarray(data, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(offsets) - 1
    p = (params if params is not None else params_default(n, key_kind=KEY_BYTES, **kw)).copy()
    pilots = np.zeros(p.num_parts * p.buckets_per_part, dtype=np.uint8)
    remap = np.zeros(remap_bytes(p), dtype=np.uint8)
    info = BuildInfo()
    _check(lib().ptrhash_build_bytes(_np_ptr(data), data.size, _np_ptr(offsets), n, C.byref(p), _np_ptr(pilots),
                                     _np_ptr(remap), int(threads), C.byref(info)), "ptrhash_build_bytes")
    return Built(p, pilots, remap, info)


def build_bytes_device(data, offsets, params: Params | None = None, threads: int = 0, stream=None,
                       placement: str = "auto", **kw) -> Built:
    """Build from byte strings in device memory (a cuda uint8 tensor, 8-byte
    aligned with 64 readable bytes after the last string, and an int64/uint64
    offsets tensor of n + 1 entries). placement as in build_u64_device;
    "host" copies the strings to the host and runs ptrhash_build_bytes."""
    if placement not in ("auto", "device", "host"):
        raise ValueError("placement must be 'auto', 'device' or 'host'")
    n = offsets.numel() - 1
    p0 = (params if params is not None else params_default(n, key_kind=KEY_BYTES, **kw)).copy()
    pilots = np.zeros(p0.num_parts * p0.buckets_per_part, dtype=np.uint8)
    remap = np.zeros(remap_bytes(p0), dtype=np.uint8)
    info = BuildInfo()
    if placement != "host":
        p = p0.copy()
        rc = lib().ptrhash_build_bytes_gpu(_device_tensor(data, "data", 1, 0), data.numel(),
                                           _device_tensor(offsets, "offsets", 8, n + 1), n, C.byref(p), _np_ptr(pilots),
                                           _np_ptr(remap), C.byref(info), _stream(stream))
        if rc == 0:
            return Built(p, pilots, remap, info, "device")
        if placement == "device" or rc != E_RANGE:
            _check(rc, "ptrhash_build_bytes_gpu")
    b = build_bytes(data.cpu().numpy(), offsets.cpu().numpy().view(np.uint64), params=p0, threads=threads)
    b.placement = "host"
    return b


class Mphf:
    """A device-resident MPHF behind one library handle."""

    def __init__(self):
        h = C.c_void_p()
        _check(lib().ptrhash_create(C.byref(h)), "ptrhash_create")
        self._h = h
        self.index_bytes = 0  # set by load

    def close(self):
        if self._h:
            lib().ptrhash_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def load(self, params: Params, pilots: np.ndarray, remap: np.ndarray | None) -> "Mphf":
        pilots = np.ascontiguousarray(pilots, dtype=np.uint8)
        remap = None if remap is None else np.ascontiguousarray(remap, dtype=np.uint8)
        _check(lib().ptrhash_load(self._h, _np_ptr(pilots), _np_ptr(remap), C.byref(params)), "ptrhash_load")
        self.index_bytes = params.index_bits // 8  # output element size, checked on every query
        return self

    @classmethod
    def from_built(cls, b: Built) -> "Mphf":
        return cls().load(b.params, b.pilots, b.remap)

    @property
    def params(self) -> Params:
        p = Params()
        _check(lib().ptrhash_get_params(self._h, C.byref(p)), "ptrhash_get_params")
        return p

    def set_kernel(self, kernel: int, keys_per_lane: int = 4, block: int = 256):
        _check(lib().ptrhash_set_kernel(self._h, int(kernel), int(keys_per_lane), int(block)), "ptrhash_set_kernel")

    def set_occupancy(self, blocks_per_cu: int = 0) -> int:
        """Cap resident workgroups per CU (0 = none); returns the effective cap."""
        eff = C.c_int()
        _check(lib().ptrhash_set_occupancy(self._h, int(blocks_per_cu), C.byref(eff)), "ptrhash_set_occupancy")
        return eff.value

    def query_into(self, keys, out, stream=None):
        """keys: cuda uint64 tensor; out: cuda tensor of index_bits width."""
        n = keys.numel()
        ob = self.index_bytes
        _check(lib().ptrhash_query(self._h, _device_tensor(keys, "keys", 8, n), n, _device_tensor(out, "out", ob, n),
                                   _stream(stream)), "ptrhash_query")
        return out

    def query(self, keys, stream=None):
        import torch

        dt = torch.int64 if self.params.index_bits == 64 else torch.int32
        out = torch.empty(keys.numel(), dtype=dt, device=keys.device)
        return self.query_into(keys, out, stream)

    def query_bytes_into(self, data, offsets, out, stream=None, check_end=True):
        """data: cuda uint8 tensor of packed strings (8-byte aligned, 64 readable
        bytes after the last string); offsets: n + 1 u64 offsets; out: n
        indices of index_bits width. check_end reads offsets[n] back (one
        synchronising 8-byte copy) and refuses a data tensor shorter than
        offsets[n] + 64 bytes; the kernel itself never reads past data and
        gives keys with bad offsets an index of all ones."""
        n = offsets.numel() - 1
        if n < 0:
            raise ValueError("offsets needs at least one entry")
        ob = self.index_bytes
        dp = _device_tensor(data, "data", 1, 0)
        op = _device_tensor(offsets, "offsets", 8, n + 1)
        if check_end and n > 0:
            end = int(offsets[n].item())
            if end < 0 or end + 64 > data.numel():
                raise ValueError(f"data holds {data.numel()} bytes; the strings end at {end} and 64 bytes of "
                                 "padding must follow")
        _check(lib().ptrhash_query_bytes(self._h, dp, data.numel(), op, n, _device_tensor(out, "out", ob, n),
                                         _stream(stream)), "ptrhash_query_bytes")
        return out

    def query_bytes(self, data, offsets, stream=None):
        import torch

        dt = torch.int64 if self.params.index_bits == 64 else torch.int32
        out = torch.empty(offsets.numel() - 1, dtype=dt, device=offsets.device)
        return self.query_bytes_into(data, offsets, out, stream)


def bench_gather(keys, table, out, keys_per_lane=4, block=256, blocks_per_cu=0, stream=None):
    n = keys.numel()
    _check(lib().ptrhash_bench_gather(_device_tensor(keys, "keys", 8, n), n, _device_tensor(table, "table", 1, 1),
                                      table.numel(), _device_tensor(out, "out", 8, n), int(keys_per_lane), int(block),
                                      int(blocks_per_cu), _stream(stream)), "ptrhash_bench_gather")


def bench_gather_pure(n, table, sink, stream=None):
    """sink: int32 cuda tensor, its length (a multiple of 256) = lanes."""
    _check(lib().ptrhash_bench_gather_pure(int(n), _device_tensor(table, "table", 1, 1), table.numel(),
                                           _device_tensor(sink, "sink", 4, 0), sink.numel(), _stream(stream)),
           "ptrhash_bench_gather_pure")


def bench_gather_pair(n, table, sink, xor_dist, stream=None):
    """Pure gather plus a second byte at o ^ xor_dist of each random offset o."""
    _check(lib().ptrhash_bench_gather_pair(int(n), _device_tensor(table, "table", 1, 1), table.numel(),
                                           _device_tensor(sink, "sink", 4, 0), sink.numel(), int(xor_dist),
                                           _stream(stream)), "ptrhash_bench_gather_pair")


def bench_gather_buckets(mphf, keys, out, keys_per_lane=4, block=256, blocks_per_cu=0, stream=None):
    """Like-for-like gather: each key's own pilot byte of a loaded u64-key MPHF."""
    n = keys.numel()
    _check(lib().ptrhash_bench_gather_buckets(mphf.handle, _device_tensor(keys, "keys", 8, n), n,
                                              _device_tensor(out, "out", 8, n), int(keys_per_lane), int(block),
                                              int(blocks_per_cu), _stream(stream)), "ptrhash_bench_gather_buckets")


def bench_gather_bytes(mphf, data, offsets, out, keys_per_lane=1, block=256, blocks_per_cu=0, stream=None):
    """String-stream gather: the memory pattern of a byte-key query (u32 out)."""
    n = offsets.numel() - 1
    _check(lib().ptrhash_bench_gather_bytes(mphf.handle, _device_tensor(data, "data", 1, 0), data.numel(),
                                            _device_tensor(offsets, "offsets", 8, n + 1), n,
                                            _device_tensor(out, "out", 4, n), int(keys_per_lane), int(block),
                                            int(blocks_per_cu), _stream(stream)), "ptrhash_bench_gather_bytes")


def bench_scatter(src, log2_n, out, stream=None):
    """out[(i * A) mod 2^log2_n] = src[i]: the cost of an un-permute pass."""
    n = 1 << int(log2_n)
    _check(lib().ptrhash_bench_scatter(_device_tensor(src, "src", 8, n), int(log2_n), _device_tensor(out, "out", 8, n),
                                       _stream(stream)), "ptrhash_bench_scatter")


def bench_copy(keys, out, keys_per_lane=4, block=256, stream=None):
    n = keys.numel()
    _check(lib().ptrhash_bench_copy(_device_tensor(keys, "keys", 8, n), n, _device_tensor(out, "out", 8, n),
                                    int(keys_per_lane), int(block), _stream(stream)), "ptrhash_bench_copy")


def gen_u64_keys(out, seed, start=0, stream=None):
    """Fill the cuda uint64 tensor ``out`` with keys start.. of the key set."""
    _check(lib().ptrhash_gen_u64_keys(int(seed), int(start), out.numel(), _device_tensor(out, "out", 8, 0),
                                      _stream(stream)), "ptrhash_gen_u64_keys")
    return out


def gen_query_stream(out, n, key_seed, order_seed, start=0, stream=None):
    """Fill ``out`` with entries start.. of the shuffled member stream of the n-key set."""
    _check(lib().ptrhash_gen_query_stream(int(n), int(key_seed), int(order_seed), int(start), out.numel(),
                                          _device_tensor(out, "out", 8, 0), _stream(stream)),
           "ptrhash_gen_query_stream")
    return out


def make_descs(batches):
    """batches: list of (Mphf, keys_or_(data, offsets), out) with cuda tensors."""
    arr = (QueryDesc * max(1, len(batches)))()
    for i, (m, keys, out) in enumerate(batches):
        d = arr[i]
        d.handle = m.handle.value if isinstance(m.handle, C.c_void_p) else m.handle
        if isinstance(keys, tuple):
            data, offsets = keys
            d.n_q = offsets.numel() - 1
            d.data = _device_tensor(data, "data", 1, 0).value
            d.data_len = data.numel()
            d.offsets = _device_tensor(offsets, "offsets", 8, d.n_q + 1).value
        else:
            d.n_q = keys.numel()
            d.keys = _device_tensor(keys, "keys", 8, d.n_q).value
        if out is not None and d.n_q:
            # an unloaded handle (index_bytes 0) is left for the library to refuse
            d.out = (_device_tensor(out, "out", m.index_bytes, d.n_q) if m.index_bytes else _dev_ptr(out)).value
    return arr


def multi_max() -> int:
    """Most batches one multi-MPHF launch (plan, server launch, query_multi) takes."""
    return int(lib().ptrhash_multi_max())


def query_multi(batches, stream=None):
    """One persistent launch over all batches (see ptrhash_query_multi)."""
    arr = make_descs(batches)
    _check(lib().ptrhash_query_multi(arr, len(batches), _stream(stream)), "ptrhash_query_multi")


def query_multi_noalloc(batches, stream=None):
    """As query_multi through the entry point that allocates nothing (a fixed
    table of at most 256 batches per GPU; see ptrhash_query_multi_noalloc)."""
    arr = make_descs(batches)
    _check(lib().ptrhash_query_multi_noalloc(arr, len(batches), _stream(stream)), "ptrhash_query_multi_noalloc")


class HostBuffer:
    """Mapped, pinned host memory from ptrhash_host_alloc (freed on close or
    collection); ``array`` is a numpy view of it."""

    def __init__(self, nbytes: int):
        p = C.c_void_p()
        _check(lib().ptrhash_host_alloc(int(max(1, nbytes)), C.byref(p)), "ptrhash_host_alloc")
        self._p = p.value
        self.nbytes = int(max(1, nbytes))
        self.array = np.ctypeslib.as_array((C.c_uint8 * self.nbytes).from_address(self._p))

    def view(self, offset: int, count: int, dtype) -> np.ndarray:
        """count elements of dtype at byte offset (a multiple of the item size)."""
        dt = np.dtype(dtype)
        return self.array[offset:offset + count * dt.itemsize].view(dt)

    def close(self):
        if self._p:
            self.array = None
            lib().ptrhash_host_free(C.c_void_p(self._p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_multi_kernel(keys_per_lane=4, block=256, blocks_per_cu=0):
    """Process default launch shape of multi-MPHF launches (new plans and
    servers, and query_multi)."""
    _check(lib().ptrhash_set_multi_kernel(int(keys_per_lane), int(block), int(blocks_per_cu)),
           "ptrhash_set_multi_kernel")


class MultiPlan:
    """A reusable, graph-capturable multi-batch launch (ptrhash_multi_plan_*)."""

    def __init__(self, max_descs: int = 64):
        h = C.c_void_p()
        _check(lib().ptrhash_multi_plan_create(int(max_descs), C.byref(h)), "ptrhash_multi_plan_create")
        self._h = h

    def set(self, batches):
        arr = make_descs(batches)
        _check(lib().ptrhash_multi_plan_set(self._h, arr, len(batches)), "ptrhash_multi_plan_set")

    def launch(self, stream=None):
        _check(lib().ptrhash_multi_plan_launch(self._h, _stream(stream)), "ptrhash_multi_plan_launch")

    def set_kernel(self, keys_per_lane=4, block=256, blocks_per_cu=0):
        """Launch shape (call set() again before the next launch)."""
        _check(lib().ptrhash_multi_plan_set_kernel(self._h, int(keys_per_lane), int(block), int(blocks_per_cu)),
               "ptrhash_multi_plan_set_kernel")

    def close(self):
        if self._h:
            lib().ptrhash_multi_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching query server over resident MPHFs (host keys in,
    host indices out); see ptrhash_server_* in include/ptrhash.h."""

    def __init__(self, streams=None, max_batches=None, slot_keys=None, max_queued_keys=None, copy_threads=None,
                 zero_copy=None, multi_kernel=None):
        """multi_kernel: (keys_per_lane, block, blocks_per_cu) of the
        multi-MPHF launches, or None for the process default."""
        cfg = ServerConfig()
        _check(lib().ptrhash_server_default_config(C.byref(cfg)), "ptrhash_server_default_config")
        if multi_kernel is not None:
            cfg.keys_per_lane, cfg.block, cfg.blocks_per_cu = (int(x) for x in multi_kernel)
        if streams is not None:
            cfg.streams = streams
        if max_batches is not None:
            cfg.max_batches = max_batches
        if slot_keys is not None:
            cfg.slot_keys = slot_keys
        if copy_threads is not None:
            cfg.copy_threads = copy_threads
        if zero_copy is not None:
            cfg.zero_copy = int(bool(zero_copy))
        if max_queued_keys is not None:
            cfg.max_queued_keys = max_queued_keys
        elif cfg.max_queued_keys < cfg.slot_keys:
            cfg.max_queued_keys = cfg.slot_keys
        self.cfg = cfg
        h = C.c_void_p()
        _check(lib().ptrhash_server_create(C.byref(cfg), C.byref(h)), "ptrhash_server_create")
        self._h = h

    def submit(self, mphf: "Mphf", keys: np.ndarray, out: np.ndarray) -> int:
        """keys: host uint64 array; out: host uint32/uint64 array (the handle's
        index width). Both must stay alive until wait() returns."""
        assert keys.dtype == np.uint64 and keys.flags.c_contiguous and out.flags.c_contiguous
        want = np.uint64 if mphf.params.index_bits == 64 else np.uint32
        if out.dtype != want or len(out) < len(keys):
            raise ValueError(f"out must be {np.dtype(want).name}[{len(keys)}]")
        t = C.c_uint64()
        _check(lib().ptrhash_server_submit(self._h, mphf.handle, _np_ptr(keys), len(keys), _np_ptr(out),
                                           C.byref(t)), "ptrhash_server_submit")
        return t.value

    def submit_mapped(self, mphf: "Mphf", keys: np.ndarray, out: np.ndarray) -> int:
        """As submit, with keys and out inside a HostBuffer (ptrhash_host_alloc
        memory): the kernel reads and writes them in place (no host copies)."""
        assert keys.dtype == np.uint64 and keys.flags.c_contiguous and out.flags.c_contiguous
        want = np.uint64 if mphf.params.index_bits == 64 else np.uint32
        if out.dtype != want or len(out) < len(keys):
            raise ValueError(f"out must be {np.dtype(want).name}[{len(keys)}]")
        t = C.c_uint64()
        _check(lib().ptrhash_server_submit_mapped(self._h, mphf.handle, _np_ptr(keys), len(keys), _np_ptr(out),
                                                  C.byref(t)), "ptrhash_server_submit_mapped")
        return t.value

    def wait(self, ticket: int) -> float:
        lat = C.c_double()
        _check(lib().ptrhash_server_wait(self._h, int(ticket), C.byref(lat)), "ptrhash_server_wait")
        return lat.value

    def replay(self, reqs, mapped=False) -> float:
        """reqs: list of (Mphf, keys ndarray, out ndarray, arrival_us);
        mapped: the arrays are inside a HostBuffer."""
        arr = (ServerRequest * max(1, len(reqs)))()
        for i, (m, k, o, t) in enumerate(reqs):
            arr[i].handle = m.handle.value if isinstance(m.handle, C.c_void_p) else m.handle
            arr[i].keys = k.ctypes.data if k.size else None
            arr[i].n_q = len(k)
            arr[i].out = o.ctypes.data if o.size else None
            arr[i].arrival_us = float(t)
            arr[i].mapped = int(bool(mapped))
        span = C.c_double()
        _check(lib().ptrhash_server_replay(self._h, arr, len(reqs), C.byref(span)), "ptrhash_server_replay")
        return span.value

    def stats(self) -> dict:
        m = ServerMetrics()
        _check(lib().ptrhash_server_stats(self._h, C.byref(m)), "ptrhash_server_stats")
        return m.as_dict()

    def reset_stats(self):
        _check(lib().ptrhash_server_reset_stats(self._h), "ptrhash_server_reset_stats")

    def close(self):
        if self._h:
            rc = lib().ptrhash_server_destroy(self._h)
            self._h = None
            _check(rc, "ptrhash_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gen_strings(n, seed, order_seed=0, shuffled=False, start=0, count=None, device="cuda", pad=64):
    """Device copy of strings start.. of the n-string set (or of its shuffled
    order): returns (data uint8 tensor with `pad` zero bytes after the last
    string, offsets int64 tensor of count+1 entries starting at 0)."""
    import torch

    count = n - start if count is None else count
    lens = torch.empty(count, dtype=torch.int64, device=device)
    _check(lib().ptrhash_gen_string_lengths(int(n), int(seed), int(order_seed), int(bool(shuffled)), int(start),
                                            count, _dev_ptr(lens), _stream(None)), "ptrhash_gen_string_lengths")
    offsets = torch.zeros(count + 1, dtype=torch.int64, device=device)
    torch.cumsum(lens, 0, out=offsets[1:])
    del lens
    total = int(offsets[-1])
    data = torch.zeros(total + pad, dtype=torch.uint8, device=device)
    _check(lib().ptrhash_gen_string_bytes(int(n), int(seed), int(order_seed), int(bool(shuffled)), int(start),
                                          count, _dev_ptr(offsets), _dev_ptr(data), _stream(None)),
           "ptrhash_gen_string_bytes")
    return data, offsets
