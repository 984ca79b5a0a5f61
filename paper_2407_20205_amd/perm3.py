"""Thin ctypes binding of libperm3.so (include/perm3.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  Loading fails loudly when the library has not been
built; calls that need the GPU fail with PERM_EDEVICE when there is none.
torch is used only to hand over device memory and streams.
"""
from __future__ import annotations

import ctypes
import functools
import os
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libperm3.so")

PERM_MAX_N = 63
PERM_MAX_N_WIDE = 128
PERM_WIDE_MAX_COUNT = 1 << 62
PERM_MAX_BATCH = 1 << 22
PERM_OK = 0
PERM_EINVAL = -1
PERM_EDOMAIN = -2
PERM_ENOMEM = -3
PERM_EDEVICE = -4
PERM_EAGAIN = -5
PERM_ESTATE = -6
PERM_RESULT_INVALID = 0xFF
PERM_GEN_ENUMERATE = 0
PERM_GEN_SPLITMIX = 1
PERM_F3_ADD = 0
PERM_F3_SUB = 1
PERM_F3_MUL = 2
PERM_F3_DIV = 3
PERM_F3_NEG = 4
PERM_F3_MAX_LEN = 1 << 40
PERM_MAX_TALLIES = 1 << 20
PERM_NOALLOC_MAX_COUNT = 8192
PERM_NOALLOC_SCRATCH_BYTES = 17212416
PERM_POLICY_SRPT = 0
PERM_POLICY_FIFO = 1
PERM_TUNE_SMALL = 0
PERM_TUNE_MID = 1
PERM_TUNE_LARGE = 2
PERM_TUNE_BATCH = 3
PERM_TUNE_CLASSES = 4
TUNE_CLASS_NAMES = ("small", "mid", "large", "batch")
PERM_TUNE_SRC_DEFAULT = 0
PERM_TUNE_SRC_CACHE = 1
PERM_TUNE_SRC_SET = 2
PERM_TUNE_SRC_AUTOTUNE = 3
TUNE_SOURCE_NAMES = ("default", "cache", "set", "autotune")


class PermError(RuntimeError):
    def __init__(self, code: int, msg: str, index: int = -1):
        super().__init__(f"{msg} (status {code})")
        self.code = code
        self.index = index


class perm_server_cfg(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("queue_cap", ctypes.c_int32),
                ("work_budget", ctypes.c_uint64), ("quantum", ctypes.c_uint64),
                ("policy", ctypes.c_int32), ("fast_max_n", ctypes.c_int32),
                ("tick_timeout_ms", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class perm_done(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("n", ctypes.c_int32),
                ("result", ctypes.c_uint8), ("pad", ctypes.c_uint8 * 7),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]


class perm_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("ticks", ctypes.c_uint64), ("tick_indices", ctypes.c_uint64),
                ("busy_ns", ctypes.c_uint64), ("active_slots", ctypes.c_int32),
                ("queued", ctypes.c_int32)]


class perm_tuning(ctypes.Structure):
    _fields_ = [("waves_per_simd", ctypes.c_int32), ("body_log", ctypes.c_int32),
                ("chunk_log_max", ctypes.c_int32), ("tasks_per_wave", ctypes.c_int32),
                ("direct_max_n", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("states_per_lane", ctypes.c_int32), ("body_log_mid", ctypes.c_int32),
                ("mid_max_n", ctypes.c_int32), ("max_tasks_log", ctypes.c_int32),
                ("min_task_log", ctypes.c_int32), ("queue_task_log", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class perm_timing(ctypes.Structure):
    _fields_ = [("hot_kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("indices", ctypes.c_uint64), ("launches", ctypes.c_int32),
                ("graph_replayed", ctypes.c_int32)]


class perm_device_info(ctypes.Structure):
    _fields_ = [("compute_units", ctypes.c_int32), ("simds_per_cu", ctypes.c_int32),
                ("wave_size", ctypes.c_int32), ("max_clock_khz", ctypes.c_int32),
                ("arch", ctypes.c_char * 64)]


# (name, restype, argtypes) for every export of include/perm3.h
_u8p = ctypes.POINTER(ctypes.c_uint8)
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
EXPORTS = [
    ("perm_mod3", _i32, [_vp, _i32, _vp]),
    ("perm_mod3_range_tally", _i32, [_vp, _i32, ctypes.c_uint64, ctypes.c_uint64, _vp]),
    ("perm_mod3_range_tally_wide", _i32, [_vp, _i32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _vp]),
    ("perm_f3_pack", _i32, [_vp, ctypes.c_int64, _vp, _vp, _vp]),
    ("perm_f3_unpack", _i32, [_vp, ctypes.c_int64, _vp, _vp]),
    ("perm_f3_op", _i32, [_i32, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    ("perm_f3_dot", _i32, [_vp, _vp, ctypes.c_int64, _vp, _vp]),
    ("perm_mod3_batch", _i32, [_vp, _vp, _i32, _vp]),
    ("perm_mod3_batch_dev", _i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    ("perm_mod3_batch_packed", _i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    ("perm_mod3_batch_packed_noalloc", _i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    ("perm_mod3_from_tallies", _i32, [_i32, _vp, _i32, _vp]),
    ("perm_mod3_pack", _i32, [_vp, _i32, _vp]),
    ("perm_mod3_census", _i32, [_i32, _i32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _vp]),
    ("perm_server_create", _i32, [_vp, _vp]),
    ("perm_server_submit", _i32, [_vp, _vp, _i32, ctypes.c_uint64]),
    ("perm_server_poll", _i32, [_vp, _vp, _i32, _vp, ctypes.c_int64]),
    ("perm_server_stats_get", _i32, [_vp, _vp]),
    ("perm_server_destroy", _i32, [_vp]),
    ("perm_tuning_get", _i32, [_vp]),
    ("perm_tuning_set", _i32, [_vp]),
    ("perm_tuning_get_class", _i32, [_i32, _vp, _vp]),
    ("perm_tuning_set_class", _i32, [_i32, _vp]),
    ("perm_tuning_reset", _i32, [_i32]),
    ("perm_tuning_cache_load", _i32, [ctypes.c_char_p, _vp]),
    ("perm_tuning_cache_save", _i32, [ctypes.c_char_p]),
    ("perm_autotune", _i32, [_i32, _i32, _vp]),
    ("perm_autotune_batch", _i32, [_vp, _vp, _vp, _i32, _vp, _i32, _vp]),
    ("perm_timing_enable", _i32, [_i32]),
    ("perm_timing_last", _i32, [_vp]),
    ("perm_device_info_get", _i32, [_vp]),
    ("perm_bipedal_ops", _i32, [_vp, _i32, _vp]),
    ("perm_strerror", ctypes.c_char_p, [_i32]),
    ("perm_last_error", ctypes.c_char_p, []),
    ("perm_last_error_index", ctypes.c_int64, []),
    ("perm_version", ctypes.c_char_p, []),
]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libperm3.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2407_20205_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in EXPORTS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != PERM_OK:
        L = lib()
        raise PermError(rc, L.perm_last_error().decode(errors="replace"), L.perm_last_error_index())


def _mat(A) -> tuple[np.ndarray, int]:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.uint8))
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("square matrix expected")
    return A, A.shape[0]


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# ---------------------------------------------------------------- host calls

def perm_mod3(A) -> int:
    A, n = _mat(A)
    out = ctypes.c_uint8(0)
    _check(lib().perm_mod3(_ptr(A) if A.size else None, n, ctypes.addressof(out)))
    return int(out.value)


def perm_mod3_range_tally(A, begin: int, end: int) -> int:
    A, n = _mat(A)
    t = ctypes.c_int64(0)
    _check(lib().perm_mod3_range_tally(_ptr(A) if A.size else None, n, begin, end, ctypes.addressof(t)))
    return int(t.value)


def perm_mod3_range_tally_wide(A, begin: int, count: int) -> int:
    """T(begin, begin + count) for an n x n matrix with n <= 128 (Gray indices up to 2^128)."""
    A, n = _mat(A)
    if not 0 <= begin < (1 << 128) or not 0 <= count < (1 << 64):
        raise ValueError("begin must fit 128 bits and count 64 bits")
    t = ctypes.c_int64(0)
    _check(lib().perm_mod3_range_tally_wide(_ptr(A) if A.size else None, n, begin >> 64,
                                            begin & ((1 << 64) - 1), count, ctypes.addressof(t)))
    return int(t.value)


def perm_mod3_batch(mats: Sequence) -> np.ndarray:
    arrs = [_mat(M)[0] for M in mats]
    count = len(arrs)
    ns = np.array([a.shape[0] for a in arrs], dtype=np.int32)
    ptrs = (ctypes.c_void_p * max(count, 1))(*[a.ctypes.data if a.size else None for a in arrs])
    out = np.zeros(max(count, 1), dtype=np.uint8)
    _check(lib().perm_mod3_batch(ptrs, _ptr(ns), count, _ptr(out)))
    return out[:count]


def perm_mod3_pack(A) -> np.ndarray:
    A, n = _mat(A)
    planes = np.zeros(max(2 * n, 1), dtype=np.uint64)
    _check(lib().perm_mod3_pack(_ptr(A) if A.size else None, n, _ptr(planes)))
    return planes[:2 * n]


def perm_mod3_census(n: int, generator: int, key: int, first: int, count: int) -> tuple[int, int, int]:
    """How many of the generated matrices have perm mod 3 = 0, 1, 2 (see include/perm3.h)."""
    c = (ctypes.c_uint64 * 3)()
    _check(lib().perm_mod3_census(n, generator, key, first, count, ctypes.addressof(c)))
    return int(c[0]), int(c[1]), int(c[2])


def perm_mod3_from_tallies(n: int, tallies) -> int:
    """perm(A) mod 3 of an n x n matrix from the exact tallies of Gray ranges covering [0, 2^n) once
    (the shards of a long run); the sum and its reduction run on the device."""
    t = np.ascontiguousarray(np.asarray(tallies, dtype=np.int64).reshape(-1))
    out = ctypes.c_uint8(0)
    _check(lib().perm_mod3_from_tallies(n, _ptr(t) if t.size else None, int(t.size), ctypes.addressof(out)))
    return int(out.value)


# ---------------------------------------------------------------- device calls (torch tensors)
#
# The C calls take raw device addresses and sizes; a tensor of the wrong type,
# length or device would send the kernels outside their buffers.  Each tensor
# is therefore checked here, before any C call: dtype, contiguity, length and
# device, in that order.

@functools.lru_cache(maxsize=None)
def _dtypes(*names):
    import torch
    return tuple(getattr(torch, k) for k in names if hasattr(torch, k))


def _need(t, name, dtypes, min_numel):
    """Check one tensor argument's type, layout and length."""
    if t is None:
        raise ValueError(f"{name} is required")
    if not hasattr(t, "data_ptr") or not hasattr(t, "dtype"):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} elements; the call needs at least {min_numel}")


def _one_device(**tensors):
    """Every given tensor (None skipped) on the same CUDA device."""
    dev = None
    for name, t in tensors.items():
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError(f"{name} must be on a CUDA device, not {t.device}")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{name} is on {t.device}, the other tensors on {dev}")


def _check_batch_args(first, first_name, first_dtypes, index, index_name, ns_dev, out_dev, hist_dev):
    """Arguments of the batched device calls; returns count."""
    i32, i64, u8 = _dtypes("int32"), _dtypes("int64"), _dtypes("uint8")
    _need(ns_dev, "ns_dev", i32, 0)
    count = int(ns_dev.numel())
    _need(first, first_name, first_dtypes, 0)
    _need(index, index_name, i64, count)
    _need(out_dev, "out_dev", u8, count)
    if hist_dev is not None:
        _need(hist_dev, "hist_dev", _dtypes("int64", "uint64"), 64 * 3)
    _one_device(ns_dev=ns_dev, **{first_name: first, index_name: index}, out_dev=out_dev, hist_dev=hist_dev)
    return count


def _dptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream))


def perm_mod3_batch_dev(mats_dev, offs_dev, ns_dev, out_dev, hist_dev=None, stream=None) -> None:
    """All tensors on one GPU: uint8 bytes, int64 offsets, int32 n, uint8 out, int64/uint64 hist[64*3]."""
    count = _check_batch_args(mats_dev, "mats_dev", _dtypes("uint8"), offs_dev, "offs_dev", ns_dev, out_dev,
                              hist_dev)
    _check(lib().perm_mod3_batch_dev(_dptr(mats_dev), _dptr(offs_dev), _dptr(ns_dev), count,
                                     _dptr(out_dev), _dptr(hist_dev), _stream(stream)))


def perm_mod3_batch_packed(planes_dev, row_off_dev, ns_dev, out_dev, hist_dev=None, stream=None) -> None:
    """planes_dev: int64/uint64 (mag, sgn) word pairs; row_off_dev: int64 first row per matrix."""
    count = _check_batch_args(planes_dev, "planes_dev", _dtypes("int64", "uint64"), row_off_dev, "row_off_dev",
                              ns_dev, out_dev, hist_dev)
    _check(lib().perm_mod3_batch_packed(_dptr(planes_dev), _dptr(row_off_dev), _dptr(ns_dev), count,
                                        _dptr(out_dev), _dptr(hist_dev), _stream(stream)))


def perm_mod3_batch_packed_noalloc(planes_dev, row_off_dev, ns_dev, out_dev, hist_dev=None, stream=None) -> None:
    """perm_mod3_batch_packed with the library's static work set: allocates no device memory;
    at most PERM_NOALLOC_MAX_COUNT matrices; overlapping calls on one GPU race (include/perm3.h)."""
    count = _check_batch_args(planes_dev, "planes_dev", _dtypes("int64", "uint64"), row_off_dev, "row_off_dev",
                              ns_dev, out_dev, hist_dev)
    _check(lib().perm_mod3_batch_packed_noalloc(_dptr(planes_dev), _dptr(row_off_dev), _dptr(ns_dev), count,
                                                _dptr(out_dev), _dptr(hist_dev), _stream(stream)))


# ---------------------------------------------------------------- vectors over F_3 (device tensors)

def f3_words(length: int) -> int:
    """Word pairs of a bipedal vector of `length` elements."""
    return (length + 63) // 64


def _planes_dtypes():
    return _dtypes("int64", "uint64")


def f3_pack(v_dev, planes_dev, invalid_dev=None, stream=None) -> None:
    """phi: uint8 tensor v_dev (values 0, 1, 2) into int64 planes_dev[2 * f3_words(len)]; bytes > 2 are
    packed as 0 and their count is added to invalid_dev[0] (int64/uint64 tensor) when given."""
    _need(v_dev, "v_dev", _dtypes("uint8"), 0)
    length = int(v_dev.numel())
    _need(planes_dev, "planes_dev", _planes_dtypes(), 2 * f3_words(length))
    if invalid_dev is not None:
        _need(invalid_dev, "invalid_dev", _planes_dtypes(), 1)
    _one_device(v_dev=v_dev, planes_dev=planes_dev, invalid_dev=invalid_dev)
    _check(lib().perm_f3_pack(_dptr(v_dev), length, _dptr(planes_dev), _dptr(invalid_dev), _stream(stream)))


def f3_unpack(planes_dev, length: int, v_dev, stream=None) -> None:
    """psi: planes into uint8 v_dev[length]."""
    # a negative length is refused by the C call (PERM_EINVAL)
    _need(planes_dev, "planes_dev", _planes_dtypes(), 2 * f3_words(max(length, 0)))
    _need(v_dev, "v_dev", _dtypes("uint8"), max(length, 0))
    _one_device(planes_dev=planes_dev, v_dev=v_dev)
    _check(lib().perm_f3_unpack(_dptr(planes_dev), length, _dptr(v_dev), _stream(stream)))


def f3_op(op: int, a_dev, b_dev, out_dev, words: int | None = None, stream=None) -> None:
    """out = a op b (Theorem 2.1) over `words` word pairs (default: all of a)."""
    _need(a_dev, "a_dev", _planes_dtypes(), 0)
    w = int(a_dev.numel()) // 2 if words is None else words
    need = 2 * max(w, 0)          # a negative count is refused by the C call (PERM_EINVAL)
    _need(a_dev, "a_dev", _planes_dtypes(), need)
    if op != PERM_F3_NEG or b_dev is not None:
        _need(b_dev, "b_dev", _planes_dtypes(), need)
    _need(out_dev, "out_dev", _planes_dtypes(), need)
    _one_device(a_dev=a_dev, b_dev=b_dev, out_dev=out_dev)
    _check(lib().perm_f3_op(op, _dptr(a_dev), _dptr(b_dev), _dptr(out_dev), w, _stream(stream)))


def f3_dot(a_dev, b_dev, sum_dev, words: int | None = None, stream=None) -> None:
    """sum_dev[0] (int64 tensor) = sum_e a_e b_e over the integers; the F_3 dot product is it mod 3."""
    _need(a_dev, "a_dev", _planes_dtypes(), 0)
    w = int(a_dev.numel()) // 2 if words is None else words
    need = 2 * max(w, 0)
    _need(a_dev, "a_dev", _planes_dtypes(), need)
    _need(b_dev, "b_dev", _planes_dtypes(), need)
    _need(sum_dev, "sum_dev", _dtypes("int64"), 1)
    _one_device(a_dev=a_dev, b_dev=b_dev, sum_dev=sum_dev)
    _check(lib().perm_f3_dot(_dptr(a_dev), _dptr(b_dev), w, _dptr(sum_dev), _stream(stream)))


# ---------------------------------------------------------------- tuning, timing, device

def tuning_get() -> perm_tuning:
    t = perm_tuning()
    _check(lib().perm_tuning_get(ctypes.addressof(t)))
    return t


def tuning_set(t: perm_tuning) -> None:
    _check(lib().perm_tuning_set(ctypes.addressof(t)))


def tuning_get_class(cls: int) -> tuple[perm_tuning, int]:
    """(tuning, source) of one tuning class (PERM_TUNE_*; source PERM_TUNE_SRC_*)."""
    t = perm_tuning()
    src = ctypes.c_int32(0)
    _check(lib().perm_tuning_get_class(cls, ctypes.addressof(t), ctypes.addressof(src)))
    return t, int(src.value)


def tuning_set_class(cls: int, t: perm_tuning) -> None:
    _check(lib().perm_tuning_set_class(cls, ctypes.addressof(t)))


def tuning_reset(with_cache: bool = False) -> None:
    """Every class back to the library's defaults; with_cache: then the tuning cache a new context
    loads, as when the context was made."""
    _check(lib().perm_tuning_reset(1 if with_cache else 0))


def tuning_cache_load(path: str) -> int:
    """Apply the lines of a tuning cache file that match this device; returns the classes set."""
    got = ctypes.c_int32(0)
    _check(lib().perm_tuning_cache_load(os.fsencode(path), ctypes.addressof(got)))
    return int(got.value)


def tuning_cache_save(path: str) -> None:
    _check(lib().perm_tuning_cache_save(os.fsencode(path)))


class saved_tunings:
    """Context manager: every class's tuning, and where it came from, put back on exit.  The
    classes start again as a new context makes them (defaults, then the tuning cache); a class
    whose saved values differ from that is set, and then reads as source PERM_TUNE_SRC_SET unless
    it was that already."""

    def __enter__(self):
        self._saved = [tuning_get_class(k) for k in range(PERM_TUNE_CLASSES)]
        return self

    def __exit__(self, *exc):
        tuning_reset(with_cache=True)
        for k, (t, src) in enumerate(self._saved):
            now, now_src = tuning_get_class(k)
            if now.as_dict() != t.as_dict() or now_src != src:
                tuning_set_class(k, t)
        return False


def autotune(n: int, budget_ms: int = 20000) -> perm_tuning:
    """Tune the class of a one-matrix host call of order n (12..63); see include/perm3.h."""
    t = perm_tuning()
    _check(lib().perm_autotune(n, budget_ms, ctypes.addressof(t)))
    return t


def autotune_batch(planes_dev, row_off_dev, ns_dev, out_dev, budget_ms: int = 60000) -> perm_tuning:
    """Tune class PERM_TUNE_BATCH on a packed batch already on the GPU (as perm_mod3_batch_packed)."""
    count = _check_batch_args(planes_dev, "planes_dev", _dtypes("int64", "uint64"), row_off_dev, "row_off_dev",
                              ns_dev, out_dev, None)
    t = perm_tuning()
    _check(lib().perm_autotune_batch(_dptr(planes_dev), _dptr(row_off_dev), _dptr(ns_dev), count,
                                     _dptr(out_dev), budget_ms, ctypes.addressof(t)))
    return t


def timing_enable(on: bool = True) -> None:
    _check(lib().perm_timing_enable(1 if on else 0))


def timing_last() -> perm_timing:
    t = perm_timing()
    _check(lib().perm_timing_last(ctypes.addressof(t)))
    return t


def device_info() -> perm_device_info:
    d = perm_device_info()
    _check(lib().perm_device_info_get(ctypes.addressof(d)))
    return d


def bipedal_ops(words: np.ndarray) -> np.ndarray:
    """words: uint32[count, 4] = (mag1, sgn1, mag2, sgn2) -> uint32[count, 8] (+, -, x, walk's -)."""
    w = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros((max(len(w), 1), 8), dtype=np.uint32)
    _check(lib().perm_bipedal_ops(_ptr(w), len(w), _ptr(out)))
    return out[:len(w)]


def strerror(code: int) -> str:
    return lib().perm_strerror(code).decode()


def version() -> str:
    return lib().perm_version().decode()


# ---------------------------------------------------------------- serving

class Server:
    """perm_server_*: continuous-batching request loop (C++ worker thread)."""

    def __init__(self, max_slots: int = 4096, queue_cap: int = 1 << 16, work_budget: int = 0,
                 quantum: int = 0, policy: int = PERM_POLICY_SRPT, fast_max_n: int = 0,
                 tick_timeout_ms: int = 0):
        """fast_max_n: requests of order <= fast_max_n run in one-launch batches beside the tick
        (0: the library default, -1: none).  tick_timeout_ms: a tick running longer fails the
        server and every request it holds (0: no limit)."""
        cfg = perm_server_cfg(max_slots, queue_cap, work_budget, quantum, policy, fast_max_n,
                              tick_timeout_ms, 0)
        h = ctypes.c_void_p(None)
        _check(lib().perm_server_create(ctypes.addressof(cfg), ctypes.addressof(h)))
        self._h = h

    def submit(self, A, tag: int) -> bool:
        """False when the queue is full (PERM_EAGAIN)."""
        A, n = _mat(A)
        rc = lib().perm_server_submit(self._h, _ptr(A) if A.size else None, n, tag)
        if rc == PERM_EAGAIN:
            return False
        _check(rc)
        return True

    def poll(self, max_items: int = 1024, timeout_us: int = 0) -> list[perm_done]:
        buf = (perm_done * max_items)()
        got = ctypes.c_int32(0)
        _check(lib().perm_server_poll(self._h, buf, max_items, ctypes.addressof(got), timeout_us))
        return [buf[i] for i in range(got.value)]

    def stats(self) -> perm_server_stats:
        s = perm_server_stats()
        _check(lib().perm_server_stats_get(self._h, ctypes.addressof(s)))
        return s

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(lib().perm_server_destroy(self._h))
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
