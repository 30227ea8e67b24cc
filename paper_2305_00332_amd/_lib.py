"""ctypes binding of libmmlttb.so: argument marshalling only.

Every step of the downsampling path runs in the library's HIP kernels. torch
supplies device memory (tensors) and the stream (the current HIP stream).
There is no fallback: if the library is missing or no GPU is present the
calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmlttb.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP = 0, -1, -2, -3, -4
NOALLOC_SCRATCH_BYTES = 4 << 20  # MMLTTB_NOALLOC_SCRATCH_BYTES
X_IMPLICIT, X_INT64, X_F64 = 0, 1, 2
Y_F32, Y_F64, Y_I32 = 0, 1, 2

# names declared in include/libmmlttb.h
EXPORTS = (
    "mmlttb_version",
    "mmlttb_last_error",
    "mmlttb_workspace_size",
    "mmlttb_lttb_workspace_size",
    "mmlttb_minmax",
    "mmlttb_lttb",
    "mmlttb_minmaxlttb",
    "mmlttb_minmaxlttb_noalloc",
    "mmlttb_lttb_means",
    "mmlttb_batched_workspace_size",
    "mmlttb_minmaxlttb_batched",
    "mmlttb_simplify_workspace_size",
    "mmlttb_minmax_simplify",
    "mmlttb_typed_workspace_size",
    "mmlttb_minmax_typed",
    "mmlttb_minmaxlttb_typed",
    "mmlttb_xbins_workspace_size",
    "mmlttb_minmax_xbins",
    "mmlttb_minmaxlttb_xbins",
    "mmlttb_m4_workspace_size",
    "mmlttb_m4",
    "mmlttb_everynth",
    "mmlttb_set_graph_cache",
    "mmlttb_graph_cache_stats",
    "mmlttb_set_tuning",
    "mmlttb_get_tuning",
    "mmlttb_profile_enable",
    "mmlttb_profile_reset",
    "mmlttb_profile_read",
    "mmlttb_profile_samples",
)


class MmlttbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libmmlttb error {code}: {msg}")
        self.code = code


class Segment(ctypes.Structure):
    _fields_ = [
        ("offset", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("n_out", ctypes.c_int64),
        ("r_ps", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("out_offset", ctypes.c_int64),
    ]


_lib = None
tuning_source = None  # what set the execution tuning when the library loaded (MMLTTB_TUNE)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def load(path: str = LIB_PATH):
    """Load libmmlttb.so (raises if it is not built) and apply the execution
    tuning that MMLTTB_TUNE selects (off | use, the default | retune)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2305_00332_amd.build` first")
    lib = ctypes.CDLL(path)
    lib.mmlttb_version.restype = ctypes.c_char_p
    lib.mmlttb_last_error.restype = ctypes.c_char_p
    lib.mmlttb_workspace_size.argtypes = [_i64, _i64, _i32]
    lib.mmlttb_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_lttb_workspace_size.argtypes = [_i64, _i64]
    lib.mmlttb_lttb_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_minmax.argtypes = [ctypes.c_int, _vp, _vp, _i64, _i64, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.mmlttb_lttb.argtypes = [ctypes.c_int, _vp, _vp, _i64, _i64, _vp, _vp, ctypes.c_size_t, _vp]
    lib.mmlttb_minmaxlttb.argtypes = [ctypes.c_int, _vp, _vp, _i64, _i64, _i32, _vp, _vp, ctypes.c_size_t, _vp]
    lib.mmlttb_minmaxlttb_noalloc.argtypes = [ctypes.c_int, _vp, _vp, _i64, _i64, _i32, _vp, _vp]
    lib.mmlttb_batched_workspace_size.argtypes = [ctypes.POINTER(Segment), _i64]
    lib.mmlttb_batched_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_minmaxlttb_batched.argtypes = [ctypes.c_int, _vp, _vp, ctypes.POINTER(Segment), _i64, _vp, _vp,
                                              ctypes.c_size_t, _vp]
    lib.mmlttb_simplify_workspace_size.argtypes = [_i64, _i64, _i32]
    lib.mmlttb_simplify_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_minmax_simplify.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _i64, _i64, _i32, _vp, _vp,
                                           ctypes.c_size_t, _vp]
    lib.mmlttb_typed_workspace_size.argtypes = [_i64, _i64, _i32]
    lib.mmlttb_typed_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_minmax_typed.argtypes = [ctypes.c_int, _vp, _i64, _i64, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.mmlttb_minmaxlttb_typed.argtypes = [ctypes.c_int, _vp, ctypes.c_int, _vp, _i64, _i64, _i32, _vp, _vp,
                                            ctypes.c_size_t, _vp]
    lib.mmlttb_xbins_workspace_size.argtypes = [_i64, _i64, _i32]
    lib.mmlttb_xbins_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_minmax_xbins.argtypes = [_vp, _vp, _i64, _i64, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.mmlttb_minmaxlttb_xbins.argtypes = [_vp, _vp, _i64, _i64, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.mmlttb_m4_workspace_size.argtypes = [_i64, _i64]
    lib.mmlttb_m4_workspace_size.restype = ctypes.c_size_t
    lib.mmlttb_m4.argtypes = [_vp, _i64, _i64, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.mmlttb_everynth.argtypes = [_i64, _i64, _vp, _vp]
    lib.mmlttb_set_graph_cache.argtypes = [ctypes.c_int]
    lib.mmlttb_graph_cache_stats.argtypes = [ctypes.POINTER(_i64)] * 3
    lib.mmlttb_set_tuning.argtypes = [ctypes.c_int, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64]
    lib.mmlttb_get_tuning.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64)]
    lib.mmlttb_lttb_means.argtypes = [ctypes.c_int, _vp, _vp, _i64, _i64, _vp, _vp, _vp]
    lib.mmlttb_profile_enable.argtypes = [ctypes.c_int]
    lib.mmlttb_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    lib.mmlttb_profile_samples.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_float), _i64,
                                           ctypes.POINTER(_i64)]
    for f in ("mmlttb_minmax", "mmlttb_lttb", "mmlttb_minmaxlttb", "mmlttb_minmaxlttb_noalloc", "mmlttb_lttb_means", "mmlttb_minmaxlttb_batched",
              "mmlttb_m4",
              "mmlttb_minmax_xbins", "mmlttb_minmaxlttb_xbins", "mmlttb_minmax_typed", "mmlttb_minmaxlttb_typed",
              "mmlttb_minmax_simplify",
              "mmlttb_everynth", "mmlttb_set_graph_cache", "mmlttb_graph_cache_stats", "mmlttb_set_tuning",
              "mmlttb_get_tuning", "mmlttb_profile_enable", "mmlttb_profile_reset", "mmlttb_profile_read",
              "mmlttb_profile_samples"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    from . import autotune

    global tuning_source
    tuning_source = autotune.on_load()
    return lib


def check(rc: int):
    if rc != OK:
        raise MmlttbError(rc, load().mmlttb_last_error().decode())


def last_error() -> str:
    return load().mmlttb_last_error().decode()


def version() -> str:
    return load().mmlttb_version().decode()


def stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def ptr(t) -> int | None:
    return None if t is None else t.data_ptr()
