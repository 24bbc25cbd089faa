"""ctypes binding of ``libmvd.so`` (the C ABI declared in ``include/mvd.h``).

Argument marshalling only: every step of the deconvolution runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int, c_int32, c_size_t, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmvd.so")

MVD_OK = 0
MVD_ERR_ARG = -1
MVD_ERR_STATE = -2
MVD_ERR_WORKSPACE = -3
MVD_ERR_DEVICE = -4
MVD_ERR_LAUNCH = -5
MVD_ERR_UNSUPPORTED = -6
MVD_ERR_ALLOC = -7
MVD_ERR_IO = -8

MVD_U16, MVD_F32 = 1, 2
MVD_STACK_ZYX, MVD_PLANES_YZX = 1, 2
BACK = {"flipped": 0, "efficient_bayes": 1, "opt1": 2, "opt2": 3, "explicit": 4}
UPDATE = {"simultaneous": 0, "sequential": 1}
BOUNDARY = {"zero": 0, "periodic": 1}
INIT = {"mean": 0, "given": 1, "const": 2}
MVD_FLAG_FORCE_2D = 0x1
MVD_FLAG_TIMING = 0x2
MVD_FLAG_GRAPH = 0x4
MVD_FLAG_TUNE = 0x8
MVD_FLAG_NORMALIZE = 0x10
MVD_DEVICE_NONE = -1
MVD_MAX_VIEWS = 8
MVD_MAX_K = 63
MVD_SCRATCH_BYTES = 64 << 20   # static scratch of mvd_deconvolve_planes_static (per GPU)


class MvdRun(ctypes.Structure):
    """Mirror of ``mvd_run``."""

    _fields_ = [
        ("struct_size", c_uint32),
        ("flags", c_uint32),
        ("n_planes", c_int32),
        ("n_iters", c_int32),
        ("update", c_int32),
        ("boundary", c_int32),
        ("init", c_int32),
        ("init_const", c_float),
        ("obs_dtype", c_int32),
        ("obs_layout", c_int32),
        ("view_weights", POINTER(c_float)),
        ("checkpoints", c_void_p),
        ("workspace", c_void_p),
        ("workspace_bytes", c_size_t),
        ("weight_planes", c_void_p),
    ]


class MvdTiming(ctypes.Structure):
    """Mirror of ``mvd_timing``."""

    _fields_ = [("struct_size", c_uint32), ("count", c_int32 * 6), ("ms", ctypes.c_double * 6)]


class MvdItem(ctypes.Structure):
    """Mirror of ``mvd_item``."""

    _fields_ = [("ctx", c_void_p), ("obs", POINTER(c_void_p)), ("est", c_void_p), ("run", POINTER(MvdRun))]


MVD_BATCH_TUNE = 0x1
MVD_BATCH_GRAPH = 0x2

MVD_FILES_SYNC = 0x1
MVD_FILES_DROP_CACHE = 0x2


class MvdFiles(ctypes.Structure):
    """Mirror of ``mvd_files``."""

    _fields_ = [
        ("struct_size", c_uint32),
        ("flags", c_uint32),
        ("obs_fd", c_int32 * MVD_MAX_VIEWS),
        ("obs_offset", ctypes.c_int64 * MVD_MAX_VIEWS),
        ("est_fd", c_int32),
        ("est_offset", ctypes.c_int64),
        ("host_slots", c_int32),
        ("io_threads", c_int32),
        ("seconds", ctypes.c_double * 4),
        ("bytes", ctypes.c_int64 * 2),
    ]


class MvdGrads(ctypes.Structure):
    """Mirror of ``mvd_grads``."""

    _fields_ = [
        ("struct_size", c_uint32),
        ("grad_psf", POINTER(c_void_p)),
        ("grad_back", POINTER(c_void_p)),
        ("grad_weights", c_void_p),
        ("grad_init", c_void_p),
        ("grad_weight_planes", POINTER(c_void_p)),
    ]


class MvdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"mvd status {status}: {message}")
        self.status = status


# name -> (restype, argtypes); the exported symbol set of include/mvd.h
SIGNATURES = {
    "mvd_version": (c_int, []),
    "mvd_status_string": (ctypes.c_char_p, [c_int]),
    "mvd_create": (c_int, [POINTER(c_void_p), c_int, c_int, c_int, c_int]),
    "mvd_destroy": (None, [c_void_p]),
    "mvd_set_psf": (c_int, [c_void_p, c_int, POINTER(c_float), c_int, c_int, c_int, POINTER(c_float)]),
    "mvd_get_back_taps": (c_int, [c_void_p, c_int, POINTER(c_float)]),
    "mvd_psf_info": (c_int, [c_void_p, c_int, POINTER(c_int), POINTER(c_int)]),
    "mvd_workspace_bytes": (c_int, [c_void_p, POINTER(MvdRun), POINTER(c_size_t)]),
    "mvd_reslice": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "mvd_deconvolve_planes": (c_int, [c_void_p, POINTER(c_void_p), c_void_p, POINTER(MvdRun), c_void_p]),
    "mvd_deconvolve_planes_static": (c_int, [c_void_p, POINTER(c_void_p), c_void_p, POINTER(MvdRun), c_void_p]),
    "mvd_get_timing": (c_int, [c_void_p, POINTER(MvdTiming), c_int]),
    "mvd_backward_workspace_bytes": (c_int, [c_void_p, POINTER(MvdRun), POINTER(c_size_t)]),
    "mvd_backward": (c_int, [c_void_p, POINTER(c_void_p), c_void_p, POINTER(MvdRun), POINTER(c_void_p),
                             POINTER(c_void_p), c_void_p, c_void_p, c_void_p]),
    "mvd_backward_grads": (c_int, [c_void_p, POINTER(c_void_p), c_void_p, POINTER(MvdRun), POINTER(MvdGrads),
                                   c_void_p]),
    "mvd_batch_create": (c_int, [POINTER(c_void_p), POINTER(MvdItem), c_int, c_uint32, c_void_p]),
    "mvd_batch_launch": (c_int, [c_void_p, c_void_p]),
    "mvd_batch_wait": (c_int, [c_void_p, c_void_p]),
    "mvd_batch_info": (c_int, [c_void_p, POINTER(c_int)]),
    "mvd_batch_form_times": (c_int, [c_void_p, POINTER(ctypes.c_double)]),
    "mvd_batch_tuning": (c_int, [c_void_p, c_int, POINTER(c_int)]),
    "mvd_batch_destroy": (None, [c_void_p]),
    "mvd_batch_run": (c_int, [POINTER(MvdItem), c_int, c_void_p]),
    "mvd_stream_workspace_bytes": (c_int, [c_void_p, POINTER(MvdRun), c_int, c_int, POINTER(c_size_t)]),
    "mvd_deconvolve_stream": (c_int, [c_void_p, POINTER(c_void_p), c_void_p, POINTER(MvdRun), c_int, c_void_p]),
    "mvd_deconvolve_files": (c_int, [c_void_p, POINTER(MvdFiles), POINTER(MvdRun), c_int, c_void_p]),
    "mvd_last_error": (ctypes.c_char_p, [c_void_p]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error(ctx) -> str:
    msg = lib().mvd_last_error(ctx)
    return msg.decode() if msg else ""


def check(status: int, ctx=None):
    if status != MVD_OK:
        raise MvdError(status, last_error(ctx))
    return status
