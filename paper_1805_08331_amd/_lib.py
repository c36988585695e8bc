"""ctypes declarations of the C ABI in include/pdsink.h.

Loading fails loudly when ``libpdsink.so`` has not been built: there is no
CPU fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PDSINK_PROFILE_BUILD=1 selects the instrumented build (phase cycle counters,
# python -m paper_1805_08331_amd.build --profile); it computes the same results.
LIB_NAME = "libpdsink_prof.so" if os.environ.get("PDSINK_PROFILE_BUILD") == "1" else "libpdsink.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)

c_int = ctypes.c_int
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_size = ctypes.c_size_t
c_vp = ctypes.c_void_p
c_char_p = ctypes.c_char_p


class Params(ctypes.Structure):
    """Mirror of ``pdsink_params``."""
    _fields_ = [
        ("d", c_i32),
        ("p", c_dbl),
        ("gamma", c_dbl),
        ("tol", c_dbl),
        ("max_iter", c_i32),
        ("precision", c_i32),
        ("switch_tol", c_dbl),
        ("kernel", c_i32),
    ]


PDSINK_OK = 0
PDSINK_EINVAL = -1
PDSINK_ENOMEM = -2
PDSINK_EDEVICE = -3
PDSINK_ERANGE = -4

PDSINK_KERNEL_AUTO = 0
PDSINK_KERNEL_RESIDENT = 1
PDSINK_KERNEL_GENERAL = 2

PDSINK_FP32 = 0
PDSINK_BF16_REFINE = 1

PDSINK_ST_MAX_ITER = 1
PDSINK_ST_NONFINITE = 2
PDSINK_ST_RANGE = 4
PDSINK_ST_LOG_PATH = 8

PDSINK_NOALLOC_SCRATCH_BYTES = 64 << 20
PDSINK_NOALLOC_MAX_PAIRS = 1 << 18

# pdsink_done: one pair's completion record (tag stored last by the device)
DONE_DTYPE = np.dtype([("cost", "<f8"), ("err", "<f4"), ("status", "<i4"), ("iters", "<i4", (2,)),
                       ("tag", "<u4"), ("reserved", "<u4")])
assert DONE_DTYPE.itemsize == 32

PDSINK_OP_DIST = 0
PDSINK_OP_KMEANS = 1
PDSINK_OP_BARYCENTER = 2
PDSINK_OP_DIST_WARM = 3

# name -> (restype, argtypes); every function declared in include/pdsink.h
SIGNATURES = {
    "pdsink_ctx_create": (c_int, [ctypes.POINTER(Params), c_int, ctypes.POINTER(c_vp)]),
    "pdsink_ctx_destroy": (None, [c_vp]),
    "pdsink_ctx_params": (c_int, [c_vp, ctypes.POINTER(Params)]),
    "pdsink_workspace_bytes": (c_int, [c_vp, c_int, c_i64, ctypes.POINTER(c_size)]),
    "pd_discretize": (c_int, [c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "pdsink_phase_profile": (c_int, [c_vp, c_int]),
    "sinkhorn_dist_batch": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                    c_vp, c_size, c_vp]),
    "sinkhorn_dist_batch_noalloc": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "sinkhorn_dist_batch_notify": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                           ctypes.c_uint32, c_vp, c_size, c_vp]),
    "sinkhorn_dist_bounds_batch": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                           c_vp, c_vp, c_vp, c_size, c_vp]),
    "pd_barycenter": (c_int, [c_vp, c_i64, c_vp, c_dbl, c_i32, c_dbl, c_i32, c_vp,
                              ctypes.POINTER(c_dbl), ctypes.POINTER(c_i32), c_vp, c_size, c_vp]),
    "pd_sharpen": (c_int, [c_vp, c_i64, c_vp, c_dbl, c_vp, c_vp]),
    "pd_quantize": (c_int, [c_vp, c_i64, c_vp, c_vp, c_vp]),
    "kmeans_assign": (c_int, [c_vp, c_i64, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]),
    "pdsink_lloyd_workspace_bytes": (c_int, [c_vp, c_i64, c_i32, ctypes.POINTER(c_size)]),
    "kmeans_lloyd": (c_int, [c_vp, c_i64, c_vp, c_i32, c_vp, c_i32, c_dbl, c_i32, c_dbl, c_vp, c_vp, c_vp,
                             c_vp, c_size, c_vp]),
    "pdsink_strerror": (c_char_p, [c_int]),
}

_LIB = None


def load():
    """Load libpdsink.so (once) and declare every exported function."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1805_08331_amd.build` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class PdsinkError(RuntimeError):
    def __init__(self, fn: str, code: int):
        msg = load().pdsink_strerror(code).decode()
        super().__init__(f"{fn} failed: {msg} ({code})")
        self.code = code


def check(fn: str, code: int):
    if code != PDSINK_OK:
        raise PdsinkError(fn, code)
