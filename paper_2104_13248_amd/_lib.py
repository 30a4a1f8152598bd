"""ctypes binding of libfdk.so (include/fdk.h, fdk_learn.h, fdk_ablation.h):
argument marshalling only.

Every operation runs in the HIP kernels of the library; this module checks
tensor placement, dtype and contiguity, passes raw device pointers and the
current HIP stream, and turns status codes into ``FdkError``.  There is no
fallback: if the library is missing, importing the package fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# FDK_LIBRARY may name another build of the same library (e.g. a tuning build)
LIB_PATH = os.environ.get("FDK_LIBRARY") or os.path.join(_PKG, "libfdk.so")

FDK_F32 = 0
FDK_F16 = 1


class FdkError(RuntimeError):
    """Non-OK status from the library; ``code`` is the fdk_status value."""

    def __init__(self, code: int, message: str):
        super().__init__("fdk status %d: %s" % (code, message))
        self.code = code


class Volume(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double)]


class Stack(ctypes.Structure):
    _fields_ = [("np", ctypes.c_int32), ("nh", ctypes.c_int32), ("nw", ctypes.c_int32),
                ("dtype", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfdk.so not built: run `python paper_2104_13248_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int32
    D = ctypes.c_double
    F = ctypes.c_float
    VP = ctypes.POINTER(Volume)
    SP = ctypes.POINTER(Stack)
    sigs = {
        "fdk_backproject": [VP, P, SP, P, P, P, P],
        "fdk_backproject_slab": [VP, I, I, P, SP, P, P, P, P],
        "fdk_backproject_noalloc": [VP, P, SP, P, P, P, P],
        "fdk_forwardproject": [VP, P, SP, P, P, P],
        "fdk_filter": [SP, P, I, P, P, D, D, D, D, D, D, D, I, P],
        "fdk_quantize_f16": [I, I, I, P, P, P, P],
        "fdk_circular_matrices": [I, D, D, D, D, I, I, D, D, D, D, P],
        "fdk_phantom_project": [P, I, SP, P, D, D, D, D, D, D, D, D, I, I, P],
        "fdk_bp_plan": [VP, SP, P, P],
        # include/fdk_learn.h
        "fdk_cosine_weight": [SP, P, P, D, D, D, D, D, P],
        "fdk_conv1d_forward": [I, I, I, I, P, P, P, P, P, F, I, P, P],
        "fdk_conv1d_backward_data": [I, I, I, I, P, P, P, P, P],
        "fdk_conv1d_backward_weight": [I, I, I, I, P, P, P, P, P],
        "fdk_sqerr": [ctypes.c_int64, P, P, P, F, P, P],
        "fdk_adam": [I, P, P, P, P, F, F, F, F, I, P],
        # include/fdk_ablation.h
        "fdk_backproject_variant": [I, I, VP, P, SP, P, P, P],
        # include/fdk_peaks.h
        "fdk_peak_hbm_read": [P, ctypes.c_int64, I, P, P],
        "fdk_peak_lds_read": [I, I, I, P, P, P],
        "fdk_peak_valu_fma": [I, I, P, P, P],
        "fdk_peak_valu_op": [I, I, I, P, P, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.fdk_last_error.restype = ctypes.c_char_p
    lib.fdk_last_error.argtypes = []
    lib.fdk_status_string.restype = ctypes.c_char_p
    lib.fdk_status_string.argtypes = [ctypes.c_int]
    return lib


lib = _load()

#: names declared in include/fdk.h, include/fdk_learn.h and include/fdk_ablation.h
EXPORTS = ("fdk_backproject", "fdk_backproject_slab", "fdk_backproject_noalloc",
           "fdk_forwardproject", "fdk_filter",
           "fdk_quantize_f16", "fdk_circular_matrices", "fdk_phantom_project", "fdk_bp_plan",
           "fdk_last_error", "fdk_status_string",
           "fdk_cosine_weight", "fdk_conv1d_forward", "fdk_conv1d_backward_data",
           "fdk_conv1d_backward_weight", "fdk_sqerr", "fdk_adam",
           "fdk_backproject_variant",
           "fdk_peak_hbm_read", "fdk_peak_lds_read", "fdk_peak_valu_fma",
           "fdk_peak_valu_op")


def check(code: int) -> None:
    if code != 0:
        msg = lib.fdk_last_error().decode() or lib.fdk_status_string(code).decode()
        raise FdkError(code, msg)


def volume_struct(shape, voxel, centre=(0.0, 0.0, 0.0)) -> Volume:
    nz, ny, nx = (int(n) for n in shape)
    return Volume(nx, ny, nz, float(voxel[0]), float(voxel[1]), float(voxel[2]),
                  float(centre[0]), float(centre[1]), float(centre[2]))


def stack_struct(np_views, nh, nw, dtype=FDK_F32) -> Stack:
    return Stack(int(np_views), int(nh), int(nw), int(dtype))


def host_f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)
