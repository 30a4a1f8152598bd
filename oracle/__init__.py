"""FP64 CPU oracle for voxel-driven FDK back-projection.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  The product library never imports,
links or calls anything here, and nothing here imports the product package.

The arithmetic lives in ``oracle.c`` (plain C, double precision, OpenMP over
the voxels); this module only marshals numpy arrays into
it.  ``geometry.py`` holds the closed-form circular-orbit matrices and
``quantize.py`` the FP16 storage rule.  Each function names the passage of
Chen et al., ICS'21 ("Performance Portable Back-projection Algorithms on
CPUs") that it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from .geometry import circular_matrices, index_matrices  # noqa: F401
from .quantize import quantize_f16, dequantize_f16  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_I64 = ctypes.c_int64
_D = ctypes.c_double
_P = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc (-O3, OpenMP, no fast-math)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-Wall",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            # ORACLE_LIBRARY: another build of oracle.c (e.g. with sanitizers)
            path = os.environ.get("ORACLE_LIBRARY")
            if not path:
                build()
                path = _SO
            lib = ctypes.CDLL(path)
            vol = [_I64] * 3 + [_D] * 6
            stk = [_I64] * 3 + [_P] * 3
            lib.oracle_bp.argtypes = vol + stk + [_P, _P, ctypes.c_int]
            lib.oracle_bp_points.argtypes = vol + stk + [_P, _I64, _P, _P, ctypes.c_int]
            lib.oracle_bp_block.argtypes = (vol + [_I64] * 5 + [_P] + [_P] * 3 + [_P] + [_I64] * 6
                                            + [_P, ctypes.c_int])
            lib.oracle_bp_hoisted.argtypes = vol + stk + [_P, _P, ctypes.c_int]
            lib.oracle_bp_geometry.argtypes = vol + stk + [_D] * 8 + [_P, ctypes.c_int]
            lib.oracle_project_points.argtypes = [_D] * 5 + [_I64, _I64, _D, _D, _I64, _P, _P]
            lib.oracle_fp.argtypes = vol + [_I64] * 3 + [_P, _P, _P, ctypes.c_int]
            lib.oracle_filter.argtypes = [_I64] * 3 + [_P, _P] + [_D] * 7 + [_I64, ctypes.c_int]
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _vol_args(shape, voxel, centre):
    nz, ny, nx = shape
    dx, dy, dz = voxel
    cx, cy, cz = centre
    return [int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
            float(cx), float(cy), float(cz)]


def _stack_args(proj, scale):
    """proj: float32 [np,nh,nw], or float16 [np,nh,nw] with float32 scale [np]."""
    if proj.dtype == np.float32:
        p32, p16, sc = np.ascontiguousarray(proj), None, None
    elif proj.dtype == np.float16:
        if scale is None:
            raise ValueError("float16 projections need a per-view scale")
        p32 = None
        p16 = np.ascontiguousarray(proj).view(np.uint16)
        sc = np.ascontiguousarray(scale, dtype=np.float32)
    else:
        raise TypeError("projections must be float32 or float16")
    npv, nh, nw = proj.shape
    keep = (p32, p16, sc)
    return [int(npv), int(nh), int(nw), _ptr(p32), _ptr(p16), _ptr(sc)], keep


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def backproject(proj, mats, shape, voxel, centre=(0.0, 0.0, 0.0), scale=None,
                vol=None, threads=0):
    """vol[nz,ny,nx] += sum_s p_s(u, v) / w^2 (Section 2.1.2), FP64; p_s(u, v)
    is the tent-weighted (bilinear) value of view s, zero off the detector.

    ``mats`` are world-mm 3x4 matrices [np,3,4] applied to voxel centres.
    Returns the float64 volume (a new zero volume unless ``vol`` is given)."""
    lib = _load()
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    if vol is None:
        vol = np.zeros(shape, dtype=np.float64)
    assert vol.dtype == np.float64 and vol.flags.c_contiguous and vol.shape == tuple(shape)
    stk, keep = _stack_args(proj, scale)
    lib.oracle_bp(*_vol_args(shape, voxel, centre), *stk, _ptr(mats), _ptr(vol), int(threads))
    del keep
    return vol


def backproject_points(proj, mats, shape, voxel, ijk, centre=(0.0, 0.0, 0.0),
                       scale=None, threads=0):
    """Back-projected value of the voxels listed in ``ijk`` ([n,3] as i,j,k)."""
    lib = _load()
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    ijk = np.ascontiguousarray(ijk, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(len(ijk), dtype=np.float64)
    stk, keep = _stack_args(proj, scale)
    lib.oracle_bp_points(*_vol_args(shape, voxel, centre), *stk, _ptr(mats),
                         int(len(ijk)), _ptr(ijk), _ptr(out), int(threads))
    del keep
    return out


def backproject_block(proj, mats, shape, voxel, box, centre=(0.0, 0.0, 0.0),
                      scale=None, threads=0, origin=None, detector=None):
    """Back-projection of the sub-block box = ((k0,k1),(j0,j1),(i0,i1)).

    ``proj`` holds whole views ([np,nh,nw]), or, with ``origin`` ([np,2] int:
    first detector row and column of each view's window) and ``detector``
    ((nh, nw)), only a window of each view ([np,wr,wc]).  A window must hold
    every detector pixel the block's voxels reach; if one does not, this
    raises instead of returning an incomplete sum."""
    lib = _load()
    (k0, k1), (j0, j1), (i0, i1) = box
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    out = np.zeros((k1 - k0, j1 - j0, i1 - i0), dtype=np.float64)
    stk, keep = _stack_args(proj, scale)
    npv, wr, wc = stk[0], stk[1], stk[2]
    if origin is None:
        nh, nw, org = wr, wc, None
    else:
        nh, nw = (int(n) for n in detector)
        org = np.ascontiguousarray(origin, dtype=np.int64).reshape(npv, 2)
    miss = lib.oracle_bp_block(*_vol_args(shape, voxel, centre), npv, nh, nw, wr, wc,
                               _ptr(org), *stk[3:], _ptr(mats),
                               int(i0), int(i1), int(j0), int(j1), int(k0), int(k1),
                               _ptr(out), int(threads))
    del keep
    if miss:
        raise ValueError("a voxel of the block reaches a detector pixel outside its view's window")
    return out


def backproject_hoisted(proj, mats, shape, voxel, centre=(0.0, 0.0, 0.0), scale=None,
                        threads=0):
    """u and w computed once per voxel column and view (Section 3.1.2)."""
    lib = _load()
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    vol = np.zeros(shape, dtype=np.float64)
    stk, keep = _stack_args(proj, scale)
    lib.oracle_bp_hoisted(*_vol_args(shape, voxel, centre), *stk, _ptr(mats), _ptr(vol),
                          int(threads))
    del keep
    return vol


def backproject_geometry(proj, shape, voxel, scan, centre=(0.0, 0.0, 0.0), scale=None,
                         threads=0):
    """Geometry mode: (u, v, w) by ray/plane intersection, no matrices.

    ``scan`` holds arc, theta0, sod, sdd, du, dv, u_off, v_off."""
    lib = _load()
    vol = np.zeros(shape, dtype=np.float64)
    stk, keep = _stack_args(proj, scale)
    g = [float(scan[k]) for k in ("arc", "theta0", "sod", "sdd", "du", "dv", "u_off", "v_off")]
    lib.oracle_bp_geometry(*_vol_args(shape, voxel, centre), *stk, *g, _ptr(vol), int(threads))
    del keep
    return vol


def project_points(theta, scan, nh, nw, xyz):
    """(u, v, w) of world points [n,3] for one view angle, geometry mode."""
    lib = _load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    out = np.zeros_like(xyz)
    lib.oracle_project_points(float(theta), float(scan["sod"]), float(scan["sdd"]),
                              float(scan["du"]), float(scan["dv"]), int(nh), int(nw),
                              float(scan["u_off"]), float(scan["v_off"]), int(len(xyz)),
                              _ptr(xyz), _ptr(out))
    return out


def forwardproject(vol, mats, nh, nw, voxel, centre=(0.0, 0.0, 0.0), proj=None, threads=0):
    """Exact transpose of ``backproject``: proj[np,nh,nw] += A^T-adjoint splat."""
    lib = _load()
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    npv = mats.shape[0]
    if proj is None:
        proj = np.zeros((npv, nh, nw), dtype=np.float64)
    assert proj.dtype == np.float64 and proj.flags.c_contiguous
    lib.oracle_fp(*_vol_args(vol.shape, voxel, centre), int(npv), int(nh), int(nw),
                  _ptr(vol), _ptr(mats), _ptr(proj), int(threads))
    return proj


def fdk_filter(raw, scan, np_total=None, threads=0):
    """Cosine weight + Ram-Lak ramp (zero-padded linear convolution) + angular
    quadrature weight, per detector row, FP64.  ``raw``: [np,nh,nw]."""
    lib = _load()
    raw = np.ascontiguousarray(raw, dtype=np.float64)
    npv, nh, nw = raw.shape
    out = np.zeros_like(raw)
    if np_total is None:
        np_total = npv
    lib.oracle_filter(int(npv), int(nh), int(nw), _ptr(raw), _ptr(out),
                      float(scan["du"]), float(scan["dv"]), float(scan["sod"]),
                      float(scan["sdd"]), float(scan["u_off"]), float(scan["v_off"]),
                      float(scan["arc"]), int(np_total), int(threads))
    return out
