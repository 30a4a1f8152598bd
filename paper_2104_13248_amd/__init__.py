"""MI355X-native voxel-driven FDK back-projection (hot path of Chen et al., ICS'21).

Thin Python layer over ``libfdk.so`` (include/fdk.h).  Tensors are PyTorch
device tensors (HIP memory); work is enqueued on torch's current stream of the
tensors' device.  Host-side numpy arrays carry the 3x4 matrices and ellipsoid
tables.  All arithmetic happens in the library's HIP kernels.

Layouts: volume [nz, ny, nx] float32 (x fastest); projections [np, nh, nw]
(float32, or float16 with a per-view float32 scale); matrices [np, 3, 4]
float64 mapping world millimetres to (u w, v w, w).
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import (FDK_F16, FDK_F32, FdkError, EXPORTS, check, host_f64, lib, ptr,  # noqa: F401
                   stack_struct, volume_struct)

__all__ = ["FdkError", "backproject", "backproject_slab", "forwardproject", "fdk_filter",
           "quantize_f16", "circular_matrices", "scan_matrices", "phantom_project", "bp_plan"]


def _dev_ptr(t: torch.Tensor, name: str, dtypes, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device (HIP) tensor, got %s" % (name, t.device))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    if t.dtype not in dtypes:
        raise TypeError("%s must be one of %s, got %s" % (name, dtypes, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _mats(mats, np_views):
    m = host_f64(mats)
    if m.shape != (np_views, 3, 4):
        raise ValueError("mats must have shape [%d, 3, 4], got %s" % (np_views, m.shape))
    return m


def backproject(vol: torch.Tensor, proj: torch.Tensor, mats, voxel, centre=(0.0, 0.0, 0.0),
                scale: torch.Tensor | None = None) -> torch.Tensor:
    """vol += BP(proj) in place (Listings 1-2).  Returns ``vol``."""
    nz, ny, nx = vol.shape
    return backproject_slab(vol, (nz, ny, nx), 0, proj, mats, voxel, centre, scale)


def backproject_slab(vol_slab: torch.Tensor, shape, k_begin: int, proj: torch.Tensor, mats,
                     voxel, centre=(0.0, 0.0, 0.0), scale: torch.Tensor | None = None):
    """Back-project into slices [k_begin, k_begin + vol_slab.shape[0]) of a
    volume of ``shape``; bitwise equal to the same slices of a full call."""
    dev = vol_slab.device
    v = _dev_ptr(vol_slab, "vol", (torch.float32,))
    f16 = proj.dtype == torch.float16
    p = _dev_ptr(proj, "proj", (torch.float32, torch.float16), dev)
    s = None
    if f16:
        if scale is None:
            raise ValueError("float16 projections need a per-view scale")
        s = _dev_ptr(scale, "scale", (torch.float32,), dev)
        if tuple(scale.shape) != (proj.shape[0],):
            raise ValueError("scale must have shape [%d] (one per view), got %s"
                             % (proj.shape[0], tuple(scale.shape)))
    elif scale is not None:
        raise ValueError("scale is only accepted with float16 projections")
    npv, nh, nw = proj.shape
    if tuple(vol_slab.shape[1:]) != tuple(shape[1:]):
        raise ValueError("slab rows/columns do not match the volume shape")
    m = _mats(mats, npv)
    vg = volume_struct(shape, voxel, centre)
    sg = stack_struct(npv, nh, nw, FDK_F16 if f16 else FDK_F32)
    with torch.cuda.device(dev):
        check(lib.fdk_backproject_slab(vg, int(k_begin), int(vol_slab.shape[0]), v, sg, p, s,
                                       ptr(m), _stream(dev)))
    return vol_slab


def forwardproject(vol: torch.Tensor, proj: torch.Tensor, mats, voxel,
                   centre=(0.0, 0.0, 0.0)) -> torch.Tensor:
    """proj += A vol, the exact transpose of ``backproject``.  Returns ``proj``."""
    dev = vol.device
    v = _dev_ptr(vol, "vol", (torch.float32,))
    p = _dev_ptr(proj, "proj", (torch.float32,), dev)
    npv, nh, nw = proj.shape
    m = _mats(mats, npv)
    vg = volume_struct(vol.shape, voxel, centre)
    sg = stack_struct(npv, nh, nw, FDK_F32)
    with torch.cuda.device(dev):
        check(lib.fdk_forwardproject(vg, v, sg, p, ptr(m), _stream(dev)))
    return proj


def fdk_filter(raw: torch.Tensor, scan: dict, np_total: int | None = None,
               out: torch.Tensor | None = None, dtype=torch.float32,
               scale: torch.Tensor | None = None):
    """Cosine weight + Ram-Lak ramp + angular weight of raw line integrals.

    dtype float32: returns the filtered stack (``out`` if given).
    dtype float16: returns (binary16 stack, float32 per-view scale), the FP16
    storage rule applied by the filter itself (``out`` / ``scale`` if given)."""
    dev = raw.device
    r = _dev_ptr(raw, "raw", (torch.float32,))
    npv, nh, nw = raw.shape
    if dtype == torch.float32:
        if scale is not None:
            raise ValueError("scale is only written with float16 output")
        if out is None:
            out = torch.empty_like(raw)
        code, sp = FDK_F32, None
    elif dtype == torch.float16:
        if out is None:
            out = torch.empty(raw.shape, dtype=torch.float16, device=dev)
        if scale is None:
            scale = torch.empty(npv, dtype=torch.float32, device=dev)
        if tuple(scale.shape) != (npv,):
            raise ValueError("scale must have shape [%d], got %s" % (npv, tuple(scale.shape)))
        code, sp = FDK_F16, _dev_ptr(scale, "scale", (torch.float32,), dev)
    else:
        raise TypeError("dtype must be torch.float32 or torch.float16")
    o = _dev_ptr(out, "out", (dtype,), dev)
    if tuple(out.shape) != tuple(raw.shape):
        raise ValueError("out must have the shape of raw")
    sg = stack_struct(npv, nh, nw)
    with torch.cuda.device(dev):
        check(lib.fdk_filter(sg, r, code, o, sp, scan["du"], scan["dv"], scan["sod"], scan["sdd"],
                             scan["u_off"], scan["v_off"], scan["arc"],
                             int(np_total if np_total is not None else npv), _stream(dev)))
    return out if dtype == torch.float32 else (out, scale)


def quantize_f16(proj: torch.Tensor):
    """float32 stack -> (float16 stack, float32 per-view scale), bit-exact rule."""
    dev = proj.device
    p = _dev_ptr(proj, "proj", (torch.float32,))
    npv, nh, nw = proj.shape
    h = torch.empty(proj.shape, dtype=torch.float16, device=dev)
    sc = torch.empty(npv, dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(lib.fdk_quantize_f16(npv, nh, nw, p, h.data_ptr(), sc.data_ptr(), _stream(dev)))
    return h, sc


def circular_matrices(np_views, arc, theta0, sod, sdd, nh, nw, du, dv, u_off=0.0, v_off=0.0):
    """Matrices of a circular orbit (host, FP64): [np, 3, 4]."""
    out = np.zeros((int(np_views), 3, 4), dtype=np.float64)
    check(lib.fdk_circular_matrices(int(np_views), float(arc), float(theta0), float(sod),
                                    float(sdd), int(nh), int(nw), float(du), float(dv),
                                    float(u_off), float(v_off), ptr(out)))
    return out


def scan_matrices(scan: dict, np_views: int, nh: int, nw: int):
    return circular_matrices(np_views, scan["arc"], scan["theta0"], scan["sod"], scan["sdd"],
                             nh, nw, scan["du"], scan["dv"], scan["u_off"], scan["v_off"])


def phantom_project(ell, scan: dict, proj: torch.Tensor, view_begin: int = 0,
                    np_total: int | None = None) -> torch.Tensor:
    """proj += analytic line integrals of the ellipsoid rows ``ell`` ([n, 16])."""
    dev = proj.device
    p = _dev_ptr(proj, "proj", (torch.float32,))
    e = host_f64(ell).reshape(-1, 16)
    npv, nh, nw = proj.shape
    sg = stack_struct(npv, nh, nw)
    with torch.cuda.device(dev):
        check(lib.fdk_phantom_project(ptr(e), int(e.shape[0]), sg, p, scan["arc"],
                                      scan["theta0"], scan["sod"], scan["sdd"], scan["du"],
                                      scan["dv"], scan["u_off"], scan["v_off"], int(view_begin),
                                      int(np_total if np_total is not None else npv),
                                      _stream(dev)))
    return proj


def bp_plan(shape, voxel, np_views, nh, nw, mats, centre=(0.0, 0.0, 0.0), f16=False) -> dict:
    """Launch configuration the back-projector would choose (host only)."""
    import ctypes
    out = (ctypes.c_int64 * 12)()
    m = _mats(mats, np_views)
    check(lib.fdk_bp_plan(volume_struct(shape, voxel, centre),
                          stack_struct(np_views, nh, nw, FDK_F16 if f16 else FDK_F32), ptr(m),
                          ctypes.cast(out, ctypes.c_void_p)))
    keys = ("tile_x", "tile_y", "kz", "lds_pitch", "lds_rows", "lds_bytes", "blocks", "threads",
            "rows_full", "fp_lds_bytes", "fp_rows", "fp_cols")
    return dict(zip(keys, [int(x) for x in out]))
