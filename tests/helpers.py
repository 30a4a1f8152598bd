"""Shared helpers for the parity tests (no arithmetic of the method here)."""
import functools
import time

import numpy as np

import oracle
from oracle import geometry as og
from oracle import phantom as oph
import workloads as wl


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def log(*args):
    print("[%s]" % time.strftime("%H:%M:%S"), *args, flush=True)


@functools.lru_cache(maxsize=4)
def c1_filtered(index: int = 0):
    """Ramp-filtered analytic projections of C1 phantom ``index`` (oracle side):
    float32 [64, 128, 128] and the world matrices."""
    cfg = wl.CONFIGS["c1"]
    ell = wl.config_ellipsoids(cfg, index)
    raw = oph.line_integrals(ell, cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    filt = oracle.fdk_filter(raw, cfg["scan"]).astype(np.float32)
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    return filt, mats


def subblocks(shape, b=64):
    """Eight b^3 boxes ((k0,k1),(j0,j1),(i0,i1)) of a [nz,ny,nx] volume: the
    centre, four corners and three edge midpoints."""
    nz, ny, nx = shape

    def at(n, where):
        b_ = min(b, n)
        return {"lo": 0, "mid": n // 2 - b_ // 2, "hi": n - b_}[where], b_

    out = []
    for kw, jw, iw in (("mid", "mid", "mid"), ("lo", "lo", "lo"), ("hi", "lo", "hi"),
                       ("lo", "hi", "hi"), ("hi", "hi", "lo"), ("mid", "lo", "lo"),
                       ("lo", "mid", "hi"), ("hi", "hi", "mid")):
        (k0, bk), (j0, bj), (i0, bi) = at(nz, kw), at(ny, jw), at(nx, iw)
        out.append(((k0, k0 + bk), (j0, j0 + bj), (i0, i0 + bi)))
    return out


def gpu_phantom_stacks(cfg, index=0, chunk=64):
    """The benchmark's input recipe, on the GPU: analytic line integrals of
    phantom ``index`` of a workload, FDK-filtered into a float32 stack and,
    by the same filter call with binary16 output, into binary16 codes + one
    scale per view.  Returns (filt, h, scale, mats) as device tensors and
    host matrices."""
    import torch
    import paper_2104_13248_amd as fdk
    npv, nh, nw, scan = cfg["np"], cfg["nh"], cfg["nw"], cfg["scan"]
    ell = wl.config_ellipsoids(cfg, index)
    filt = torch.empty((npv, nh, nw), dtype=torch.float32, device="cuda")
    h = torch.empty((npv, nh, nw), dtype=torch.float16, device="cuda")
    sc = torch.empty(npv, dtype=torch.float32, device="cuda")
    raw = torch.empty((min(chunk, npv), nh, nw), dtype=torch.float32, device="cuda")
    for v0 in range(0, npv, chunk):
        n = min(chunk, npv - v0)
        raw[:n].zero_()
        fdk.phantom_project(ell, scan, raw[:n], view_begin=v0, np_total=npv)
        fdk.fdk_filter(raw[:n], scan, np_total=npv, out=filt[v0:v0 + n])
        fdk.fdk_filter(raw[:n], scan, np_total=npv, out=h[v0:v0 + n], dtype=torch.float16,
                       scale=sc[v0:v0 + n])
    torch.cuda.synchronize()
    del raw
    mats = og.scan_matrices(scan, npv, nh, nw)
    return filt, h, sc, mats


def subblock_errors(cfg, mats, filt, h, sc, vol32, vol16, boxes=None):
    """rel-L2 over the union of sub-blocks of two GPU volumes (float32- and
    binary16-storage back-projections of ``filt`` and ``h``/``sc``) against
    the FP64 oracle, which reads only each view's detector window of the same
    device stacks: f32 vs oracle(float32 stack), f16 vs oracle(float32 stack),
    f16 vs oracle(dequantised binary16 stack)."""
    from oracle import window as ow
    shape, voxel = cfg["shape"], cfg["voxel"]
    nh, nw = cfg["nh"], cfg["nw"]
    sc_h = sc.cpu().numpy()
    acc = dict(e32=0.0, r32=0.0, e16=0.0, e16d=0.0, r16=0.0)
    for box in boxes or subblocks(shape):
        (k0, k1), (j0, j1), (i0, i1) = box
        origin, wr, wc = ow.block_windows(mats, shape, voxel, box)
        w32 = ow.cut_windows_device(filt, origin, wr, wc)
        w16 = ow.cut_windows_device(h, origin, wr, wc)
        ref32 = oracle.backproject_block(w32, mats, shape, voxel, box, origin=origin,
                                         detector=(nh, nw))
        ref16 = oracle.backproject_block(w16, mats, shape, voxel, box, scale=sc_h, origin=origin,
                                         detector=(nh, nw))
        g32 = vol32[k0:k1, j0:j1, i0:i1].double().cpu().numpy()
        g16 = vol16[k0:k1, j0:j1, i0:i1].double().cpu().numpy()
        acc["e32"] += float(((g32 - ref32) ** 2).sum())
        acc["r32"] += float((ref32 ** 2).sum())
        acc["e16"] += float(((g16 - ref32) ** 2).sum())
        acc["e16d"] += float(((g16 - ref16) ** 2).sum())
        acc["r16"] += float((ref16 ** 2).sum())
        log("block", box, "window", wr, wc, "block rel-L2 f32 %.2e f16 %.2e"
            % (rel(g32, ref32), rel(g16, ref32)))
    return {"f32": (acc["e32"] / acc["r32"]) ** 0.5, "f16": (acc["e16"] / acc["r32"]) ** 0.5,
            "f16_dequantised": (acc["e16d"] / acc["r16"]) ** 0.5}


def whole_rel(a, b):
    """rel-L2 of two device volumes of the same shape, in float64 slabs."""
    num = den = 0.0
    for k0 in range(0, a.shape[0], 64):
        x = a[k0:k0 + 64].double()
        y = b[k0:k0 + 64].double()
        num += float(((x - y) ** 2).sum())
        den += float((y ** 2).sum())
    return (num / den) ** 0.5
