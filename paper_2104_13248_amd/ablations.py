"""The paper's CPU optimisations measured on the GPU (include/fdk_ablation.h).

Variants of the same back-projection (float32 projections):

* ``production`` with ``nb`` < np: the production kernel called once per
  batch of nb views, so the volume is read and written np/nb times -- the
  batching of Section 3.1.3 (the paper's Fig. 6 sweeps nb = 1 .. 32);
* ``global_taps``: hoisting and register accumulation kept, the LDS window
  of Section 3.2 removed (taps read from global memory);
* ``listing1``: Listing 1 as a GPU kernel (thread per voxel, full
  projection per (voxel, view), taps from global memory), with the volume
  updated once per batch of nb views;
* ``symmetry``: the geometric symmetry of Section 3.1.2 (slices k and
  nz-1-k share v's row, fraction and LDS address);
* ``subline``: the sub-line interpolation of Section 3.1.5 (two detector
  columns blended once per (column, view) into an LDS line, one 1-D
  interpolation per update).

    python -m paper_2104_13248_amd.ablations [--config c2] [--views N]

prints one JSON line per (variant, nb) with milliseconds and GUPS, timed with
HIP events on the current stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import torch

from . import backproject, scan_matrices
from ._lib import FDK_F32, FdkError, check, host_f64, lib, ptr, stack_struct, volume_struct

VARIANTS = {"production": 0, "global_taps": 1, "listing1": 2, "symmetry": 3, "subline": 4}


def backproject_variant(vol: torch.Tensor, proj: torch.Tensor, mats, voxel, variant: str,
                        nb: int | None = None, centre=(0.0, 0.0, 0.0)) -> torch.Tensor:
    """vol += BP(proj) with the given kernel organisation (see module doc)."""
    if proj.dtype != torch.float32 or vol.dtype != torch.float32:
        raise TypeError("variants take float32 volumes and projections")
    if not (vol.is_cuda and proj.is_cuda and vol.is_contiguous() and proj.is_contiguous()):
        raise ValueError("vol and proj must be contiguous device tensors")
    npv, nh, nw = proj.shape
    m = host_f64(mats)
    if m.shape != (npv, 3, 4):
        raise ValueError("mats must have shape [np, 3, 4]")
    vg = volume_struct(vol.shape, voxel, centre)
    sg = stack_struct(npv, nh, nw, FDK_F32)
    dev = vol.device
    with torch.cuda.device(dev):
        check(lib.fdk_backproject_variant(VARIANTS[variant], int(nb if nb else npv), vg,
                                          vol.data_ptr(), sg, proj.data_ptr(), ptr(m),
                                          torch.cuda.current_stream(dev).cuda_stream))
    return vol


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def sweep(config: str = "c2", views: int | None = None, nbs=(1, 2, 4, 8, 16, 32, 64, 256),
          reps: int = 2, out=sys.stdout):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import workloads as wl       # seeded shapes only

    cfg = wl.CONFIGS[config]
    npv = int(views or cfg["np"])
    nh, nw = cfg["nh"], cfg["nw"]
    mats = scan_matrices(cfg["scan"], npv, nh, nw)
    g = torch.Generator(device="cuda")
    g.manual_seed(cfg["seed"] + 77)
    proj = torch.randn((npv, nh, nw), generator=g, device="cuda")
    vol = torch.zeros(cfg["shape"], dtype=torch.float32, device="cuda")
    n_upd = vol.numel() * npv
    rows = []

    def emit(variant, nb, ms):
        r = {"config": config, "views": npv, "variant": variant, "nb": nb, "ms": ms,
             "gups": n_upd / (ms * 1e-3) / 1e9}
        rows.append(r)
        print(json.dumps(r), file=out, flush=True)

    emit("production", npv, _time(lambda: backproject(vol, proj, mats, cfg["voxel"]), reps))
    emit("symmetry", npv, _time(lambda: backproject_variant(vol, proj, mats, cfg["voxel"],
                                                            "symmetry"), reps))
    emit("subline", npv, _time(lambda: backproject_variant(vol, proj, mats, cfg["voxel"],
                                                           "subline"), reps))
    emit("global_taps", npv, _time(lambda: backproject_variant(vol, proj, mats, cfg["voxel"],
                                                               "global_taps"), reps))
    for nb in nbs:
        if nb >= npv:
            continue
        emit("production", nb, _time(lambda: backproject_variant(vol, proj, mats, cfg["voxel"],
                                                                 "production", nb), reps))
    for nb in nbs:
        if nb > npv:
            continue
        emit("listing1", nb, _time(lambda: backproject_variant(vol, proj, mats, cfg["voxel"],
                                                               "listing1", nb), 1))
    return rows


def compare_problem(name: str, reps: int = 2, out=sys.stdout):
    """Production against the sub-line, symmetric and global-taps
    organisations on one of the paper's problem sizes (Table 3; geometry
    reading of problems.py)."""
    from . import problems
    shape, voxel, mats, nh, nw = problems.geometry(name)
    npv = problems.VIEWS
    g = torch.Generator(device="cuda")
    g.manual_seed(9100 + int(name[1:]))
    proj = torch.randn((npv, nh, nw), generator=g, device="cuda")
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    n_upd = vol.numel() * npv
    rows = []
    for variant in ("production", "subline", "symmetry", "global_taps"):
        fn = (lambda: backproject(vol, proj, mats, voxel)) if variant == "production" else \
            (lambda: backproject_variant(vol, proj, mats, voxel, variant))
        r = {"problem": name, "detector": nh, "volume": shape[0], "views": npv,
             "variant": variant}
        try:
            ms = _time(fn, reps)
            r.update(ms=ms, gups=n_upd / (ms * 1e-3) / 1e9)
        except FdkError as e:           # e.g. window and lines beyond the LDS
            r.update(unsupported=str(e))
        rows.append(r)
        print(json.dumps(r), file=out, flush=True)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description="back-projection ablations on one GPU")
    ap.add_argument("--config", default="c2")
    ap.add_argument("--views", type=int, default=None, help="views (default: the workload's)")
    ap.add_argument("--problem", default=None,
                    help="comma-separated problems of Table 3 (P1..P10): production, sub-line, "
                         "symmetric and global-taps organisations only")
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if a.problem:
        for name in a.problem.split(","):
            compare_problem(name, a.reps)
        return
    sweep(a.config, a.views, reps=a.reps)


if __name__ == "__main__":
    main()
