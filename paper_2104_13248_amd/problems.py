"""Back-projection throughput on the paper's problem sizes (Table 3):
P1..P10 = {256^2, 512^2, 1024^2} x 512 views => {256^3, 512^3, 1024^3}, and
P10 = 1024^2 x 512 => 1300^3 (8.2 GiB of volume).

The paper does not state its scan geometry (RTK forward projections of the
RabbitCT volume).  Reading used here: the circular orbit of the 512^3
benchmark (SOD 750 mm, SDD 1200 mm) with a fixed 512 mm field of view and a
1024 mm detector, so a problem n_det^2 => n_vox^3 has voxel 512/n_vox mm and
pixel 1024/n_det mm (magnification 0.8 n_det / n_vox pixels per voxel).
Seeded standard-normal projections (content does not change the
arithmetic); float32 storage and binary16 storage.

    python -m paper_2104_13248_amd.problems [--only P5,P10]

prints one JSON line per problem and storage with ms and GUPS (HIP events).
"""
from __future__ import annotations

import argparse
import json
import sys

import torch

from . import backproject, bp_plan, circular_matrices, quantize_f16

PROBLEMS = {
    "P1": (256, 256), "P2": (256, 512), "P3": (256, 1024),
    "P4": (512, 256), "P5": (512, 512), "P6": (512, 1024),
    "P7": (1024, 256), "P8": (1024, 512), "P9": (1024, 1024),
    "P10": (1024, 1300),
}
VIEWS = 512
FOV_MM = 512.0
DET_MM = 1024.0
SOD, SDD = 750.0, 1200.0


def geometry(name: str):
    """(shape, voxel, mats, nh, nw) of problem ``name``."""
    ndet, nvox = PROBLEMS[name]
    voxel = FOV_MM / nvox
    pix = DET_MM / ndet
    mats = circular_matrices(VIEWS, 2 * 3.141592653589793, 0.0, SOD, SDD, ndet, ndet, pix, pix)
    return (nvox, nvox, nvox), (voxel, voxel, voxel), mats, ndet, ndet


def run(names, reps: int = 2, out=sys.stdout):
    rows = []
    for name in names:
        shape, voxel, mats, nh, nw = geometry(name)
        g = torch.Generator(device="cuda")
        g.manual_seed(9000 + int(name[1:]))
        proj = torch.randn((VIEWS, nh, nw), generator=g, device="cuda")
        h, s = quantize_f16(proj)
        vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
        n_upd = vol.numel() * VIEWS
        for storage in ("f32", "f16"):
            def call():
                if storage == "f32":
                    backproject(vol, proj, mats, voxel)
                else:
                    backproject(vol, h, mats, voxel, scale=s)
            call()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                call()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            plan = bp_plan(shape, voxel, VIEWS, nh, nw, mats, f16=storage == "f16")
            r = {"problem": name, "detector": nh, "volume": shape[0], "views": VIEWS,
                 "storage": storage, "ms": ms, "gups": n_upd / (ms * 1e-3) / 1e9,
                 "kz": plan["kz"], "lds_pitch": plan["lds_pitch"], "lds_rows": plan["lds_rows"]}
            rows.append(r)
            print(json.dumps(r), file=out, flush=True)
        del vol, proj, h, s
        torch.cuda.empty_cache()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description="back-projection on the paper's problem sizes")
    ap.add_argument("--only", default=None, help="comma-separated problem labels")
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    names = a.only.split(",") if a.only else list(PROBLEMS)
    run(names, a.reps)


if __name__ == "__main__":
    main()
