"""Train the learned row filter for sparse-view FDK and compare it with the
ramp filter.

Workload (defaults): 256^3 volume of 0.25 mm voxels, 512^2 detector of
0.25 mm pixels, source-isocentre 500 mm, source-detector 1000 mm; 90-view
scans of seeded random-ellipsoid phantoms (10 ellipsoids each), trained against
720-view ramp-filter FDK reconstructions of the same phantoms.  Every scan,
target and training step runs on the GPU through libfdk.so.

    python -m paper_2104_13248_amd.train_learned --phantoms 2000 --epochs 1

Prints one JSON line per log interval and a final summary line with the
held-out relative L2 error of both filters against the dense-view targets and
the throughput of the learned sparse-view reconstruction.  --checkpoint saves
parameters, Adam state and the position in the data stream; --resume
continues from it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import torch

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import workloads as wl  # noqa: E402  (seeded phantom tables only)

from . import backproject, fdk_filter, phantom_project, scan_matrices  # noqa: E402
from .autograd import Geometry  # noqa: E402
from .learned import LearnedFilter, cosine_weight  # noqa: E402


class Data:
    """Sparse-view scans and dense-view FDK targets of seeded phantoms."""

    def __init__(self, cfg: dict, views: int, target_views: int, device):
        self.cfg = cfg
        self.scan = cfg["scan"]
        self.dev = device
        nh, nw = cfg["nh"], cfg["nw"]
        self.sparse = Geometry(cfg["shape"], cfg["voxel"],
                               scan_matrices(self.scan, views, nh, nw), nh, nw)
        self.dense = Geometry(cfg["shape"], cfg["voxel"],
                              scan_matrices(self.scan, target_views, nh, nw), nh, nw)
        self.views, self.target_views = views, target_views

    def scan_of(self, index: int, views: int) -> torch.Tensor:
        ell = wl.config_ellipsoids(self.cfg, index)
        raw = torch.zeros((views, self.cfg["nh"], self.cfg["nw"]), dtype=torch.float32,
                          device=self.dev)
        for v0 in range(0, views, 128):
            phantom_project(ell, self.scan, raw[v0:v0 + 128], view_begin=v0, np_total=views)
        return raw

    def pair(self, index: int):
        raw = self.scan_of(index, self.views)
        dense = self.scan_of(index, self.target_views)
        tgt = torch.zeros(self.cfg["shape"], dtype=torch.float32, device=self.dev)
        backproject(tgt, fdk_filter(dense, self.scan), self.dense.mats, self.cfg["voxel"])
        return raw, tgt


def rel_l2(a: torch.Tensor, b: torch.Tensor) -> float:
    return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))


def evaluate(f: LearnedFilter, data: Data, held) -> dict:
    e_ramp = e_learn = 0.0
    for raw, tgt in held:
        ramp = torch.zeros_like(tgt)
        backproject(ramp, fdk_filter(raw, data.scan), data.sparse.mats, data.cfg["voxel"])
        e_ramp += rel_l2(ramp, tgt) ** 2
        e_learn += rel_l2(f.reconstruct(raw, data.scan, data.sparse), tgt) ** 2
    n = len(held)
    return {"ramp_rel_l2": math.sqrt(e_ramp / n), "learned_rel_l2": math.sqrt(e_learn / n)}


def timed_reconstruction(f: LearnedFilter, data: Data, raw: torch.Tensor, reps: int = 5) -> dict:
    """ms and GUPS of one learned sparse-view reconstruction (filter + BP) and
    of one ramp one, from HIP events on the current stream."""
    out = {}
    for name, fn in (("learned", lambda: f.reconstruct(raw, data.scan, data.sparse)),
                     ("ramp", lambda: backproject(
                         torch.zeros(data.cfg["shape"], device=raw.device),
                         fdk_filter(raw, data.scan), data.sparse.mats, data.cfg["voxel"]))):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        nz, ny, nx = data.cfg["shape"]
        out[name + "_ms"] = ms
        out[name + "_gups"] = nx * ny * nz * data.views / (ms * 1e-3) / 1e9
    return out


def learning_rate(a, it: int, total: int) -> float:
    """Rate of step it of total.  Cosine decay to zero (the default) lets the
    final parameters, which are the ones evaluated, settle: at a constant rate
    the single-phantom steps leave them wherever the last noisy updates put
    them."""
    if a.schedule == "constant":
        return a.lr
    return a.lr * 0.5 * (1.0 + math.cos(math.pi * it / max(total, 1)))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--phantoms", type=int, default=2000, help="training phantoms per epoch")
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--views", type=int, default=90)
    ap.add_argument("--target-views", type=int, default=720)
    ap.add_argument("--held-out", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--schedule", choices=("cosine", "constant"), default="cosine",
                    help="learning rate over the run: cosine decay from --lr to 0, or constant")
    ap.add_argument("--replace", action="store_true",
                    help="network replaces the ramp filter instead of correcting it")
    ap.add_argument("--scale", type=int, default=1,
                    help="divide volume and detector sampling by this factor (same FOV)")
    ap.add_argument("--log-every", type=int, default=50)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = dict(wl.CONFIGS["c5"])
    if a.scale > 1:
        s = a.scale
        cfg["shape"] = tuple(n // s for n in cfg["shape"])
        cfg["voxel"] = tuple(v * s for v in cfg["voxel"])
        cfg["nh"], cfg["nw"] = cfg["nh"] // s, cfg["nw"] // s
        cfg["scan"] = dict(cfg["scan"], du=cfg["scan"]["du"] * s, dv=cfg["scan"]["dv"] * s)
    data = Data(cfg, a.views, a.target_views, dev)
    held = [data.pair(cfg["n_phantoms"] + 1000 + i) for i in range(a.held_out)]

    start = 0
    if a.resume and a.checkpoint and os.path.exists(a.checkpoint):
        f, meta = LearnedFilter.load(a.checkpoint, dev)
        start = int(meta.get("next", 0))
    else:
        # input normalisation from training phantoms only (the held-out set is
        # used by evaluate() alone)
        first = [data.pair(i)[0] for i in range(min(4, a.phantoms))]
        std = float(torch.cat([cosine_weight(r, data.scan).flatten()[::97] for r in first]).std())
        del first
        f = LearnedFilter(dev, residual=not a.replace, seed=a.seed, input_std=std)

    base = evaluate(f, data, held)
    print(json.dumps(dict(step=start, **base)), flush=True)
    total = a.phantoms * a.epochs
    t0 = time.time()
    loss_acc = torch.zeros(1, device=dev)
    for it in range(start, total):
        raw, tgt = data.pair(it % a.phantoms)
        loss_acc += f.train_step(raw, tgt, data.scan, data.sparse, learning_rate(a, it, total))
        if (it + 1) % a.log_every == 0 or it + 1 == total:
            n = int(torch.tensor(cfg["shape"]).prod())
            mse = float(loss_acc) / (n * a.log_every)
            loss_acc.zero_()
            print(json.dumps({"step": it + 1, "train_mse": mse,
                              "s_per_step": (time.time() - t0) / (it + 1 - start)}), flush=True)
            if a.checkpoint:
                f.save(a.checkpoint, next=it + 1, phantoms=a.phantoms, seed=cfg["seed"])
    final = evaluate(f, data, held)
    perf = timed_reconstruction(f, data, held[0][0])
    summary = dict(steps=total, views=a.views, target_views=a.target_views,
                   shape=list(cfg["shape"]), detector=[cfg["nh"], cfg["nw"]],
                   residual=f.residual, ramp_rel_l2_before=base["ramp_rel_l2"],
                   learned_rel_l2_before=base["learned_rel_l2"], **final, **perf)
    print(json.dumps(summary), flush=True)
    return summary


if __name__ == "__main__":
    main()
