#!/usr/bin/env python3
"""Throughput of voxel-driven FDK back-projection on one MI355X.

Workload (default): 512^3 volume (1 mm voxels), 1024 views over 360 degrees,
1024 x 1024 detector (1 mm), SOD 750 mm, SDD 1200 mm; filtered projections of a
seeded 40-ellipsoid phantom generated on the GPU (analytic line integrals +
FDK ramp filter), volume zero-initialised.

One step = zero the volume, FP16 storage pre-pass (per-view scale + binary16
codes), back-projection of all views with FP32 coordinates and accumulation.
The FP32-storage step (zero + back-projection of the float32 stack) is timed
the same way and reported beside it.  GUPS = nx ny nz np / t / 1e9.

Prints ONE JSON line.  Also reports the dominant kernel against its roofline
(timed with HIP events on the stream it runs on) and the FP64 oracle timed on
the host's cores on a bounded sub-block of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operations per voxel update in the hoisted method, FP32, no packed
# math: v = v0 + k dv (1), fraction and row of v (2), two horizontal lerps
# (2 + 2), one vertical lerp (2), weighted accumulation (1).
OPS_PER_UPDATE = 10
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = issue rate of non-packed
# FP32 VALU lane-operations.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# On-chip gather bound: LDS delivers 128 bytes per clock per CU; an update
# reads its four taps from LDS, 16 bytes as float32 or 8 bytes as two
# binary16 pair words.
LDS_BYTES_PER_CLK_CU = 128
# Calibration copy for the HBM byte counters: a plain device-to-device copy of
# this many bytes, run once when --calibrate-copy is given.
CALIBRATION_BYTES = 1 << 30
# Measured HBM traffic of the back-projection kernel (FETCH_SIZE + WRITE_SIZE,
# scaled by the calibration copy) and the hash of the sources it was taken on.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "bp_kernel_c2_512cube_1024views_traffic.md")
KERNEL_SOURCES = ("bp.hip", "footprint.h", "internal.h", "geometry.cpp")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_13248_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the FP16 back-projection from the committed
    counter summary, or None if it is missing, for another workload, or taken
    on other kernel sources."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^(\w+)\s*=\s*(\S+)\s*$", text, flags=re.M))
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if fields.get("workload") != workload:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(*a):
    print("[bench %s]" % time.strftime("%H:%M:%S"), *a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, mats, seconds: float):
    """The FP64 oracle on a centred sub-block of the same workload."""
    import numpy as np
    import oracle
    import workloads as wl
    nz, ny, nx = cfg["shape"]
    npv, nh, nw = cfg["np"], cfg["nh"], cfg["nw"]
    log("cpu baseline: host stack", (npv, nh, nw))
    proj = wl.gaussian(cfg["seed"] + 999, (npv, nh, nw))
    threads = oracle.max_threads()

    def run(b):
        k0, j0, i0 = nz // 2 - b // 2, ny // 2 - b // 2, nx // 2 - b // 2
        t = time.perf_counter()
        oracle.backproject_block(proj, mats, cfg["shape"], cfg["voxel"],
                                 ((k0, k0 + b), (j0, j0 + b), (i0, i0 + b)))
        return time.perf_counter() - t

    b = 8
    dt = run(b)
    while dt < 0.5 and b < 64:
        b *= 2
        dt = run(b)
    rate = b ** 3 * npv / dt
    b2 = int(round((seconds * rate / npv) ** (1.0 / 3.0)))
    b2 = max(8, min(b2, min(nx, ny, nz)))
    dt = run(b2)
    gups = b2 ** 3 * npv / dt / 1e9
    log("cpu baseline: %d^3 block x %d views in %.2fs, %d threads" % (b2, npv, dt, threads))
    return {"value": gups, "unit": "GUPS", "cores": threads, "kind": "oracle",
            "sample": "centred %d^3 sub-block of the %dx%dx%d volume, all %d views, "
                      "Gaussian projections of the same shape; %.1f s" % (b2, nx, ny, nz, npv, dt)}


# Dense FP32 matrix-core peak of MI355X (v_mfma_f32_* instructions).
MFMA_F32_PEAK_TFLOPS = 157.3


def _timed_ms(fn, reps=5):
    """Average ms of fn() over reps runs, HIP events on torch's current
    stream (every operation below runs on that stream)."""
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def ops_report(seconds: float) -> int:
    """--ops: one JSON line per operation beside the back-projector (forward
    projector, FDK filter, learned-filter layers), each against its roofline,
    with the FP64 oracle timed on a bounded sample of the same workload."""
    import numpy as np
    import torch
    import oracle
    from oracle import learned as ol
    import workloads as wl
    import paper_2104_13248_amd as fdk
    from paper_2104_13248_amd import learned as L

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    threads = oracle.max_threads()
    budget = seconds / 4.0                 # oracle seconds per operation, about

    def emit(d):
        print(json.dumps(d), flush=True)

    def scaled(run, b0, cap, cost):
        """Grow the sample size b until the oracle takes ~budget seconds."""
        b = b0
        dt = run(b)
        while dt < 0.1 and 2 * b <= cap:
            b *= 2
            dt = run(b)
        b2 = int(max(b0, min(cap, b * (budget / max(dt, 1e-6)) ** (1.0 / cost))))
        return b2, run(b2)

    # ---- forward projector (exact transpose), 256^3 x 360 views x 384^2
    cfg = wl.CONFIGS["c4"]
    nz, ny, nx = cfg["shape"]
    npv, nh, nw = cfg["np"], cfg["nh"], cfg["nw"]
    mats = np.asarray(fdk.scan_matrices(cfg["scan"], npv, nh, nw))
    vol_h = wl.gaussian(cfg["seed"] + 7, cfg["shape"])
    vol = torch.from_numpy(vol_h.astype(np.float32)).to(dev)
    proj = torch.zeros((npv, nh, nw), dtype=torch.float32, device=dev)
    ms = _timed_ms(lambda: fdk.forwardproject(vol, proj, mats, cfg["voxel"]))
    upd = nx * ny * nz * npv
    gups = upd / (ms * 1e-3) / 1e9
    log("ops: forward projection %.2f ms" % ms)

    def fp_run(b):
        c = nx // 2 - b // 2
        sub = np.ascontiguousarray(vol_h[c:c + b, c:c + b, c:c + b], dtype=np.float64)
        t = time.perf_counter()
        oracle.forwardproject(sub, mats, nh, nw, cfg["voxel"])
        return time.perf_counter() - t

    b, dt = scaled(fp_run, 16, nx, 3.0)
    emit({"op": "forward_projection", "metric": "GUPS (voxel-view updates/s)", "value": gups,
          "unit": "GUPS", "ms": ms, "dtype": "f32", "data": "synthetic: seeded Gaussian volume",
          "config": {"workload": "fdk_forwardprojection_256x256x256_360views_384x384",
                     "voxel_mm": list(cfg["voxel"]), "views": npv, "detector": [nh, nw]},
          "roofline": {"bound": "alu", "achieved": OPS_PER_UPDATE * gups / 1e3,
                       "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                       "frac": OPS_PER_UPDATE * gups / 1e3 / VALU_PEAK_TOPS,
                       "ops_per_update": OPS_PER_UPDATE},
          "cpu_baseline": {"value": b ** 3 * npv / dt / 1e9, "unit": "GUPS", "cores": threads,
                           "kind": "oracle",
                           "sample": "centred %d^3 sub-block, all %d views; %.1f s" % (b, npv, dt)}})
    del vol, proj

    # ---- FDK filter, 128 views x 1024^2 (one chunk of the 1024-view stack)
    cfg = wl.CONFIGS["c2"]
    nh, nw = cfg["nh"], cfg["nw"]
    views = 128
    raw_h = wl.gaussian(cfg["seed"] + 11, (views, nh, nw))
    raw = torch.from_numpy(raw_h).to(dev)
    out = torch.empty_like(raw)
    ms = _timed_ms(lambda: fdk.fdk_filter(raw, cfg["scan"], np_total=cfg["np"], out=out))
    nbytes = 8 * raw.numel()               # read and write one float32 per pixel
    gbs = nbytes / (ms * 1e-3) / 1e9
    log("ops: filter %.2f ms" % ms)

    def filt_run(v):
        t = time.perf_counter()
        oracle.fdk_filter(raw_h[:v].astype(np.float64), cfg["scan"], np_total=cfg["np"])
        return time.perf_counter() - t

    nv, dt = scaled(filt_run, 1, views, 1.0)
    emit({"op": "fdk_filter", "metric": "FDK filter throughput (HBM bytes/s of the stack)",
          "value": gbs, "unit": "GB/s", "ms": ms, "dtype": "f32",
          "data": "synthetic: seeded Gaussian line integrals",
          "config": {"workload": "fdk_filter_128views_1024x1024", "algorithmic_bytes": nbytes},
          "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs / HBM_PEAK_GBS},
          "cpu_baseline": {"value": 8.0 * nv * nh * nw / dt / 1e9, "unit": "GB/s",
                           "cores": threads, "kind": "oracle",
                           "sample": "%d views of %dx%d; %.1f s" % (nv, nh, nw, dt)}})
    del raw, out

    # ---- learned-filter layers, 46080 rows x 512 (one 90-view scan, 512^2)
    rows, n = 90 * 512, 512
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    x32 = torch.randn((rows, 32, n), generator=g, device=dev)
    w2 = torch.randn((32, 32, 9), generator=g, device=dev) * 0.1
    w3 = torch.randn((1, 32, 9), generator=g, device=dev) * 0.1
    b2 = torch.zeros(32, device=dev)
    y32 = torch.empty_like(x32)
    y1 = torch.empty((rows, 1, n), device=dev)
    gw = torch.zeros_like(w2)
    gb = torch.zeros_like(b2)
    flops = 2.0 * rows * n * 32 * 32 * 9
    xs = np.random.default_rng(5).standard_normal((64, 32, n))
    ws = np.random.default_rng(6).standard_normal((32, 32, 9)) * 0.1

    def conv_run(r):
        t = time.perf_counter()
        ol.conv(xs[:r], ws)
        return time.perf_counter() - t

    def wgrad_run(r):
        t = time.perf_counter()
        ol.conv_backward_weight(xs[:r], xs[:r])
        return time.perf_counter() - t

    for name, fn, run, what in (("learned_conv32_forward",
                                 lambda: L.conv1d_forward(x32, w2, b2, relu=True, out=y32),
                                 conv_run, "forward"),
                                ("learned_conv32_weight_gradient",
                                 lambda: L.conv1d_backward_weight(x32, x32, gw, gb),
                                 wgrad_run, "weight gradient")):
        r_cpu, dt_cpu = scaled(run, 1, 64, 1.0)
        cpu_tflops = 2.0 * r_cpu * n * 32 * 32 * 9 / dt_cpu / 1e12
        ms = _timed_ms(fn)
        tf = flops / (ms * 1e-3) / 1e12
        log("ops: %s %.2f ms" % (name, ms))
        emit({"op": name, "metric": "FP32 TFLOP/s (32 -> 32 channels, 9 taps)", "value": tf,
              "unit": "TFLOP/s", "ms": ms, "dtype": "f32", "data": "synthetic: seeded Gaussian",
              "config": {"workload": "conv1d_32x32_k9_46080rows_x512", "flops": flops},
              "roofline": {"bound": "mfma", "achieved": tf, "peak": MFMA_F32_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": tf / MFMA_F32_PEAK_TFLOPS},
              "cpu_baseline": {"value": cpu_tflops, "unit": "TFLOP/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "%s of %d rows (FP64 NumPy); %.1f s" % (what, r_cpu, dt_cpu)}})
    ms = _timed_ms(lambda: L.conv1d_forward(x32, w3, None, out=y1))
    nbytes = 4.0 * rows * n * 33
    gbs = nbytes / (ms * 1e-3) / 1e9
    log("ops: conv 32->1 %.2f ms" % ms)
    w3s = np.random.default_rng(7).standard_normal((1, 32, 9)) * 0.1

    def to1_run(r):
        t = time.perf_counter()
        ol.conv(xs[:r], w3s)
        return time.perf_counter() - t

    r1, dt1 = scaled(to1_run, 1, 64, 1.0)
    emit({"op": "learned_conv_32to1_forward", "metric": "HBM bytes/s (32 channels in, 1 out)",
          "value": gbs, "unit": "GB/s", "ms": ms, "dtype": "f32", "data": "synthetic: seeded Gaussian",
          "config": {"workload": "conv1d_32x1_k9_46080rows_x512", "algorithmic_bytes": nbytes},
          "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs / HBM_PEAK_GBS},
          "cpu_baseline": {"value": 4.0 * r1 * n * 33 / dt1 / 1e9, "unit": "GB/s",
                           "cores": threads, "kind": "oracle",
                           "sample": "%d rows (FP64 NumPy); %.1f s" % (r1, dt1)}})
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy (reference for byte counters)")
    ap.add_argument("--ops", action="store_true",
                    help="report the operations beside the back-projector instead (one JSON "
                         "line each: forward projector, FDK filter, learned-filter layers)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the back-projector has no multi-GPU path in this "
              "build (a z-slab split needs no exchange; see the design notes). Use --gpus 1.",
              file=sys.stderr)
        return 2
    if args.ops:
        return ops_report(args.cpu_seconds)

    import numpy as np
    import torch
    import workloads as wl
    import paper_2104_13248_amd as fdk

    cfg = wl.CONFIGS[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    nz, ny, nx = cfg["shape"]
    npv, nh, nw = cfg["np"], cfg["nh"], cfg["nw"]
    scan = cfg["scan"]
    mats = fdk.scan_matrices(scan, npv, nh, nw)
    plan = fdk.bp_plan(cfg["shape"], cfg["voxel"], npv, nh, nw, mats, f16=True)   # the FP16 step's launch
    log("config", args.config, cfg["shape"], (npv, nh, nw), "plan", plan)

    # ---- synthetic input, generated on the GPU (not timed)
    ell = wl.config_ellipsoids(cfg, 0)
    filt = torch.empty((npv, nh, nw), dtype=torch.float32, device=dev)
    chunk = 128
    raw = torch.empty((chunk, nh, nw), dtype=torch.float32, device=dev)
    for v0 in range(0, npv, chunk):
        n = min(chunk, npv - v0)
        raw[:n].zero_()
        fdk.phantom_project(ell, scan, raw[:n], view_begin=v0, np_total=npv)
        fdk.fdk_filter(raw[:n], scan, np_total=npv, out=filt[v0:v0 + n])
    del raw
    torch.cuda.synchronize()
    log("input ready: filtered stack %.2f GiB" % (filt.numel() * 4 / 2**30))

    if args.calibrate_copy:
        src = torch.ones(CALIBRATION_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: %d bytes" % CALIBRATION_BYTES)

    vol = torch.zeros(cfg["shape"], dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    n_upd = nx * ny * nz * npv

    def step_f16(events=None):
        vol.zero_()
        h, s = fdk.quantize_f16(filt)
        if events is not None:
            events[0].record(stream)
        fdk.backproject(vol, h, mats, cfg["voxel"], scale=s)
        if events is not None:
            events[1].record(stream)

    def step_f32(events=None):
        vol.zero_()
        if events is not None:
            events[0].record(stream)
        fdk.backproject(vol, filt, mats, cfg["voxel"])
        if events is not None:
            events[1].record(stream)

    results = {}
    for name, step in (("f32", step_f32), ("f16", step_f16)):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(args.steps):
            step(ev[q])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        ms = (t1 - t0) * 1e3 / args.steps
        results[name] = dict(ms_per_step=ms, kernel_ms=k_ms, gups=n_upd / (ms * 1e-3) / 1e9,
                             kernel_gups=n_upd / (k_ms * 1e-3) / 1e9)
        log(name, results[name])
        print("progress: %s timed" % name, file=sys.stderr, flush=True)

    f16 = results["f16"]
    f32 = results["f32"]
    k_s = f16["kernel_ms"] * 1e-3
    achieved = n_upd * OPS_PER_UPDATE / k_s / 1e12
    vol_bytes = nx * ny * nz * 4
    hbm_alg = 2 * vol_bytes + npv * nh * nw * 2 + npv * 4           # volume RMW + f16 stack
    lds_bound = 256 * 2.4e9 * LDS_BYTES_PER_CLK_CU / 8 / 1e9      # FP16 storage: 8 B/update
    workload = "fdk_backprojection_%dx%dx%d_%dviews_%dx%d" % (nx, ny, nz, npv, nh, nw)
    traffic = measured_traffic(workload)
    out = {
        "metric": "GUPS (giga voxel-updates/s) FDK backproject, FP16-store vs FP32 at rel-L2<=1e-3",
        "value": f16["gups"],
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f16["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: GPU analytic line integrals of a seeded 40-ellipsoid phantom, "
                "FDK ramp-filtered; FP16 storage with per-view scale",
        "config": {"workload": workload,
                   "volume": [nz, ny, nx], "voxel_mm": list(cfg["voxel"]), "views": npv,
                   "detector": [nh, nw], "pixel_mm": [scan["du"], scan["dv"]],
                   "sod_mm": scan["sod"], "sdd_mm": scan["sdd"], "storage": "f16",
                   "tile": [plan["tile_x"], plan["tile_y"], plan["kz"]],
                   "lds_bytes": plan["lds_bytes"]},
        "fp32_storage": {"value": f32["gups"], "unit": "GUPS", "ms_per_step": f32["ms_per_step"],
                         "kernel_ms": f32["kernel_ms"]},
        "f16_over_f32": f16["gups"] / f32["gups"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                     "traffic_unit": "bytes/launch", "kernel": "bp_kernel", "kernel_ms": f16["kernel_ms"],
                     "ops_per_update": OPS_PER_UPDATE,
                     "hbm_algorithmic_bytes": hbm_alg,
                     "hbm_algorithmic_gbs": hbm_alg / k_s / 1e9,
                     "hbm_frac": hbm_alg / k_s / 1e9 / HBM_PEAK_GBS,
                     "lds_gather_bound_gups": lds_bound,
                     "lds_gather_frac": f16["kernel_gups"] / lds_bound},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, np.asarray(mats), args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
