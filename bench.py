#!/usr/bin/env python3
"""Throughput of voxel-driven FDK back-projection on one MI355X.

Workload (default, the FP16-storage metric's configuration): 1024^3 volume
(0.5 mm voxels), 2048 views over 360 degrees, 2048 x 2048 detector (0.5 mm),
SOD 750 mm, SDD 1200 mm; filtered projections of a seeded 60-ellipsoid
phantom generated on the GPU (analytic line integrals + FDK ramp filter),
stored once as float32 and once as binary16 with one power-of-two scale per
view (written by the filter itself); volume zero-initialised.

One step = zero the volume, back-project all views with FP32 coordinates and
accumulation.  Both storages are timed the same way; the binary16 one is the
headline `value`, the float32 one is reported beside it.
GUPS = nx ny nz np / t / 1e9 (Section 2.3).

After timing, the last volume of each storage is checked: rel-L2 of the
binary16-storage volume against the float32-storage volume (whole volume),
and of both against the FP64 oracle on eight 64^3 sub-blocks (centre, corners,
edges), the oracle reading only each view's window of the same stacks.  The
run fails (exit 3) if float32 storage is above 1e-5 or binary16 storage above
1e-3 of the oracle.  The oracle's timing on those blocks is the CPU baseline.

Prints ONE JSON line, with the dominant kernel against its rooflines (timed
with HIP events on the stream it runs on) and the ceilings measured on the
same GPU by the microbenchmarks of include/fdk_peaks.h.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operations per voxel update in the hoisted method, FP32, no packed
# math: v = v0 + k dv (1), fraction and row of v (2), two horizontal lerps
# (2 + 2), one vertical lerp (2), weighted accumulation (1).
OPS_PER_UPDATE = 10
# MI355X vector FP32 peak: 157.3 TFLOP/s counting an FMA as two flops, i.e.
# 256 CUs x 128 FP32 lane-operations per clock x 2.4 GHz = 78.6 T lane-ops/s.
# (Non-packed FMAs reach it: the fdk_peak_valu_fma microbenchmark issues
# v_fma_f32 at 68 T lane-ops/s, well above a 64-lane-per-clock reading.)
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Nominal LDS bandwidth: 128 bytes per clock per CU.
LDS_NOMINAL_GBS = 256 * 128 * 2.4e9 / 1e9
# LDS bytes an update reads: binary16 taps are one ds_read2_b32 of two pair
# words (8 bytes), float32 taps two of them (16 bytes).
TAP_BYTES = {"f16": 8, "f32": 16}
# Measured HBM traffic of the back-projection kernel (FETCH_SIZE + WRITE_SIZE,
# scaled by a plain copy of known size) and the hash of the sources it was
# taken on, per storage; one summary per workload.
TRAFFIC_PROFILES = tuple(os.path.join(ROOT, "profiles", f) for f in (
    "bp_kernel_c3_1024cube_2048views_traffic.md", "bp_kernel_c2_512cube_1024views_traffic.md"))
KERNEL_SOURCES = ("bp.hip", "footprint.h", "internal.h", "geometry.cpp")
TOL = {"f32": 1e-5, "f16": 1e-3}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_13248_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, storage: str):
    """HBM bytes per launch of the back-projection for one storage from the
    committed counter summary of this workload, or None if there is none or
    it was taken on other kernel sources."""
    for path in TRAFFIC_PROFILES:
        try:
            text = open(path).read()
        except OSError:
            continue
        fields = dict(re.findall(r"^(\w+)\s*=\s*(\S+)\s*$", text, flags=re.M))
        if fields.get("workload") != workload:
            continue
        if fields.get("kernel_source_sha256") != kernel_source_hash():
            return None
        try:
            return float(fields["traffic_bytes_per_launch_" + storage])
        except (KeyError, ValueError):
            return None
    return None


def log(*a):
    print("[bench %s]" % time.strftime("%H:%M:%S"), *a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def subblocks(shape, b=64):
    """Eight b^3 boxes ((k0,k1),(j0,j1),(i0,i1)): the centre, four corners and
    three edge midpoints of a [nz,ny,nx] volume."""
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


def accuracy_and_oracle(cfg, mats, filt, h, sc, vol32, vol16):
    """rel-L2 of the timed volumes (binary16 against float32 storage over the
    whole volume; both against the FP64 oracle on eight 64^3 sub-blocks) and
    the oracle's own throughput on those blocks (the CPU baseline)."""
    import numpy as np
    import torch
    import oracle
    from oracle import window as ow

    shape, voxel = cfg["shape"], cfg["voxel"]
    nz, ny, nx = shape
    npv, nh, nw = cfg["np"], cfg["nh"], cfg["nw"]
    # whole volume, binary16 against float32 storage (slabs of 64 slices)
    num = den = 0.0
    for k0 in range(0, nz, 64):
        a = vol16[k0:k0 + 64].double()
        b = vol32[k0:k0 + 64].double()
        num += float(((a - b) ** 2).sum())
        den += float((b ** 2).sum())
    f16_vs_f32 = (num / den) ** 0.5 if den > 0 else float("inf")
    log("accuracy: f16 vs f32 storage (whole volume) %.3e" % f16_vs_f32)

    threads = oracle.max_threads()
    sc_h = sc.cpu().numpy()
    acc = dict(e32=0.0, r32=0.0, e16=0.0, e16d=0.0, r16=0.0)
    t_oracle = 0.0
    n_oracle = 0
    single = None
    for q, box in enumerate(subblocks(shape)):
        (k0, k1), (j0, j1), (i0, i1) = box
        origin, wr, wc = ow.block_windows(mats, shape, voxel, box)
        w32 = ow.cut_windows_device(filt, origin, wr, wc)
        w16 = ow.cut_windows_device(h, origin, wr, wc)
        t = time.perf_counter()
        ref32 = oracle.backproject_block(w32, mats, shape, voxel, box, origin=origin,
                                         detector=(nh, nw), threads=threads)
        ref16 = oracle.backproject_block(w16, mats, shape, voxel, box, scale=sc_h,
                                         origin=origin, detector=(nh, nw), threads=threads)
        t_oracle += time.perf_counter() - t
        n_oracle += 2 * ref32.size * npv
        g32 = vol32[k0:k1, j0:j1, i0:i1].double().cpu().numpy()
        g16 = vol16[k0:k1, j0:j1, i0:i1].double().cpu().numpy()
        acc["e32"] += float(((g32 - ref32) ** 2).sum())
        acc["r32"] += float((ref32 ** 2).sum())
        acc["e16"] += float(((g16 - ref32) ** 2).sum())
        acc["e16d"] += float(((g16 - ref16) ** 2).sum())
        acc["r16"] += float((ref16 ** 2).sum())
        if q == 0:
            # one thread, the first 256 views of the centre block (the
            # thread count is passed explicitly to every call)
            nv = min(256, npv)
            t = time.perf_counter()
            oracle.backproject_block(w32[:nv], mats[:nv], shape, voxel, box, origin=origin[:nv],
                                     detector=(nh, nw), threads=1)
            dt1 = time.perf_counter() - t
            single = ref32.size * nv / dt1 / 1e9
        log("accuracy: block %d %s window %dx%d" % (q, box, wr, wc))
    rel = {
        "f16_vs_f32_storage": f16_vs_f32,
        "f32_vs_oracle": (acc["e32"] / acc["r32"]) ** 0.5,
        "f16_vs_oracle": (acc["e16"] / acc["r32"]) ** 0.5,
        "f16_vs_oracle_dequantised": (acc["e16d"] / acc["r16"]) ** 0.5,
        "oracle_blocks": "eight 64^3 sub-blocks (centre, four corners, three edges), all %d views" % npv,
    }
    rel["ok"] = bool(rel["f32_vs_oracle"] <= TOL["f32"] and rel["f16_vs_oracle"] <= TOL["f16"]
                     and rel["f16_vs_f32_storage"] <= TOL["f16"])
    cpu = {"value": n_oracle / t_oracle / 1e9, "unit": "GUPS", "cores": threads, "kind": "oracle",
           "sample": "FP64 oracle on the eight 64^3 sub-blocks of the accuracy check, %d views, "
                     "both stacks (float32 and dequantised binary16), each view's detector "
                     "window only; %.1f s" % (npv, t_oracle),
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "single_core_gups": single,
           "single_core_sample": "centre 64^3 block, first %d views, 1 thread" % min(256, npv)}
    return rel, cpu


def measure_peaks(buf, dev):
    """Ceilings measured on this GPU (include/fdk_peaks.h): best of 5 launches
    of an HBM stream read, LDS reads and a float32 FMA loop."""
    import torch
    from paper_2104_13248_amd import peaks as pk

    stream = torch.cuda.current_stream(dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)

    def best(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            work = fn()
            b.record(stream)
            torch.cuda.synchronize()
            out.append(work / (a.elapsed_time(b) * 1e-3))
        return max(out)

    nbytes = min(buf.numel() * buf.element_size(), 16 << 30) // 16 * 16
    res = {"hbm_read_gbs": best(lambda: pk.hbm_read(buf, nbytes, 256 * 16, sink)) / 1e9,
           "hbm_read_bytes": nbytes}
    for pat in ("b32", "read2_b32", "b64", "b128", "taps_f16", "taps_f32"):
        res["lds_%s_gbs" % pat] = best(lambda: pk.lds_read(pat, 256 * 20, 1000, dev, sink)) / 1e9
    res["valu_fma_tops"] = best(lambda: pk.valu_fma(256 * 16, 1000, dev, sink)) / 1e12
    return res


def h2d_inclusive(vol, h, sc, mats, voxel, dev):
    """Secondary timing: back-projection including the host-to-device copy
    of the binary16 stack from pinned host memory (the paper's GPU comparison
    counts the upload of the projections, Section 4.5)."""
    import torch
    import paper_2104_13248_amd as fdk
    host = torch.empty(h.shape, dtype=h.dtype, pin_memory=True)
    host.copy_(h)
    dst = torch.empty_like(h)
    torch.cuda.synchronize()
    times = []
    for _ in range(2):
        vol.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        dst.copy_(host, non_blocking=True)
        fdk.backproject(vol, dst, mats, voxel, scale=sc)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    del host, dst
    return min(times)


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
    # The Fourier-domain filter is bound by its transforms' arithmetic: per
    # pair of rows one forward and one inverse complex transform of length M
    # (the power of two >= 2 nw - 1), 5 M log2 M flops each (radix-2 count).
    m_fft = 16
    while m_fft < 2 * nw - 1:
        m_fft *= 2
    fft_flops = (views * nh + 1) // 2 * 2 * 5 * m_fft * int(math.log2(m_fft))
    fft_tops = fft_flops / (ms * 1e-3) / 1e12
    emit({"op": "fdk_filter", "metric": "FDK filter throughput (HBM bytes/s of the stack)",
          "value": gbs, "unit": "GB/s", "ms": ms, "dtype": "f32",
          "data": "synthetic: seeded Gaussian line integrals",
          "config": {"workload": "fdk_filter_128views_1024x1024", "algorithmic_bytes": nbytes,
                     "transform_length": m_fft, "algorithmic_flops": fft_flops},
          "roofline": {"bound": "alu", "achieved": fft_tops, "peak": VALU_PEAK_TOPS,
                       "unit": "TFLOP/s", "frac": fft_tops / VALU_PEAK_TOPS,
                       "hbm_frac": gbs / HBM_PEAK_GBS},
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
    ap.add_argument("--config", default="c3")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle seconds per operation of --ops")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the accuracy check and the CPU baseline (profiling runs)")
    ap.add_argument("--no-h2d", action="store_true", help="skip the upload-inclusive timing")
    ap.add_argument("--only", choices=("f16", "f32"), default=None,
                    help="time one storage only (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy (reference for byte counters)")
    ap.add_argument("--ops", action="store_true",
                    help="report the operations beside the back-projector instead (one JSON "
                         "line each: forward projector, FDK filter, learned-filter layers)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the back-projector runs on one GPU per call "
              "(a volume split into z-slabs needs no exchange between GPUs). Use --gpus 1.",
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
    mats = np.asarray(fdk.scan_matrices(scan, npv, nh, nw))
    plans = {st: fdk.bp_plan(cfg["shape"], cfg["voxel"], npv, nh, nw, mats, f16=(st == "f16"))
             for st in ("f16", "f32")}
    log("config", args.config, cfg["shape"], (npv, nh, nw), "plans", plans)
    stream = torch.cuda.current_stream(dev)

    # ---- synthetic input, generated on the GPU (not timed): one phantom,
    # line integrals, FDK filter into float32 and into binary16 + scale
    ell = wl.config_ellipsoids(cfg, 0)
    filt = torch.empty((npv, nh, nw), dtype=torch.float32, device=dev)
    h = torch.empty((npv, nh, nw), dtype=torch.float16, device=dev)
    sc = torch.empty(npv, dtype=torch.float32, device=dev)
    chunk = 64
    raw = torch.empty((chunk, nh, nw), dtype=torch.float32, device=dev)
    for v0 in range(0, npv, chunk):
        n = min(chunk, npv - v0)
        raw[:n].zero_()
        fdk.phantom_project(ell, scan, raw[:n], view_begin=v0, np_total=npv)
        fdk.fdk_filter(raw[:n], scan, np_total=npv, out=filt[v0:v0 + n])
        fdk.fdk_filter(raw[:n], scan, np_total=npv, out=h[v0:v0 + n], dtype=torch.float16,
                       scale=sc[v0:v0 + n])
    torch.cuda.synchronize()
    log("input ready: %d ellipsoids, float32 stack %.2f GiB, binary16 stack %.2f GiB"
        % (len(ell), filt.numel() * 4 / 2**30, h.numel() * 2 / 2**30))

    # filter and stand-alone FP16 pre-pass cost (context: not in the step)
    n = min(chunk, npv)
    tmp32 = torch.empty_like(raw[:n])
    tmp16 = torch.empty(raw[:n].shape, dtype=torch.float16, device=dev)
    tmps = torch.empty(n, dtype=torch.float32, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    fdk.fdk_filter(raw[:n], scan, np_total=npv, out=tmp32)
    ev[1].record(stream)
    fdk.fdk_filter(raw[:n], scan, np_total=npv, out=tmp16, dtype=torch.float16, scale=tmps)
    ev[2].record(stream)
    torch.cuda.synchronize()
    del tmp32, tmp16, tmps
    filter_ms = {"f32_per_view": ev[0].elapsed_time(ev[1]) / n,
                 "f16_per_view": ev[1].elapsed_time(ev[2]) / n}
    del raw
    torch.cuda.synchronize()
    ev[0].record(stream)
    hq, sq = fdk.quantize_f16(filt)
    ev[1].record(stream)
    torch.cuda.synchronize()
    prepass_ms = ev[0].elapsed_time(ev[1])
    same = bool(torch.equal(hq.view(torch.int16), h.view(torch.int16)) and torch.equal(sq, sc))
    del hq, sq
    log("filter ms/view f32 %.3f f16 %.3f; stand-alone pre-pass %.2f ms; filter f16 output "
        "bit-equal to the pre-pass: %s" % (filter_ms["f32_per_view"], filter_ms["f16_per_view"],
                                           prepass_ms, same))

    if args.calibrate_copy:
        src = torch.ones((1 << 30) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: %d bytes" % (1 << 30))

    vols = {st: torch.zeros(cfg["shape"], dtype=torch.float32, device=dev) for st in ("f16", "f32")}
    n_upd = nx * ny * nz * npv

    def step(st, events=None):
        vol = vols[st]
        vol.zero_()
        if events is not None:
            events[0].record(stream)
        if st == "f16":
            fdk.backproject(vol, h, mats, cfg["voxel"], scale=sc)
        else:
            fdk.backproject(vol, filt, mats, cfg["voxel"])
        if events is not None:
            events[1].record(stream)

    results = {}
    for st in (("f32", "f16") if args.only is None else (args.only,)):
        for _ in range(args.warmup):
            step(st)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q in range(args.steps):
            step(st, evs[q])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        ms = (t1 - t0) * 1e3 / args.steps
        results[st] = dict(ms_per_step=ms, kernel_ms=k_ms, gups=n_upd / (ms * 1e-3) / 1e9,
                           kernel_gups=n_upd / (k_ms * 1e-3) / 1e9)
        log(st, results[st])
        print("progress: %s timed" % st, file=sys.stderr, flush=True)
    if args.only is not None:
        print(json.dumps({"storage": args.only, **results[args.only]}), flush=True)
        return 0

    peaks = measure_peaks(filt, dev)
    log("peaks", peaks)
    workload = "fdk_backprojection_%dx%dx%d_%dviews_%dx%d" % (nx, ny, nz, npv, nh, nw)
    vol_bytes = nx * ny * nz * 4

    def roofline(st):
        r = results[st]
        k_s = r["kernel_ms"] * 1e-3
        ops = n_upd * OPS_PER_UPDATE / k_s / 1e12
        hbm_alg = 2 * vol_bytes + npv * nh * nw * (2 if st == "f16" else 4) + \
            (npv * 4 if st == "f16" else 0)
        lds_gbs = n_upd * TAP_BYTES[st] / k_s / 1e9
        lds_peak = peaks["lds_read2_b32_gbs"]
        hbm_gbs = hbm_alg / k_s / 1e9
        mem_bound_gups = min(lds_peak * 1e9 / TAP_BYTES[st],
                             peaks["hbm_read_gbs"] * 1e9 / (hbm_alg / n_upd)) / 1e9
        valu_bound_gups = peaks["valu_fma_tops"] * 1e12 / OPS_PER_UPDATE / 1e9
        return {"bound": "alu", "achieved": ops, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": ops / VALU_PEAK_TOPS, "traffic": measured_traffic(workload, st),
                "traffic_unit": "bytes/launch",
                "kernel": "bp_kernel<%d,%d,%s>" % (plans[st]["kz"], plans[st]["lds_pitch"],
                                                   "true" if st == "f16" else "false"),
                "kernel_ms": r["kernel_ms"], "ops_per_update": OPS_PER_UPDATE,
                "measured_peak": peaks["valu_fma_tops"],
                "frac_of_measured": ops / peaks["valu_fma_tops"],
                "memory_roofline": {
                    "bound": "lds_gather", "tap_bytes_per_update": TAP_BYTES[st],
                    "achieved_gbs": lds_gbs, "peak_gbs": lds_peak,
                    "peak_source": "measured ds_read2_b32, no bank conflict",
                    "frac": lds_gbs / lds_peak, "nominal_peak_gbs": LDS_NOMINAL_GBS,
                    "tap_pattern_gbs": peaks["lds_taps_%s_gbs" % st],
                    "hbm_algorithmic_bytes": hbm_alg, "hbm_achieved_gbs": hbm_gbs,
                    "hbm_peak_gbs": peaks["hbm_read_gbs"],
                    "hbm_frac": hbm_gbs / peaks["hbm_read_gbs"],
                    "bound_gups": mem_bound_gups,
                    "frac_of_bound": r["kernel_gups"] / mem_bound_gups},
                "valu_bound_gups": valu_bound_gups,
                "binding_ceiling": "valu" if valu_bound_gups < mem_bound_gups else "memory"}

    f16, f32 = results["f16"], results["f32"]
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
        "data": "synthetic: GPU analytic line integrals of a seeded %d-ellipsoid phantom, "
                "FDK ramp-filtered; binary16 storage with per-view scale written by the "
                "filter" % len(ell),
        "config": {"workload": workload,
                   "volume": [nz, ny, nx], "voxel_mm": list(cfg["voxel"]), "views": npv,
                   "detector": [nh, nw], "pixel_mm": [scan["du"], scan["dv"]],
                   "sod_mm": scan["sod"], "sdd_mm": scan["sdd"], "storage": "f16",
                   "tile": [plans["f16"]["tile_x"], plans["f16"]["tile_y"], plans["f16"]["kz"]],
                   "lds_bytes": plans["f16"]["lds_bytes"]},
        "fp32_storage": {"value": f32["gups"], "unit": "GUPS", "ms_per_step": f32["ms_per_step"],
                         "kernel_ms": f32["kernel_ms"], "roofline": roofline("f32")},
        "f16_over_f32": f16["gups"] / f32["gups"],
        "roofline": roofline("f16"),
        "peaks_measured": peaks,
        "filter_ms": filter_ms,
        "f16_prepass_ms": prepass_ms,
        "filter_f16_equals_prepass": same,
    }
    if not args.no_h2d:
        t = h2d_inclusive(vols["f16"], h, sc, mats, cfg["voxel"], dev)
        out["h2d_inclusive"] = {"value": n_upd / t / 1e9, "unit": "GUPS", "s": t,
                                "what": "binary16 stack uploaded from pinned host memory, "
                                        "then back-projected (one call)"}
        log("h2d inclusive %.3f s" % t)
        step("f16")                     # the checked volume is a timed-step result
        torch.cuda.synchronize()
    rc = 0
    if not args.no_check:
        rel, cpu = accuracy_and_oracle(cfg, mats, filt, h, sc, vols["f32"], vols["f16"])
        out["rel_l2"] = rel
        out["cpu_baseline"] = cpu
        rc = 0 if rel["ok"] else 3
    print(json.dumps(out), flush=True)
    return rc


if __name__ == "__main__":
    sys.exit(main())
