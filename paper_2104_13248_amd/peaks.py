"""Binding of include/fdk_peaks.h: one launch of each ceiling microbenchmark on
torch's current stream (argument marshalling only; the caller times it)."""
from __future__ import annotations

import ctypes

import torch

from ._lib import check, lib

LDS_PATTERNS = {"b32": 0, "read2_b32": 1, "b64": 2, "b128": 3, "taps_f16": 4, "taps_f32": 5,
                "b64_asm": 6, "b64_asm_dword": 7}
VALU_OPS = {"v_fma_f32": 0, "v_fmac_f32": 1, "v_sub_f32": 2, "v_fract_f32": 3,
            "v_cvt_i32_f32": 4, "v_mad_u32_u24": 5, "v_fma_mix_f32": 6, "v_cvt_f32_f16": 7,
            "v_dot2_f32_f16": 8, "v_pk_fma_f16": 9, "v_add_u32": 10, "v_floor_f32": 11}


def _sink(dev):
    return torch.zeros(1, dtype=torch.int32, device=dev)


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def hbm_read(buf: torch.Tensor, nbytes: int, blocks: int, sink=None) -> int:
    """Stream the first ``nbytes`` of ``buf`` (a contiguous device tensor) once.
    Returns the bytes read."""
    if buf.device.type != "cuda" or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    if nbytes > buf.numel() * buf.element_size():
        raise ValueError("nbytes exceeds the buffer")
    sink = _sink(buf.device) if sink is None else sink
    with torch.cuda.device(buf.device):
        check(lib.fdk_peak_hbm_read(buf.data_ptr(), int(nbytes), int(blocks), sink.data_ptr(),
                                    _stream(buf.device)))
    return int(nbytes)


def lds_read(pattern: str, blocks: int, iters: int, device, sink=None) -> int:
    """One LDS read launch of ``pattern``; returns the bytes it reads from LDS."""
    out = ctypes.c_int64(0)
    sink = _sink(device) if sink is None else sink
    with torch.cuda.device(device):
        check(lib.fdk_peak_lds_read(LDS_PATTERNS[pattern], int(blocks), int(iters),
                                    sink.data_ptr(), ctypes.addressof(out), _stream(device)))
    return int(out.value)


def valu_fma(blocks: int, iters: int, device, sink=None) -> int:
    """One float32 FMA launch; returns its lane-operations."""
    out = ctypes.c_int64(0)
    sink = _sink(device) if sink is None else sink
    with torch.cuda.device(device):
        check(lib.fdk_peak_valu_fma(int(blocks), int(iters), sink.data_ptr(),
                                    ctypes.addressof(out), _stream(device)))
    return int(out.value)


def valu_op(op: str, blocks: int, iters: int, device, sink=None) -> int:
    """One launch issuing only instruction ``op``; returns its lane-operations."""
    out = ctypes.c_int64(0)
    sink = _sink(device) if sink is None else sink
    with torch.cuda.device(device):
        check(lib.fdk_peak_valu_op(VALU_OPS[op], int(blocks), int(iters), sink.data_ptr(),
                                   ctypes.addressof(out), _stream(device)))
    return int(out.value)


def _best(fn, reps=5):
    """Best work/second of ``reps`` launches of fn() (HIP events, current stream)."""
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        work = fn()
        b.record(s)
        torch.cuda.synchronize()
        best = max(best, work / (a.elapsed_time(b) * 1e-3))
    return best


def main():
    """python -m paper_2104_13248_amd.peaks: one JSON line per ceiling."""
    import json
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    buf = torch.ones((8 << 30) // 4, dtype=torch.float32, device=dev)
    print(json.dumps({"what": "hbm_read", "bytes": 8 << 30,
                      "GB/s": _best(lambda: hbm_read(buf, 8 << 30, 256 * 16, sink)) / 1e9}),
          flush=True)
    del buf
    for pat in LDS_PATTERNS:
        r = _best(lambda: lds_read(pat, 256 * 20, 1000, dev, sink))
        print(json.dumps({"what": "lds_" + pat, "GB/s": r / 1e9,
                          "bytes_per_clk_per_cu_at_2.4GHz": r / (256 * 2.4e9)}), flush=True)
    for op in VALU_OPS:
        r = _best(lambda: valu_op(op, 256 * 16, 500, dev, sink))
        print(json.dumps({"what": op, "Tlane-ops/s": r / 1e12,
                          "lanes_per_clk_per_cu_at_2.4GHz": r / (256 * 2.4e9)}), flush=True)


if __name__ == "__main__":
    main()
