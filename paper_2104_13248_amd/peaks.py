"""Binding of include/fdk_peaks.h: one launch of each ceiling microbenchmark on
torch's current stream (argument marshalling only; the caller times it)."""
from __future__ import annotations

import ctypes

import torch

from ._lib import check, lib

LDS_PATTERNS = {"b32": 0, "read2_b32": 1, "b64": 2, "b128": 3, "taps_f16": 4, "taps_f32": 5}


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
