"""FP16 storage rule for filtered projections (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes in single precision throughout (Section 4.1); storing the
filtered projections as binary16 with one scale per view is an extension of
this repository.  The rule, fixed so that both sides can agree bit for bit:

  m_s     = max |p_s|  over the view (float32 values, exact)
  m_s = 0 -> scale_s = 1
  else    -> write m_s = f * 2^e with f in [0.5, 1);
             scale_s = 2^(e - 15) if f > 0.5, else 2^(e - 16)
             (i.e. 2^(ceil(log2 m_s) - 15), so |p / scale| <= 2^15)
  h       = round-to-nearest-even(p / scale_s) as binary16

p / scale_s is exact in float32 (a power-of-two scale), so the only rounding
is the final conversion; |h| <= 32768 < 65504 never overflows.
"""
from __future__ import annotations

import numpy as np


def view_scales(proj: np.ndarray) -> np.ndarray:
    proj = np.asarray(proj, dtype=np.float32)
    m = np.abs(proj.reshape(proj.shape[0], -1)).max(axis=1).astype(np.float64)
    scale = np.ones(proj.shape[0], dtype=np.float64)
    nz = m > 0
    f, e = np.frexp(m[nz])
    scale[nz] = np.ldexp(1.0, np.where(f > 0.5, e - 15, e - 16))
    return scale.astype(np.float32)


def quantize_f16(proj: np.ndarray):
    """float32 [np,nh,nw] -> (float16 [np,nh,nw], float32 scale [np])."""
    proj = np.asarray(proj, dtype=np.float32)
    scale = view_scales(proj)
    h = (proj / scale[:, None, None]).astype(np.float16)   # numpy casts with RNE
    return h, scale


def dequantize_f16(h: np.ndarray, scale: np.ndarray) -> np.ndarray:
    return h.astype(np.float32) * np.asarray(scale, dtype=np.float32)[:, None, None]
