"""Learned row filter: FP64 reference of its layer operations, gradients,
loss and optimiser step (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper takes filtered projections as input and does not describe the
filter (Sections 2.1.2 and 3.1.1); the textbook FDK filter is in ``oracle.c``.
This module covers the data-driven alternative: a 1-D convolutional network
applied to each cosine-weighted detector row,

    a1 = relu(conv(q, W1) + b1)        1 -> 32 channels
    a2 = relu(conv(a1, W2) + b2)      32 -> 32 channels
    y  = ramp(q) + alpha (conv(a2, W3) + b3)     32 -> 1 channel   (residual form)
    y  = alpha (conv(a2, W3) + b3)                                 (replacement form)

with conv the zero-padded ("same") cross-correlation of 9 taps,
    conv(x, W)[r, o, x] = sum_i sum_t W[o, i, t] x[r, i, x + t - 4],
trained through the back-projector on the mean squared error of the
reconstruction.  Arrays are float64 [rows, channels, len].

Written from the definitions: each gradient is the adjoint of the forward
map it differentiates, and Adam follows Kingma and Ba (ICLR 2015),
Algorithm 1.
"""
from __future__ import annotations

import math

import numpy as np

K = 9
HALO = K // 2


def cosine_weight(raw: np.ndarray, scan: dict) -> np.ndarray:
    """Step 1 of the FDK filter: raw * sdd / |ray| for every pixel; the ray from
    the source to pixel (r, c) has in-plane and axial offsets u_mm, v_mm from
    the principal ray (Section 2.1.1 geometry)."""
    raw = np.asarray(raw, dtype=np.float64)
    npv, nh, nw = raw.shape
    cu = 0.5 * (nw - 1) + scan["u_off"]
    cv = 0.5 * (nh - 1) + scan["v_off"]
    u = (np.arange(nw) - cu) * scan["du"]
    v = (np.arange(nh) - cv) * scan["dv"]
    sdd = scan["sdd"]
    w = sdd / np.sqrt(sdd * sdd + u[None, :] ** 2 + v[:, None] ** 2)
    return raw * w[None, :, :]


def _windows(x: np.ndarray) -> np.ndarray:
    """[rows, ch, len] -> [rows, ch, len, K]: the K samples x[.., x + t - 4]
    each output position reads, zeros outside the row."""
    pad = np.pad(np.asarray(x, dtype=np.float64), ((0, 0), (0, 0), (HALO, HALO)))
    return np.lib.stride_tricks.sliding_window_view(pad, K, axis=2)


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """out[r, o, x] = b[o] + sum_{i, t} w[o, i, t] x[r, i, x + t - 4]."""
    out = np.einsum("rixt,oit->rox", _windows(x), np.asarray(w, dtype=np.float64))
    if b is not None:
        out = out + np.asarray(b, dtype=np.float64)[None, :, None]
    return out


def conv_backward_data(gout: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of x -> conv(x, w): every output sample gout[r, o, x] sends
    w[o, i, t] gout[r, o, x] back to the input sample x + t - 4 it read
    (dropped when that sample is padding)."""
    gout = np.asarray(gout, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    rows, cout, n = gout.shape
    gin = np.zeros((rows, w.shape[1], n))
    for t in range(K):
        s = t - HALO                     # input index = x + s
        lo, hi = max(0, -s), min(n, n - s)
        if lo >= hi:
            continue
        # gin[:, i, x + s] += sum_o w[o, i, t] gout[:, o, x]
        gin[:, :, lo + s:hi + s] += np.einsum("rox,oi->rix", gout[:, :, lo:hi], w[:, :, t])
    return gin


def conv_backward_weight(x: np.ndarray, gout: np.ndarray):
    """Gradients of sum(gout * conv(x, w, b)) with respect to w and b."""
    gw = np.einsum("rox,rixt->oit", np.asarray(gout, dtype=np.float64), _windows(x))
    gb = np.asarray(gout, dtype=np.float64).sum(axis=(0, 2))
    return gw, gb


def relu(x):
    return np.maximum(x, 0.0)


def init_params(seed: int, input_std: float = 1.0, residual: bool = True) -> dict:
    """He-normal initialisation of the three layers (the first scaled to an
    input of standard deviation ``input_std``); in the residual form the last
    layer starts at zero, so the untrained filter is the ramp filter."""
    rng = np.random.default_rng(seed)
    p = {
        "w1": rng.standard_normal((32, 1, K)) * math.sqrt(2.0 / K) / input_std,
        "b1": np.zeros(32),
        "w2": rng.standard_normal((32, 32, K)) * math.sqrt(2.0 / (32 * K)),
        "b2": np.zeros(32),
        "w3": rng.standard_normal((1, 32, K)) * math.sqrt(1.0 / (32 * K)),
        "b3": np.zeros(1),
    }
    if residual:
        p["w3"][:] = 0.0
    return p


PARAM_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3")


def net_forward(q: np.ndarray, p: dict, alpha: float, ramp: np.ndarray | None = None):
    """q: [rows, len] cosine-weighted rows; ramp: [rows, len] ramp-filtered rows
    (residual form) or None (replacement form).  Returns (y [rows, len], cache)."""
    x0 = np.asarray(q, dtype=np.float64)[:, None, :]
    a1 = relu(conv(x0, p["w1"], p["b1"]))
    a2 = relu(conv(a1, p["w2"], p["b2"]))
    y = alpha * conv(a2, p["w3"], p["b3"])[:, 0, :]
    if ramp is not None:
        y = y + np.asarray(ramp, dtype=np.float64)
    return y, (x0, a1, a2)


def net_backward(gy: np.ndarray, p: dict, alpha: float, cache) -> dict:
    """Gradients of sum(gy * y) with respect to every parameter (chain rule
    through the three layers; the ReLU derivative is 1 where its output is
    positive)."""
    x0, a1, a2 = cache
    g3 = alpha * np.asarray(gy, dtype=np.float64)[:, None, :]
    gw3, gb3 = conv_backward_weight(a2, g3)
    g2 = conv_backward_data(g3, p["w3"]) * (a2 > 0)
    gw2, gb2 = conv_backward_weight(a1, g2)
    g1 = conv_backward_data(g2, p["w2"]) * (a1 > 0)
    gw1, gb1 = conv_backward_weight(x0, g1)
    return {"w1": gw1, "b1": gb1, "w2": gw2, "b2": gb2, "w3": gw3, "b3": gb3}


def sqerr(a: np.ndarray, b: np.ndarray):
    """(sum (a - b)^2, gradient of the mean 2 (a - b) / n)."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return float(np.sum(d * d)), 2.0 * d / d.size


def adam(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One step of Adam (Kingma and Ba, Algorithm 1) at step t >= 1; returns
    the new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
