"""Learned row filter for sparse-view FDK, trained through the back-projector.

The paper's input is filtered projections (Sections 2.1.2 and 3.1.1); this
module replaces or corrects the fixed ramp filter with a small 1-D
convolutional network applied to every cosine-weighted detector row:

    q  = cosine_weight(raw)
    a1 = relu(conv(q, W1) + b1)            1 -> 32 channels, 9 taps
    a2 = relu(conv(a1, W2) + b2)          32 -> 32 channels, 9 taps
    z  = conv(a2, W3) + b3                32 ->  1 channel,  9 taps
    y  = ramp(raw) + alpha z   (residual form; the untrained net is the ramp filter)
    y  = alpha z               (replacement form)

with alpha = arc / (2 np), the angular weight of the FDK sum, so that one
network serves any number of views.  A training step reconstructs
vol = BP(y), takes the mean squared error against a target volume, sends the
gradient back through the exact transpose of BP (the forward projector) and
through the three layers, and applies one Adam step -- every operation in the
HIP kernels of libfdk.so (include/fdk.h, include/fdk_learn.h); this module
only sequences the calls and owns the device buffers.

Parameters, gradients and Adam moments each live in one flat device buffer
(order w1, b1, w2, b2, w3, b3), so the optimiser is a single launch and a
checkpoint is four arrays.
"""
from __future__ import annotations

import json
import math

import numpy as np
import torch

from . import backproject, fdk_filter, forwardproject
from ._lib import check, lib, stack_struct
from .autograd import Geometry

K = 9
CH = 32
SHAPES = (("w1", (CH, 1, K)), ("b1", (CH,)), ("w2", (CH, CH, K)), ("b2", (CH,)),
          ("w3", (1, CH, K)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def _p(t: torch.Tensor | None, name: str, dev=None) -> int | None:
    if t is None:
        return None
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 device tensor" % name)
    if dev is not None and t.device != dev:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, dev))
    return t.data_ptr()


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


# ---------------------------------------------------------------- layer operations

def cosine_weight(raw: torch.Tensor, scan: dict, out: torch.Tensor | None = None):
    """raw * sdd / sqrt(sdd^2 + u_mm^2 + v_mm^2) (step 1 of the FDK filter)."""
    dev = raw.device
    if out is None:
        out = torch.empty_like(raw)
    npv, nh, nw = raw.shape
    with torch.cuda.device(dev):
        check(lib.fdk_cosine_weight(stack_struct(npv, nh, nw), _p(raw, "raw"), _p(out, "out", dev),
                                    scan["du"], scan["dv"], scan["sdd"], scan["u_off"],
                                    scan["v_off"], _stream(dev)))
    return out


def _rows_len(x: torch.Tensor, ch: int, name: str):
    if x.dim() != 3 or x.shape[1] != ch:
        raise ValueError("%s must be [rows, %d, len], got %s" % (name, ch, tuple(x.shape)))
    return int(x.shape[0]), int(x.shape[2])


def conv1d_forward(x, w, bias=None, mask=None, add=None, alpha=1.0, relu=False, out=None):
    """out = alpha * mask(relu(conv(x, w) + bias)) + add; x [rows, cin, len],
    w [cout, cin, 9]."""
    cout, cin, k = w.shape
    if k != K:
        raise ValueError("conv1d takes 9 taps")
    rows, n = _rows_len(x, cin, "x")
    dev = x.device
    if out is None:
        out = torch.empty((rows, cout, n), dtype=torch.float32, device=dev)
    for t, nm in ((mask, "mask"), (add, "add")):
        if t is not None and tuple(t.shape) != (rows, cout, n):
            raise ValueError("%s must have the output's shape" % nm)
    with torch.cuda.device(dev):
        check(lib.fdk_conv1d_forward(cin, cout, rows, n, _p(x, "x", dev), _p(w, "w", dev),
                                     _p(bias, "bias", dev), _p(mask, "mask", dev),
                                     _p(add, "add", dev), float(alpha), 1 if relu else 0,
                                     _p(out, "out", dev), _stream(dev)))
    return out


def conv1d_backward_data(gout, w, mask=None, gin=None):
    """gin = [mask > 0] * conv^T(gout, w); gout [rows, cout, len]."""
    cout, cin, _ = w.shape
    rows, n = _rows_len(gout, cout, "gout")
    dev = gout.device
    if gin is None:
        gin = torch.empty((rows, cin, n), dtype=torch.float32, device=dev)
    with torch.cuda.device(dev):
        check(lib.fdk_conv1d_backward_data(cin, cout, rows, n, _p(gout, "gout", dev),
                                           _p(w, "w", dev), _p(mask, "mask", dev),
                                           _p(gin, "gin", dev), _stream(dev)))
    return gin


def conv1d_backward_weight(x, gout, gw, gb=None):
    """gw += d<gout, conv(x, w)>/dw, gb += d/db (accumulated)."""
    cout, cin, _ = gw.shape
    rows, n = _rows_len(x, cin, "x")
    dev = x.device
    with torch.cuda.device(dev):
        check(lib.fdk_conv1d_backward_weight(cin, cout, rows, n, _p(x, "x", dev),
                                             _p(gout, "gout", dev), _p(gw, "gw", dev),
                                             _p(gb, "gb", dev), _stream(dev)))
    return gw, gb


def sqerr(a, b, grad=None, grad_scale=None, loss=None):
    """loss += sum (a - b)^2 (device scalar); grad = grad_scale (a - b)."""
    dev = a.device
    n = a.numel()
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
    gs = 2.0 / n if grad_scale is None else float(grad_scale)
    with torch.cuda.device(dev):
        check(lib.fdk_sqerr(n, _p(a, "a"), _p(b, "b", dev), _p(grad, "grad", dev), gs,
                            _p(loss, "loss", dev), _stream(dev)))
    return loss


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    dev = p.device
    with torch.cuda.device(dev):
        check(lib.fdk_adam(p.numel(), _p(p, "p"), _p(g, "g", dev), _p(m, "m", dev),
                           _p(v, "v", dev), float(lr), float(beta1), float(beta2), float(eps),
                           int(t), _stream(dev)))


# ---------------------------------------------------------------- the filter network

def init_params(seed: int, input_std: float = 1.0, residual: bool = True) -> dict:
    """He-normal initialisation (first layer scaled to the input's standard
    deviation); in the residual form the last layer starts at zero."""
    rng = np.random.default_rng(seed)
    p = {
        "w1": rng.standard_normal((CH, 1, K)) * math.sqrt(2.0 / K) / input_std,
        "b1": np.zeros(CH),
        "w2": rng.standard_normal((CH, CH, K)) * math.sqrt(2.0 / (CH * K)),
        "b2": np.zeros(CH),
        "w3": rng.standard_normal((1, CH, K)) * math.sqrt(1.0 / (CH * K)),
        "b3": np.zeros(1),
    }
    if residual:
        p["w3"][:] = 0.0
    return p


class LearnedFilter:
    """Three-layer row filter with its gradient and Adam state on one device."""

    def __init__(self, device="cuda", params: dict | None = None, residual: bool = True,
                 seed: int = 0, input_std: float = 1.0):
        self.device = torch.device(device)
        self.residual = bool(residual)
        self.flat = torch.zeros(N_PARAMS, dtype=torch.float32, device=self.device)
        self.grad = torch.zeros_like(self.flat)
        self.m = torch.zeros_like(self.flat)
        self.v = torch.zeros_like(self.flat)
        self.t = 0
        self.p = self._views(self.flat)
        self.g = self._views(self.grad)
        self.set_params(params if params is not None
                        else init_params(seed, input_std, self.residual))

    @staticmethod
    def _views(buf: torch.Tensor) -> dict:
        out, o = {}, 0
        for name, shape in SHAPES:
            n = int(np.prod(shape))
            out[name] = buf[o:o + n].view(shape)
            o += n
        return out

    def set_params(self, params: dict) -> None:
        for name, shape in SHAPES:
            a = np.asarray(params[name], dtype=np.float32).reshape(shape)
            self.p[name].copy_(torch.from_numpy(a))

    def params_numpy(self) -> dict:
        return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in self.p.items()}

    # -- forward / backward over a stack [np, nh, nw]

    def forward(self, raw: torch.Tensor, scan: dict, np_total: int | None = None,
                keep: bool = False):
        """Filtered stack y [np, nh, nw] of raw line integrals; with keep=True
        also the activations the backward pass needs."""
        npv, nh, nw = raw.shape
        rows = npv * nh
        npt = int(np_total if np_total is not None else npv)
        alpha = scan["arc"] / (2.0 * npt)
        q = cosine_weight(raw, scan).view(rows, 1, nw)
        a1 = conv1d_forward(q, self.p["w1"], self.p["b1"], relu=True)
        a2 = conv1d_forward(a1, self.p["w2"], self.p["b2"], relu=True)
        add = fdk_filter(raw, scan, npt).view(rows, 1, nw) if self.residual else None
        y = conv1d_forward(a2, self.p["w3"], self.p["b3"], add=add, alpha=alpha,
                           out=add)
        y = y.view(npv, nh, nw)
        if not keep:
            del a1, a2
            return y
        return y, (q, a1, a2, alpha)

    def backward(self, gz: torch.Tensor, cache) -> None:
        """Accumulate into self.grad the gradient for dL/dz = gz, z being the
        network output before the alpha scaling ([np, nh, nw])."""
        q, a1, a2, _ = cache
        rows, _, nw = q.shape
        g3 = gz.reshape(rows, 1, nw)
        conv1d_backward_weight(a2, g3, self.g["w3"], self.g["b3"])
        g2 = conv1d_backward_data(g3, self.p["w3"], mask=a2)
        conv1d_backward_weight(a1, g2, self.g["w2"], self.g["b2"])
        g1 = conv1d_backward_data(g2, self.p["w2"], mask=a1)
        del g2
        conv1d_backward_weight(q, g1, self.g["w1"], self.g["b1"])

    def step(self, lr: float, betas=(0.9, 0.999), eps: float = 1e-8) -> None:
        self.t += 1
        adam_step(self.flat, self.grad, self.m, self.v, self.t, lr, betas[0], betas[1], eps)

    # -- reconstruction and training

    def reconstruct(self, raw: torch.Tensor, scan: dict, geom: Geometry,
                    np_total: int | None = None) -> torch.Tensor:
        y = self.forward(raw, scan, np_total)
        vol = torch.zeros(geom.shape, dtype=torch.float32, device=raw.device)
        backproject(vol, y, geom.mats, geom.voxel, geom.centre)
        return vol

    def loss_and_grad(self, raw: torch.Tensor, target: torch.Tensor, scan: dict,
                      geom: Geometry) -> torch.Tensor:
        """Accumulate the gradient of mean((BP(filter(raw)) - target)^2) into
        self.grad; returns the summed squared error as a device scalar."""
        y, cache = self.forward(raw, scan, keep=True)
        alpha = cache[3]
        vol = torch.zeros(geom.shape, dtype=torch.float32, device=raw.device)
        backproject(vol, y, geom.mats, geom.voxel, geom.centre)
        gvol = torch.empty_like(vol)
        # dL/dz = alpha FP(dL/dvol): fold alpha into the loss gradient's scale
        loss = sqerr(vol, target, gvol, grad_scale=alpha * 2.0 / vol.numel())
        del vol, y
        gz = torch.zeros(raw.shape, dtype=torch.float32, device=raw.device)
        forwardproject(gvol, gz, geom.mats, geom.voxel, geom.centre)
        del gvol
        self.backward(gz, cache)
        return loss

    def train_step(self, raw, target, scan, geom, lr, **adam_kw) -> torch.Tensor:
        self.grad.zero_()
        loss = self.loss_and_grad(raw, target, scan, geom)
        self.step(lr, **adam_kw)
        return loss

    # -- checkpoint / resume

    def save(self, path: str, **meta) -> None:
        """Parameters, Adam state and caller metadata (e.g. the next phantom
        index and the data seed) in one .npz (no pickled objects)."""
        np.savez(path, flat=self.flat.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(), t=np.int64(self.t),
                 residual=np.int64(self.residual), meta=np.array(json.dumps(meta)))

    @classmethod
    def load(cls, path: str, device="cuda"):
        z = np.load(path, allow_pickle=False)
        f = cls(device, residual=bool(int(z["residual"])))
        f.flat.copy_(torch.from_numpy(z["flat"]))
        f.m.copy_(torch.from_numpy(z["m"]))
        f.v.copy_(torch.from_numpy(z["v"]))
        f.t = int(z["t"])
        return f, json.loads(str(z["meta"]))
