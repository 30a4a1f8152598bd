"""Differentiable back-projection: torch.autograd.Functions over the C ABI.

BackProject.forward is ``fdk_backproject``; its backward is the exact
transpose, ``fdk_forwardproject`` (voxel-driven splat with the same bilinear
weights and 1/w^2), so gradients with respect to the projections are exact up
to FP32 rounding.  ForwardProject is the mirror pair.  Batched inputs
([B, np, nh, nw] / [B, nz, ny, nx]) are processed one item per library call.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import backproject, forwardproject, scan_matrices


@dataclass
class Geometry:
    """Volume grid and per-view matrices of one scan."""
    shape: tuple                 # (nz, ny, nx)
    voxel: tuple                 # (dx, dy, dz) mm
    mats: np.ndarray             # [np, 3, 4] float64, world mm -> (u w, v w, w)
    nh: int
    nw: int
    centre: tuple = (0.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)

    @property
    def np(self) -> int:
        return int(self.mats.shape[0])

    @classmethod
    def circular(cls, shape, voxel, scan: dict, np_views: int, nh: int, nw: int,
                 centre=(0.0, 0.0, 0.0)):
        return cls(tuple(shape), tuple(voxel), scan_matrices(scan, np_views, nh, nw), nh, nw,
                   tuple(centre))


def _bp(proj: torch.Tensor, g: Geometry) -> torch.Tensor:
    vol = torch.zeros(g.shape, dtype=torch.float32, device=proj.device)
    backproject(vol, proj.contiguous(), g.mats, g.voxel, g.centre)
    return vol


def _fp(vol: torch.Tensor, g: Geometry) -> torch.Tensor:
    proj = torch.zeros((g.np, g.nh, g.nw), dtype=torch.float32, device=vol.device)
    forwardproject(vol.contiguous(), proj, g.mats, g.voxel, g.centre)
    return proj


def _batched(fn, x: torch.Tensor, g: Geometry, item_ndim: int) -> torch.Tensor:
    if x.dim() == item_ndim:
        return fn(x, g)
    return torch.stack([fn(x[b], g) for b in range(x.shape[0])])


class BackProject(torch.autograd.Function):
    """vol = BP(proj); d loss / d proj = FP(d loss / d vol)."""

    @staticmethod
    def forward(ctx, proj: torch.Tensor, geom: Geometry):
        if proj.dtype != torch.float32:
            raise TypeError("BackProject differentiates float32 projections")
        ctx.geom = geom
        return _batched(_bp, proj, geom, 3)

    @staticmethod
    def backward(ctx, grad_vol: torch.Tensor):
        return _batched(_fp, grad_vol, ctx.geom, 3), None


class ForwardProject(torch.autograd.Function):
    """proj = FP(vol); d loss / d vol = BP(d loss / d proj)."""

    @staticmethod
    def forward(ctx, vol: torch.Tensor, geom: Geometry):
        if vol.dtype != torch.float32:
            raise TypeError("ForwardProject differentiates float32 volumes")
        ctx.geom = geom
        return _batched(_fp, vol, geom, 3)

    @staticmethod
    def backward(ctx, grad_proj: torch.Tensor):
        return _batched(_bp, grad_proj, ctx.geom, 3), None


def back_project(proj: torch.Tensor, geom: Geometry) -> torch.Tensor:
    return BackProject.apply(proj, geom)


def forward_project(vol: torch.Tensor, geom: Geometry) -> torch.Tensor:
    return ForwardProject.apply(vol, geom)
