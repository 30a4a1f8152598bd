"""Detector windows of a voxel sub-block (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

To check a sub-block of a large reconstruction against the FP64 oracle one
only needs, per view, the detector pixels the block's voxels reach.  Under a
pinhole matrix with positive depth over the block, the detector coordinates
u = (row0 . X) / (row2 . X) and v = (row1 . X) / (row2 . X) are monotone along
each axis of the block (a ratio of affine functions with a denominator of
fixed sign), so their extremes over the block are taken at its 8 corner
voxels.  The tent weights of a point (u, v) are non-zero only for the pixels
floor(u), floor(u) + 1 and floor(v), floor(v) + 1, so the window
[floor(vmin), floor(vmax) + 1] x [floor(umin), floor(umax) + 1], widened by a
safety margin, holds every pixel the block needs.  ``oracle.backproject_block``
raises if that were ever not so.
"""
from __future__ import annotations

import numpy as np


def block_windows(mats, shape, voxel, box, centre=(0.0, 0.0, 0.0), margin=1):
    """Per-view windows for box = ((k0,k1),(j0,j1),(i0,i1)) of a volume of
    ``shape`` ([nz,ny,nx]) under world matrices ``mats`` ([np,3,4]).

    Returns (origin [np,2] int64 of (first row, first column), wr, wc): the
    common window size is the largest over the views."""
    mats = np.asarray(mats, dtype=np.float64)
    nz, ny, nx = shape
    (k0, k1), (j0, j1), (i0, i1) = box
    idx = []
    for k in (k0, k1 - 1):
        for j in (j0, j1 - 1):
            for i in (i0, i1 - 1):
                idx.append((i, j, k))
    idx = np.asarray(idx, dtype=np.float64)
    dims = np.array([nx, ny, nz], dtype=np.float64)
    X = (idx - 0.5 * (dims - 1.0)) * np.asarray(voxel, dtype=np.float64) + np.asarray(centre)
    Xh = np.concatenate([X, np.ones((len(X), 1))], axis=1)          # [8,4]
    h = np.einsum("sab,nb->sna", mats, Xh)                          # [np,8,3]
    if not np.all(h[..., 2] > 0):
        raise ValueError("depth must be positive over the block")
    u = h[..., 0] / h[..., 2]
    v = h[..., 1] / h[..., 2]
    r0 = np.floor(v.min(axis=1)) - margin
    r1 = np.floor(v.max(axis=1)) + 1 + margin
    c0 = np.floor(u.min(axis=1)) - margin
    c1 = np.floor(u.max(axis=1)) + 1 + margin
    wr = int((r1 - r0).max()) + 1
    wc = int((c1 - c0).max()) + 1
    origin = np.stack([r0, c0], axis=1).astype(np.int64)
    return origin, wr, wc


def cut_windows(stack, origin, wr, wc):
    """Windows of a whole host stack [np,nh,nw] (pixels off the detector are
    zero): [np,wr,wc] of the stack's dtype."""
    npv, nh, nw = stack.shape
    out = np.zeros((npv, wr, wc), dtype=stack.dtype)
    for s in range(npv):
        r0, c0 = int(origin[s, 0]), int(origin[s, 1])
        ra, rb = max(r0, 0), min(r0 + wr, nh)
        ca, cb = max(c0, 0), min(c0 + wc, nw)
        if ra < rb and ca < cb:
            out[s, ra - r0:rb - r0, ca - c0:cb - c0] = stack[s, ra:rb, ca:cb]
    return out


def cut_windows_device(stack, origin, wr, wc):
    """The same for a torch tensor [np,nh,nw] (on any device): gathers the
    windows where the stack lives and returns them as a host numpy array."""
    import torch
    npv, nh, nw = stack.shape
    dev = stack.device
    org = torch.as_tensor(np.asarray(origin), dtype=torch.int64, device=dev)
    rows = org[:, 0:1] + torch.arange(wr, device=dev)[None, :]          # [np,wr]
    cols = org[:, 1:2] + torch.arange(wc, device=dev)[None, :]          # [np,wc]
    rin = (rows >= 0) & (rows < nh)
    cin = (cols >= 0) & (cols < nw)
    s = torch.arange(npv, device=dev)[:, None, None]
    got = stack[s, rows.clamp(0, nh - 1)[:, :, None], cols.clamp(0, nw - 1)[:, None, :]]
    keep = rin[:, :, None] & cin[:, None, :]
    got = torch.where(keep, got, torch.zeros((), dtype=stack.dtype, device=dev))
    return got.cpu().numpy()
