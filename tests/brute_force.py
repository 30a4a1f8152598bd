"""Brute-force tent-sum back-projection, an independent check of the oracle.

Bilinear interpolation with zero extension equals a sum over *all* detector
pixels of p[r][c] * L(u - c) * L(v - r), where L(t) = max(0, 1 - |t|) is the
tent (hat) function: only the four pixels around (u, v) have non-zero weight,
and pixels that do not exist are simply absent from the sum.  Evaluating that
sum literally needs no floor, fraction or bounds logic, so it shares neither
code nor failure modes with the oracle.  O(n_voxels * np * nh * nw): tiny
problems only.
"""
import numpy as np


def tent(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def voxel_centres(shape, voxel, centre=(0.0, 0.0, 0.0)):
    nz, ny, nx = shape
    dx, dy, dz = voxel
    z = (np.arange(nz) - (nz - 1) / 2.0) * dz + centre[2]
    y = (np.arange(ny) - (ny - 1) / 2.0) * dy + centre[1]
    x = (np.arange(nx) - (nx - 1) / 2.0) * dx + centre[0]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z, np.ones_like(X)], -1)          # [nz,ny,nx,4]


def brute_backproject(proj, mats, shape, voxel, centre=(0.0, 0.0, 0.0)):
    proj = np.asarray(proj, dtype=np.float64)
    npv, nh, nw = proj.shape
    H = voxel_centres(shape, voxel, centre)
    vol = np.zeros(shape)
    cols = np.arange(nw, dtype=np.float64)
    rows = np.arange(nh, dtype=np.float64)
    for s in range(npv):
        q = H @ np.asarray(mats[s], dtype=np.float64).T          # [...,3] = (u w, v w, w)
        w = q[..., 2]
        u = q[..., 0] / w
        v = q[..., 1] / w
        wu = tent(u[..., None] - cols)                            # [...,nw]
        wv = tent(v[..., None] - rows)                            # [...,nh]
        val = np.einsum("...r,rc,...c->...", wv, proj[s], wu)
        vol += val / (w * w)
    return vol


def brute_forwardproject(vol, mats, nh, nw, voxel, centre=(0.0, 0.0, 0.0)):
    """Transpose of ``brute_backproject`` written the same literal way."""
    vol = np.asarray(vol, dtype=np.float64)
    H = voxel_centres(vol.shape, voxel, centre)
    cols = np.arange(nw, dtype=np.float64)
    rows = np.arange(nh, dtype=np.float64)
    out = np.zeros((len(mats), nh, nw))
    for s in range(len(mats)):
        q = H @ np.asarray(mats[s], dtype=np.float64).T
        w = q[..., 2]
        u = q[..., 0] / w
        v = q[..., 1] / w
        wu = tent(u[..., None] - cols)
        wv = tent(v[..., None] - rows)
        a = (vol / (w * w)).reshape(-1)
        out[s] = (wv.reshape(-1, nh) * a[:, None]).T @ wu.reshape(-1, nw)
    return out
