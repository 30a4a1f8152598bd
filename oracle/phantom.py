"""Analytic line integrals of random-ellipsoid phantoms (oracle side, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper reconstructs projections that RTK's forward projector synthesised
from the RabbitCT volume (Section 4.2) and states that the arithmetic does not
depend on the content.  Neither is available here, so test projections are
exact line integrals through seeded ellipsoids.

Ellipsoid rows (float64, 16 values):
  [cx, cy, cz, a, b, c, R00..R22 (row-major), rho]
The solid is { X : |diag(a,b,c)^-1 R^T (X - c0)| <= 1 } with density rho;
overlapping ellipsoids add.  The columns of R are the ellipsoid's axes.

Ray of pixel (r, c) of view s (same scanner frame as ``geometry.py``): from
the source S = sod (cos, sin, 0) to the pixel centre
  C + (c - cu) du e_u + (r - cv) dv e_v,  C = -(sdd - sod)(cos, sin, 0).
In the ellipsoid's unit-sphere frame the ray S' + t d' meets the sphere where
|S' + t d'|^2 = 1; the chord between the two roots is 2 sqrt(b'^2 - a'c') / a'
in units of t, i.e. times |d| in millimetres.
"""
from __future__ import annotations

import numpy as np

from .geometry import view_angles


def _unit_frame(ell):
    c0 = ell[:, 0:3]
    axes = ell[:, 3:6]
    R = ell[:, 6:15].reshape(-1, 3, 3)
    rho = ell[:, 15]
    # T maps world offsets into the unit-sphere frame: T = diag(1/axes) R^T
    T = np.transpose(R, (0, 2, 1)) / axes[:, :, None]
    return c0, T, rho


def line_integrals(ell, scan, np_views, nh, nw, views=None, rows=None):
    """[len(views), len(rows), nw] float64 line integrals through ``ell``."""
    ell = np.asarray(ell, dtype=np.float64).reshape(-1, 16)
    th_all = view_angles(np_views, scan["arc"], scan["theta0"])
    views = np.arange(np_views) if views is None else np.asarray(views)
    rows = np.arange(nh) if rows is None else np.asarray(rows)
    sod, sdd, du, dv = scan["sod"], scan["sdd"], scan["du"], scan["dv"]
    cu = 0.5 * (nw - 1) + scan["u_off"]
    cv = 0.5 * (nh - 1) + scan["v_off"]
    c0, T, rho = _unit_frame(ell)
    out = np.zeros((len(views), len(rows), nw), dtype=np.float64)
    cc = (np.arange(nw, dtype=np.float64) - cu) * du           # u_mm per column
    rr = (rows.astype(np.float64) - cv) * dv                     # v_mm per row
    for a, s in enumerate(views):
        th = th_all[s]
        ct, st = np.cos(th), np.sin(th)
        S = np.array([sod * ct, sod * st, 0.0])
        C = np.array([-(sdd - sod) * ct, -(sdd - sod) * st, 0.0])
        eu = np.array([-st, ct, 0.0])
        # pixel centres [len(rows), nw, 3] and ray directions d = P - S
        P = (C[None, None, :] + cc[None, :, None] * eu[None, None, :]
             + rr[:, None, None] * np.array([0.0, 0.0, 1.0])[None, None, :])
        d = P - S[None, None, :]
        dn = np.sqrt((d * d).sum(-1))
        acc = np.zeros((len(rows), nw))
        for e in range(len(ell)):
            Sp = T[e] @ (S - c0[e])
            dp = d @ T[e].T
            aa = (dp * dp).sum(-1)
            bb = dp @ Sp
            cc2 = Sp @ Sp - 1.0
            disc = bb * bb - aa * cc2
            hit = disc > 0
            chord = np.where(hit, 2.0 * np.sqrt(np.where(hit, disc, 0.0)) / aa, 0.0)
            acc += rho[e] * chord * dn
        out[a] = acc
    return out


def voxelize(ell, shape, voxel, centre=(0.0, 0.0, 0.0), supersample=1):
    """Density sampled at voxel centres (or averaged over ``supersample``^3
    sub-points per voxel), float64 [nz, ny, nx]."""
    ell = np.asarray(ell, dtype=np.float64).reshape(-1, 16)
    nz, ny, nx = shape
    dx, dy, dz = voxel
    n = supersample
    off = (np.arange(n) + 0.5) / n - 0.5
    c0, T, rho = _unit_frame(ell)
    out = np.zeros(shape, dtype=np.float64)
    xs = (np.arange(nx) - 0.5 * (nx - 1)) * dx + centre[0]
    ys = (np.arange(ny) - 0.5 * (ny - 1)) * dy + centre[1]
    zs = (np.arange(nz) - 0.5 * (nz - 1)) * dz + centre[2]
    for ox in off:
        for oy in off:
            for oz in off:
                Z, Y, X = np.meshgrid(zs + oz * dz, ys + oy * dy, xs + ox * dx, indexing="ij")
                pts = np.stack([X, Y, Z], -1)
                for e in range(len(ell)):
                    q = (pts - c0[e]) @ T[e].T
                    out += rho[e] * ((q * q).sum(-1) <= 1.0)
    return out / float(n ** 3)
