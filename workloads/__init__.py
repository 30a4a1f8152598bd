"""Seeded synthetic workloads shared by the tests, the smoke check and the bench.

This module only draws random numbers and states scan shapes; it contains none
of the back-projection, filtering or forward-projection arithmetic, so both
the FP64 oracle and the HIP path can consume what it produces.

Scan shapes (volume / views / detector / distances) follow the five workloads
the repository is measured on; the paper's own problem table (Table 3) uses
256^2-1024^2 x 512 views -> 256^3-1300^3 with RabbitCT-derived data, which is
not available, so seeded random-ellipsoid phantoms stand in (the paper notes
that the arithmetic does not depend on the content, Section 4.2).

Conventions: volume arrays are [nz][ny][nx] (x fastest), projection stacks
[np][nh][nw] (u along nw fastest), voxel sizes and distances in millimetres,
view angles theta_s = theta0 + arc * s / np over a full circle.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _scan(sod, sdd, du, dv, arc=TWO_PI, theta0=0.0, u_off=0.0, v_off=0.0):
    return dict(sod=float(sod), sdd=float(sdd), du=float(du), dv=float(dv), arc=float(arc),
                theta0=float(theta0), u_off=float(u_off), v_off=float(v_off))


# name -> workload description
CONFIGS = {
    # 64^3 / 1 mm, 64 views, 128^2 / 1 mm, SOD 500, SDD 1000, 10 ellipsoids
    "c1": dict(shape=(64, 64, 64), voxel=(1.0, 1.0, 1.0), np=64, nh=128, nw=128,
               scan=_scan(500.0, 1000.0, 1.0, 1.0), n_ell=10, axes=(2.0, 20.0), seed=1000,
               dtype="f32"),
    # 512^3 / 1 mm, 1024 views, 1024^2 / 1 mm, SOD 750, SDD 1200, 40 ellipsoids
    "c2": dict(shape=(512, 512, 512), voxel=(1.0, 1.0, 1.0), np=1024, nh=1024, nw=1024,
               scan=_scan(750.0, 1200.0, 1.0, 1.0), n_ell=40, axes=(16.0, 160.0), seed=2000,
               dtype="f32"),
    # 1024^3 / 0.5 mm, 2048 views, 2048^2 / 0.5 mm (FP16 storage), 60 ellipsoids
    "c3": dict(shape=(1024, 1024, 1024), voxel=(0.5, 0.5, 0.5), np=2048, nh=2048, nw=2048,
               scan=_scan(750.0, 1200.0, 0.5, 0.5), n_ell=60, axes=(16.0, 160.0), seed=3000,
               dtype="f16"),
    # 8 x 256^3 / 0.25 mm, 360 views, 384^2 / 0.333 mm (differentiation)
    "c4": dict(shape=(256, 256, 256), voxel=(0.25, 0.25, 0.25), np=360, nh=384, nw=384,
               scan=_scan(500.0, 1000.0, 1.0 / 3.0, 1.0 / 3.0), n_ell=10, axes=(2.0, 20.0),
               seed=4000, batch=8, dtype="f32"),
    # 256^3 / 0.25 mm, 90 sparse views vs 720, 512^2 / 0.25 mm (learned filter)
    "c5": dict(shape=(256, 256, 256), voxel=(0.25, 0.25, 0.25), np=90, np_target=720,
               nh=512, nw=512, scan=_scan(500.0, 1000.0, 0.25, 0.25), n_ell=10,
               axes=(2.0, 20.0), seed=5000, n_phantoms=2000, dtype="f32"),
}


def fov_mm(cfg) -> float:
    """Edge length of the (cubic) field of view in mm."""
    nz, ny, nx = cfg["shape"]
    return float(nx * cfg["voxel"][0])


def draw_ellipsoids(seed: int, n: int, fov: float, axes=(2.0, 20.0),
                    density=(0.1, 1.0)) -> np.ndarray:
    """n ellipsoids as rows [cx,cy,cz, a,b,c, R (9, row-major), rho], float64.

    Centres uniform in the inner 80% of the FOV cube, semi-axes uniform in
    ``axes`` (mm), densities uniform in ``density``, rotations uniform on SO(3)
    (unit quaternion from a normalised 4-D Gaussian)."""
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(-0.4 * fov, 0.4 * fov, size=(n, 3))
    ax = rng.uniform(axes[0], axes[1], size=(n, 3))
    q = rng.standard_normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
        2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
        2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], axis=1)
    rho = rng.uniform(density[0], density[1], size=(n, 1))
    return np.concatenate([c0, ax, R, rho], axis=1)


def config_ellipsoids(cfg, index: int = 0) -> np.ndarray:
    """Phantom ``index`` of a workload: seed = workload seed + index."""
    return draw_ellipsoids(cfg["seed"] + index, cfg["n_ell"], fov_mm(cfg), cfg["axes"])


def gaussian(seed: int, shape, dtype=np.float32) -> np.ndarray:
    """Seeded standard-normal array (PCG64)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=shape, dtype=np.float64 if dtype == np.float64 else np.float32)


def device_f16_stack(seed: int, shape, device="cuda"):
    """Seeded binary16 projection stack generated on the GPU (for sizes where
    a host generator would be too slow): standard-normal values drawn by
    torch's counter-based generator and rounded to binary16, plus one
    power-of-two scale per view, 2^-(s mod 7).  Returned as (torch float16
    [np, nh, nw], torch float32 [np]) on ``device``; both are inputs of the
    stored (binary16 + scale) form, used unchanged by every consumer."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    h = torch.empty(tuple(shape), dtype=torch.float16, device=device)
    for v0 in range(0, shape[0], 64):      # bounded float32 temporaries
        n = min(64, shape[0] - v0)
        h[v0:v0 + n] = torch.randn((n,) + tuple(shape[1:]), generator=g, device=device).half()
    s = torch.tensor([2.0 ** -(v % 7) for v in range(shape[0])], dtype=torch.float32,
                     device=device)
    return h, s


def shrink(cfg, shape=None, np_views=None, nh=None, nw=None):
    """A copy of ``cfg`` with smaller sizes (same physical pitch and distances)."""
    out = dict(cfg)
    if shape is not None:
        out["shape"] = tuple(shape)
    if np_views is not None:
        out["np"] = int(np_views)
    if nh is not None:
        out["nh"] = int(nh)
    if nw is not None:
        out["nw"] = int(nw)
    return out
