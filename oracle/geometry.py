"""Closed-form projection matrices of a circular cone-beam orbit (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper leaves the construction of the 3x4 pinhole matrix to the literature
(Section 2.1.1) and only fixes that the detector's V-axis is parallel to the
rotation axis Z, and that the depth is d - x cos(theta) - y sin(theta)
(Section 3.1.2).  The reading used here, written from the pinhole model:

  view angle     theta_s = theta0 + arc * s / np      (no repeated endpoint)
  source         S = sod (cos, sin, 0)
  detector axes  e_u = (-sin, cos, 0), e_v = (0, 0, 1), centre on the far side
  depth          U = sod - (x cos + y sin);   w = U / sod  (1 at the isocentre)
  pixel          u = sdd * s_u / (U du) + cu,  v = sdd * z / (U dv) + cv
                 s_u = -x sin + y cos,  cu = (nw-1)/2 + u_off,  cv = (nh-1)/2 + v_off

Multiplying u and v by w gives rows that are affine in (x, y, z):
  row0 = [-k sin/du - cu cos/sod,  k cos/du - cu sin/sod,  0,     cu]
  row1 = [-cv cos/sod,            -cv sin/sod,             k/dv,  cv]
  row2 = [-cos/sod,               -sin/sod,                0,     1 ]
with k = sdd / sod.  Entries (0,2) and (2,2) are zero: u and w do not depend
on z, which is what lets a back-projector reuse them along a voxel column.
"""
from __future__ import annotations

import numpy as np


def view_angles(np_views: int, arc: float = 2.0 * np.pi, theta0: float = 0.0) -> np.ndarray:
    s = np.arange(np_views, dtype=np.float64)
    return theta0 + arc * s / float(np_views)


def circular_matrices(np_views, arc, theta0, sod, sdd, nh, nw, du, dv,
                      u_off=0.0, v_off=0.0) -> np.ndarray:
    """World-mm -> homogeneous pixel matrices, [np, 3, 4] float64."""
    th = view_angles(np_views, arc, theta0)
    c, s = np.cos(th), np.sin(th)
    k = sdd / sod
    cu = 0.5 * (nw - 1) + u_off
    cv = 0.5 * (nh - 1) + v_off
    m = np.zeros((np_views, 3, 4), dtype=np.float64)
    m[:, 0, 0] = -k * s / du - cu * c / sod
    m[:, 0, 1] = k * c / du - cu * s / sod
    m[:, 0, 3] = cu
    m[:, 1, 0] = -cv * c / sod
    m[:, 1, 1] = -cv * s / sod
    m[:, 1, 2] = k / dv
    m[:, 1, 3] = cv
    m[:, 2, 0] = -c / sod
    m[:, 2, 1] = -s / sod
    m[:, 2, 3] = 1.0
    return m


def scan_matrices(scan: dict, np_views: int, nh: int, nw: int) -> np.ndarray:
    return circular_matrices(np_views, scan["arc"], scan["theta0"], scan["sod"], scan["sdd"],
                             nh, nw, scan["du"], scan["dv"], scan["u_off"], scan["v_off"])


def index_matrices(mats, shape, voxel, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Compose world-mm matrices with the voxel-index -> world map.

    Voxel (i, j, k) sits at ((i-(nx-1)/2) dx + cx, ...); the result maps
    (i, j, k, 1) straight to homogeneous pixels, the form Listing 1 uses."""
    nz, ny, nx = shape
    dx, dy, dz = voxel
    cx, cy, cz = centre
    V = np.array([[dx, 0, 0, cx - 0.5 * (nx - 1) * dx],
                  [0, dy, 0, cy - 0.5 * (ny - 1) * dy],
                  [0, 0, dz, cz - 0.5 * (nz - 1) * dz],
                  [0, 0, 0, 1.0]], dtype=np.float64)
    return np.einsum("sab,bc->sac", np.asarray(mats, dtype=np.float64), V)
