"""Pins of the FP64 oracle against what the paper and the mathematics fix.

The paper prints no worked numbers, so every pin here is mathematical: brute
force on tiny non-cubic problems, closed forms, invariants of the geometry,
the adjoint identity and analytic phantoms.  Each pin is chosen so that a
plausible slip in the oracle (a swapped u/v, a dropped weight, a wrong sign in
the matrix, truncation instead of floor, a missing zero extension) fails.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import geometry as og
from oracle import phantom as oph
from brute_force import brute_backproject, brute_forwardproject, tent
import workloads as wl


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


SCAN_TINY = dict(sod=12.0, sdd=30.0, du=1.3, dv=0.9, arc=2 * math.pi, theta0=0.3,
                 u_off=0.4, v_off=-0.35)


def tiny_problem(seed=1, np_views=5, shape=(3, 4, 5), nh=6, nw=7, voxel=(1.1, 0.8, 1.7)):
    """Non-cubic volume and non-square detector so that axis swaps show up;
    a magnification that pushes corner voxels off the detector."""
    mats = og.circular_matrices(np_views, SCAN_TINY["arc"], SCAN_TINY["theta0"],
                                SCAN_TINY["sod"], SCAN_TINY["sdd"], nh, nw,
                                SCAN_TINY["du"], SCAN_TINY["dv"], SCAN_TINY["u_off"],
                                SCAN_TINY["v_off"])
    proj = wl.gaussian(seed, (np_views, nh, nw))
    return proj, mats, shape, voxel


# ---------------------------------------------------------------- brute force

def test_brute_force_tiny_circular():
    proj, mats, shape, voxel = tiny_problem()
    centre = (0.3, -0.2, 0.5)
    ref = brute_backproject(proj, mats, shape, voxel, centre)
    got = oracle.backproject(proj, mats, shape, voxel, centre)
    assert rel(got, ref) < 1e-13


def test_brute_force_generic_matrices():
    """Matrix mode must handle any 3x4 matrix, including k-dependent depth."""
    rng = np.random.default_rng(7)
    shape, voxel = (4, 3, 5), (1.0, 1.2, 0.9)
    nh, nw, npv = 6, 8, 3
    mats = np.zeros((npv, 3, 4))
    for s in range(npv):
        mats[s, 0] = [0.9 + 0.1 * s, 0.2, 0.1, 3.5]
        mats[s, 1] = [-0.1, 0.8, 0.7, 2.7]
        mats[s, 2] = [0.01, -0.02, 0.03, 1.0]
        mats[s] += 0.02 * rng.standard_normal((3, 4))
    proj = wl.gaussian(11, (npv, nh, nw))
    ref = brute_backproject(proj, mats, shape, voxel)
    got = oracle.backproject(proj, mats, shape, voxel)
    assert rel(got, ref) < 1e-13


def test_zero_extension_is_exercised():
    """With the tiny geometry some taps are off-detector: the brute sum and
    the oracle agree there too, and a clamped (edge-replicating) reading would
    differ."""
    proj, mats, shape, voxel = tiny_problem()
    ones = np.ones_like(proj)
    got = oracle.backproject(ones, mats, shape, voxel)
    # weight sum with every pixel present = sum 1/w^2 only where all taps exist
    ref = brute_backproject(ones, mats, shape, voxel)
    assert rel(got, ref) < 1e-13
    H = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1)
    full = np.zeros(shape)
    for s in range(len(mats)):
        M = og.index_matrices(mats[s:s + 1], shape, voxel)[0]
        q = np.stack([H[..., 2], H[..., 1], H[..., 0], np.ones(shape)], -1) @ M.T
        full += 1.0 / q[..., 2] ** 2
    assert np.any(np.abs(got - full) > 1e-6), "test geometry never leaves the detector"


# ------------------------------------------------------------ delta projection

def test_delta_projection_hand_voxels():
    npv, nh, nw = 3, 6, 7
    shape, voxel = (3, 4, 5), (1.1, 0.8, 1.7)
    mats = tiny_problem(np_views=npv)[1]
    r0, c0 = 2, 3
    proj = np.zeros((npv, nh, nw), dtype=np.float32)
    proj[:, r0, c0] = 1.0
    vol = oracle.backproject(proj, mats, shape, voxel)
    th = og.view_angles(npv, SCAN_TINY["arc"], SCAN_TINY["theta0"])
    for (k, j, i) in [(1, 1, 2), (0, 3, 4), (2, 0, 0), (1, 2, 1)]:
        X = np.array([[(i - 2.0) * voxel[0], (j - 1.5) * voxel[1], (k - 1.0) * voxel[2]]])
        expect = 0.0
        for s in range(npv):
            u, v, w = oracle.project_points(th[s], SCAN_TINY, nh, nw, X)[0]
            expect += tent(u - c0) * tent(v - r0) / (w * w)
        assert abs(vol[k, j, i] - expect) <= 1e-13 * max(1.0, abs(expect))


# ------------------------------------------------------------ closed forms

def test_affine_projection_closed_form():
    """p_s[r][c] = a_s c + b_s r + g_s is reproduced exactly by bilinear
    interpolation wherever all four taps exist: vol = sum (a u + b v + g)/w^2."""
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(9, 10, 11), np_views=12, nh=40, nw=48)
    scan = cfg["scan"]
    mats = og.scan_matrices(scan, cfg["np"], cfg["nh"], cfg["nw"])
    rng = np.random.default_rng(3)
    a, b, g = rng.uniform(-1, 1, (3, cfg["np"]))
    rr, cc = np.meshgrid(np.arange(cfg["nh"]), np.arange(cfg["nw"]), indexing="ij")
    proj = (a[:, None, None] * cc + b[:, None, None] * rr + g[:, None, None]).astype(np.float64)
    proj32 = proj.astype(np.float32)
    vol = oracle.backproject(proj32, mats, cfg["shape"], cfg["voxel"])
    H = np.stack(np.meshgrid(*[np.arange(n) for n in cfg["shape"]], indexing="ij"), -1)
    nz, ny, nx = cfg["shape"]
    X = np.stack([(H[..., 2] - (nx - 1) / 2) * cfg["voxel"][0],
                  (H[..., 1] - (ny - 1) / 2) * cfg["voxel"][1],
                  (H[..., 0] - (nz - 1) / 2) * cfg["voxel"][2], np.ones(cfg["shape"])], -1)
    expect = np.zeros(cfg["shape"])
    inside = np.ones(cfg["shape"], dtype=bool)
    p32 = proj32.astype(np.float64)
    for s in range(cfg["np"]):
        q = X @ mats[s].T
        w = q[..., 2]
        u, v = q[..., 0] / w, q[..., 1] / w
        inside &= (u >= 0) & (u <= cfg["nw"] - 1) & (v >= 0) & (v <= cfg["nh"] - 1)
        # the float32-rounded plane is still affine only up to rounding; use the
        # exact values at the 4 taps through the plane's coefficients
        expect += (a[s] * u + b[s] * v + g[s]) / (w * w)
    assert inside.all()
    err = np.abs(vol - expect).max() / np.abs(expect).max()
    assert err < 1e-6   # float32 storage of the affine plane
    # exact version with an exactly representable plane (dyadic coefficients)
    a2 = np.round(a * 64) / 64
    b2 = np.round(b * 64) / 64
    g2 = np.round(g * 64) / 64
    proj2 = (a2[:, None, None] * cc + b2[:, None, None] * rr + g2[:, None, None]).astype(np.float32)
    assert np.array_equal(proj2.astype(np.float64),
                          a2[:, None, None] * cc + b2[:, None, None] * rr + g2[:, None, None])
    vol2 = oracle.backproject(proj2, mats, cfg["shape"], cfg["voxel"])
    expect2 = np.zeros(cfg["shape"])
    for s in range(cfg["np"]):
        q = X @ mats[s].T
        w = q[..., 2]
        expect2 += (a2[s] * q[..., 0] / w + b2[s] * q[..., 1] / w + g2[s]) / (w * w)
    assert np.abs(vol2 - expect2).max() <= 1e-12 * np.abs(expect2).max()


def test_isocentre_constant_projection():
    """Odd dims, centred volume: the centre voxel is the isocentre, w = 1 in
    every view, so a constant projection gamma back-projects to np * gamma."""
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(5, 7, 9), np_views=17, nh=33, nw=31)
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    gamma = 0.625
    proj = np.full((cfg["np"], cfg["nh"], cfg["nw"]), gamma, dtype=np.float32)
    vol = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"])
    assert abs(vol[2, 3, 4] - cfg["np"] * gamma) < 1e-12
    # constant projection elsewhere: weight sum gamma * sum_s 1/w_s^2
    th = og.view_angles(cfg["np"])
    x, y = 1.0, -2.0                                     # voxel (i=5, j=1) at k=2
    U = cfg["scan"]["sod"] - (x * np.cos(th) + y * np.sin(th))
    expect = gamma * np.sum((cfg["scan"]["sod"] / U) ** 2)
    assert abs(vol[2, 1, 5] - expect) < 1e-12 * expect


# ------------------------------------------------------------ geometry helper

def test_geometry_invariants():
    scan = dict(SCAN_TINY, u_off=0.0, v_off=0.0)
    nh, nw, npv = 20, 24, 8
    mats = og.circular_matrices(npv, scan["arc"], scan["theta0"], scan["sod"], scan["sdd"],
                                nh, nw, scan["du"], scan["dv"])
    assert np.all(mats[:, 0, 2] == 0.0) and np.all(mats[:, 2, 2] == 0.0)
    iso = mats @ np.array([0, 0, 0, 1.0])
    np.testing.assert_allclose(iso[:, 0] / iso[:, 2], (nw - 1) / 2, atol=1e-12)
    np.testing.assert_allclose(iso[:, 1] / iso[:, 2], (nh - 1) / 2, atol=1e-12)
    np.testing.assert_allclose(iso[:, 2], 1.0, atol=1e-15)
    for z in (-3.0, 1.7):
        q = mats @ np.array([0, 0, z, 1.0])
        np.testing.assert_allclose(q[:, 0] / q[:, 2], (nw - 1) / 2, atol=1e-12)
        np.testing.assert_allclose(q[:, 1] / q[:, 2],
                                   (nh - 1) / 2 + z * scan["sdd"] / (scan["sod"] * scan["dv"]),
                                   atol=1e-12)
    # symmetric pair (Section 3.1.2): voxels mirrored in z land mirrored in v
    rng = np.random.default_rng(5)
    for _ in range(5):
        x, y, z = rng.uniform(-3, 3, 3)
        qa = mats @ np.array([x, y, z, 1.0])
        qb = mats @ np.array([x, y, -z, 1.0])
        np.testing.assert_allclose(qa[:, 1] / qa[:, 2] + qb[:, 1] / qb[:, 2], nh - 1, atol=1e-12)


def test_matrix_vs_ray_plane_projection():
    """The closed-form matrices agree with the ray/plane intersection."""
    scan = SCAN_TINY
    nh, nw, npv = 20, 24, 7
    mats = og.circular_matrices(npv, scan["arc"], scan["theta0"], scan["sod"], scan["sdd"],
                                nh, nw, scan["du"], scan["dv"], scan["u_off"], scan["v_off"])
    th = og.view_angles(npv, scan["arc"], scan["theta0"])
    pts = np.random.default_rng(9).uniform(-4, 4, (50, 3))
    for s in range(npv):
        uvw = oracle.project_points(th[s], scan, nh, nw, pts)
        q = np.concatenate([pts, np.ones((50, 1))], 1) @ mats[s].T
        np.testing.assert_allclose(q[:, 0] / q[:, 2], uvw[:, 0], atol=1e-11)
        np.testing.assert_allclose(q[:, 1] / q[:, 2], uvw[:, 1], atol=1e-11)
        np.testing.assert_allclose(q[:, 2], uvw[:, 2], atol=1e-13)


def test_geometry_mode_equals_matrix_mode():
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(12, 10, 14), np_views=9, nh=48, nw=40)
    scan = dict(cfg["scan"], theta0=0.2, u_off=1.25, v_off=-0.5)
    mats = og.scan_matrices(scan, cfg["np"], cfg["nh"], cfg["nw"])
    proj = wl.gaussian(21, (cfg["np"], cfg["nh"], cfg["nw"]))
    centre = (0.5, -1.0, 2.0)
    a = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"], centre)
    b = oracle.backproject_geometry(proj, cfg["shape"], cfg["voxel"], scan, centre)
    assert rel(a, b) < 1e-12


def test_hoisted_equals_plain():
    """Algorithm-1 order (u, w hoisted per column) equals Listing-1 order."""
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(11, 9, 10), np_views=13, nh=40, nw=44)
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    proj = wl.gaussian(22, (cfg["np"], cfg["nh"], cfg["nw"]))
    a = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"])
    b = oracle.backproject_hoisted(proj, mats, cfg["shape"], cfg["voxel"])
    assert rel(a, b) < 1e-13


def test_points_and_block_equal_full():
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(8, 9, 10), np_views=6, nh=30, nw=32)
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    proj = wl.gaussian(23, (cfg["np"], cfg["nh"], cfg["nw"]))
    full = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"])
    ijk = np.array([[0, 0, 0], [9, 8, 7], [3, 4, 5], [5, 1, 2]])
    pts = oracle.backproject_points(proj, mats, cfg["shape"], cfg["voxel"], ijk)
    np.testing.assert_allclose(pts, full[ijk[:, 2], ijk[:, 1], ijk[:, 0]], rtol=1e-14, atol=0)
    blk = oracle.backproject_block(proj, mats, cfg["shape"], cfg["voxel"], ((2, 6), (1, 8), (3, 9)))
    np.testing.assert_array_equal(blk, full[2:6, 1:8, 3:9])


def test_block_from_view_windows():
    """A sub-block computed from per-view windows of the stack equals the
    same block from whole views, bit for bit (same pixels, same order), at a
    corner whose windows hang over the detector edges; a window one column
    too narrow is refused rather than read as zeros."""
    from oracle import window as owin
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(12, 11, 13), np_views=7, nh=24, nw=26)
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    proj = wl.gaussian(29, (cfg["np"], cfg["nh"], cfg["nw"]))
    for box in (((0, 5), (0, 4), (0, 6)), ((4, 9), (3, 8), (5, 11)), ((7, 12), (6, 11), (8, 13))):
        whole = oracle.backproject_block(proj, mats, cfg["shape"], cfg["voxel"], box)
        origin, wr, wc = owin.block_windows(mats, cfg["shape"], cfg["voxel"], box)
        win = owin.cut_windows(proj, origin, wr, wc)
        got = oracle.backproject_block(win, mats, cfg["shape"], cfg["voxel"], box,
                                       origin=origin, detector=(cfg["nh"], cfg["nw"]))
        np.testing.assert_array_equal(got, whole)
        assert np.abs(whole).max() > 0
    mid = ((4, 9), (3, 8), (5, 11))
    origin, wr, wc = owin.block_windows(mats, cfg["shape"], cfg["voxel"], mid, margin=0)
    narrow = origin.copy()
    narrow[:, 1] += 1                       # drops each window's first needed column
    with pytest.raises(ValueError):
        oracle.backproject_block(owin.cut_windows(proj, narrow, wr, wc), mats, cfg["shape"],
                                 cfg["voxel"], mid, origin=narrow,
                                 detector=(cfg["nh"], cfg["nw"]))


def test_accumulates_into_volume():
    proj, mats, shape, voxel = tiny_problem()
    base = np.random.default_rng(4).standard_normal(shape)
    out = oracle.backproject(proj, mats, shape, voxel, vol=base.copy())
    np.testing.assert_allclose(out - base, oracle.backproject(proj, mats, shape, voxel),
                               rtol=0, atol=1e-12)


# ------------------------------------------------------------ transpose

def test_adjoint_identity():
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(10, 12, 11), np_views=8, nh=40, nw=36)
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    p = wl.gaussian(31, (cfg["np"], cfg["nh"], cfg["nw"]))
    x = wl.gaussian(32, cfg["shape"], np.float64)
    bp = oracle.backproject(p, mats, cfg["shape"], cfg["voxel"])
    fp = oracle.forwardproject(x, mats, cfg["nh"], cfg["nw"], cfg["voxel"])
    lhs = float(np.sum(bp * x))
    rhs = float(np.sum(p.astype(np.float64) * fp))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(bp) * np.linalg.norm(x))


def test_forward_projection_brute_force():
    proj, mats, shape, voxel = tiny_problem()
    x = wl.gaussian(33, shape, np.float64)
    got = oracle.forwardproject(x, mats, 6, 7, voxel)
    ref = brute_forwardproject(x, mats, 6, 7, voxel)
    assert rel(got, ref) < 1e-13


# ------------------------------------------------------------ FP16 storage

def test_quantizer_rule():
    p = wl.gaussian(41, (5, 16, 20)) * np.float32(3.7)
    p[2] = 0.0
    p[3] *= np.float32(1e-3)
    p[4, 0, 0] = np.float32(2.0 ** 7)                        # exact power-of-two max
    h, scale = oracle.quantize_f16(p)
    assert h.dtype == np.float16 and scale.dtype == np.float32
    for s in range(5):
        m, e = np.frexp(float(scale[s]))
        assert m == 0.5, "scale must be a power of two"
        assert np.abs(h[s].astype(np.float64)).max() <= 32768.0
    assert scale[2] == 1.0 and np.all(h[2] == 0)
    assert scale[4] == 2.0 ** (7 - 15) and float(h[4, 0, 0]) == 32768.0
    deq = oracle.dequantize_f16(h, scale)
    big = np.abs(p) >= scale[:, None, None] * 2.0 ** -14 * 1.0001   # normal binary16 range
    relerr = np.abs(deq - p)[big] / np.abs(p)[big]
    assert relerr.max() <= 2.0 ** -11
    # round to nearest even: an exact half-way value rounds to the even code
    q = np.zeros((1, 1, 3), dtype=np.float32)
    q[0, 0] = [32768.0, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11]
    hq, sq = oracle.quantize_f16(q)
    assert sq[0] == 1.0
    assert float(hq[0, 0, 1]) == 1.0 and float(hq[0, 0, 2]) == 1.0 + 2.0 ** -9


# ------------------------------------------------------------ filter (FDK)

def test_ramp_filter_of_a_delta():
    """A single unit pixel on the central row becomes tau * h[n] * cosine
    weight * arc/(2 np) along the row, with the Ram-Lak closed form h."""
    scan = dict(sod=500.0, sdd=1000.0, du=1.0, dv=1.0, arc=2 * math.pi, theta0=0.0,
                u_off=0.0, v_off=0.0)
    nh, nw = 5, 33
    raw = np.zeros((1, nh, nw))
    c0 = 16
    raw[0, 2, c0] = 1.0
    out = oracle.fdk_filter(raw, scan, np_total=64)
    tau = scan["du"] * scan["sod"] / scan["sdd"]
    cosw = 1.0                                                # pixel at u_mm = v_mm = 0
    n = np.arange(nw) - c0
    h = np.zeros(nw)
    odd = n % 2 != 0
    h[odd] = -1 / (np.pi ** 2 * n[odd].astype(float) ** 2 * tau * tau)
    h[n == 0] = 1 / (4 * tau * tau)
    expect = tau * h * cosw * (2 * math.pi / (2 * 64))
    np.testing.assert_allclose(out[0, 2], expect, rtol=1e-13, atol=1e-16)
    assert np.all(out[0, [0, 1, 3, 4]] == 0.0)


def test_ramp_filter_frequency_response():
    """Away from the row ends the filtered cosine cos(2 pi f x) becomes
    |f| cos(2 pi f x) (the ramp), in units where x is isocentre millimetres."""
    scan = dict(sod=1000.0, sdd=1000.0, du=1.0, dv=1.0, arc=2 * math.pi, theta0=0.0,
                u_off=0.0, v_off=0.0)
    nw = 4001
    x = (np.arange(nw) - (nw - 1) / 2) * scan["du"]
    for f in (0.05, 0.13, 0.31):
        raw = np.cos(2 * np.pi * f * x)[None, None, :]
        # undo the cosine weight so that the filter input is the pure cosine
        raw = raw * np.sqrt(scan["sdd"] ** 2 + x ** 2) / scan["sdd"]
        out = oracle.fdk_filter(raw, scan, np_total=1)[0, 0] / (2 * math.pi / 2)
        mid = slice(1500, 2501)
        err = np.abs(out[mid] - abs(f) * np.cos(2 * np.pi * f * x[mid])).max()
        assert err < 2e-3 * abs(f) + 2e-4


def test_fdk_reconstructs_a_sphere():
    """Ramp-filtered analytic projections of a centred sphere reconstruct its
    density inside (the FDK scaling: cosine weight, tau, pi/np, 1/w^2)."""
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(1, 48, 48), np_views=96, nh=8, nw=128)
    scan = cfg["scan"]
    ell = np.zeros((1, 16))
    ell[0, 3:6] = 15.0
    ell[0, 6:15] = np.eye(3).ravel()
    ell[0, 15] = 0.8
    rows = np.arange(cfg["nh"])
    raw = oph.line_integrals(ell, scan, cfg["np"], cfg["nh"], cfg["nw"])
    filt = oracle.fdk_filter(raw, scan).astype(np.float32)
    mats = og.scan_matrices(scan, cfg["np"], cfg["nh"], cfg["nw"])
    rec = oracle.backproject(filt, mats, cfg["shape"], cfg["voxel"])[0]
    yy, xx = np.meshgrid(np.arange(48) - 23.5, np.arange(48) - 23.5, indexing="ij")
    rr = np.hypot(xx, yy)
    inner = rec[rr < 10]
    outer = rec[(rr > 19) & (rr < 23)]
    assert abs(inner.mean() - 0.8) < 0.02 * 0.8
    assert np.abs(outer).mean() < 0.03
    # a mirrored u axis (wrong sign in e_u) would shift an off-centre sphere
    ell2 = ell.copy()
    ell2[0, 0:3] = [8.0, -6.0, 0.0]
    ell2[0, 3:6] = 5.0
    raw2 = oph.line_integrals(ell2, scan, cfg["np"], cfg["nh"], cfg["nw"])
    rec2 = oracle.backproject(oracle.fdk_filter(raw2, scan).astype(np.float32), mats,
                              cfg["shape"], cfg["voxel"])[0]
    jj, ii = np.nonzero(rec2 > 0.5 * rec2.max())
    assert abs((ii.mean() - 23.5) - 8.0) <= 0.5 and abs((jj.mean() - 23.5) + 6.0) <= 0.5


def test_fdk_random_ellipsoids_central_slice():
    """C1-shaped reconstruction of seeded random ellipsoids: the central slice
    matches the voxelised phantom after light smoothing (FDK is exact only in
    the mid-plane and the data are band-limited).  Ellipsoids that reach
    beyond the detector's field of view are dropped, since truncated
    projections bias any filtered back-projection."""
    from scipy.ndimage import gaussian_filter
    cfg = wl.CONFIGS["c1"]
    scan = cfg["scan"]
    ell = np.concatenate([wl.config_ellipsoids(cfg, i) for i in range(4)])
    reach = np.hypot(ell[:, 0], ell[:, 1]) + ell[:, 3:6].max(1)
    ell = ell[reach < 29.0]
    assert len(ell) >= 5
    rows = np.arange(60, 68)              # the rows the central slice projects to
    raw = oph.line_integrals(ell, scan, cfg["np"], cfg["nh"], cfg["nw"], rows=rows)
    full = np.zeros((cfg["np"], cfg["nh"], cfg["nw"]))
    full[:, rows] = raw
    filt = oracle.fdk_filter(full, scan).astype(np.float32)
    mats = og.scan_matrices(scan, cfg["np"], cfg["nh"], cfg["nw"])
    shape = cfg["shape"]
    k = shape[0] // 2
    rec = oracle.backproject_block(filt, mats, shape, cfg["voxel"], ((k, k + 1), (0, 64), (0, 64)))[0]
    truth = oph.voxelize(ell, shape, cfg["voxel"], supersample=3)[k]
    assert np.linalg.norm(truth) > 0
    assert rel(gaussian_filter(rec, 1.0), gaussian_filter(truth, 1.0)) < 0.12
    assert abs(rec.sum() / truth.sum() - 1.0) < 0.08


# ------------------------------------------------------------ phantom

def test_sphere_chord_closed_form():
    scan = dict(sod=500.0, sdd=1000.0, du=1.0, dv=1.0, arc=2 * math.pi, theta0=0.0,
                u_off=0.0, v_off=0.0)
    nh, nw = 9, 9
    R, rho = 20.0, 0.7
    ell = np.zeros((1, 16))
    ell[0, 3:6] = R
    ell[0, 6:15] = np.eye(3).ravel()
    ell[0, 15] = rho
    li = oph.line_integrals(ell, scan, 4, nh, nw)
    # central ray passes through the centre: chord = 2R
    np.testing.assert_allclose(li[:, 4, 4], 2 * R * rho, rtol=1e-13)
    # ray to pixel (4, 4+m): perpendicular distance from the centre to the ray
    for m in (1, 3):
        umm = m * scan["du"]
        d = np.array([scan["sdd"], umm])                 # in the (n, e_u) plane
        dist = scan["sod"] * umm / np.linalg.norm(d)
        np.testing.assert_allclose(li[:, 4, 4 + m], 2 * rho * math.sqrt(R * R - dist * dist),
                                   rtol=1e-12)


def test_small_sphere_peaks_where_matrix_predicts():
    cfg = wl.shrink(wl.CONFIGS["c1"], np_views=6, nh=64, nw=64)
    scan = dict(cfg["scan"], theta0=0.4, u_off=0.7, v_off=-1.2)
    X0 = np.array([9.0, -13.0, 6.0])
    ell = np.zeros((1, 16))
    ell[0, 0:3] = X0
    ell[0, 3:6] = 1.2
    ell[0, 6:15] = np.eye(3).ravel()
    ell[0, 15] = 1.0
    li = oph.line_integrals(ell, scan, cfg["np"], cfg["nh"], cfg["nw"])
    mats = og.scan_matrices(scan, cfg["np"], cfg["nh"], cfg["nw"])
    for s in range(cfg["np"]):
        q = mats[s] @ np.append(X0, 1.0)
        u, v = q[0] / q[2], q[1] / q[2]
        r, c = np.unravel_index(np.argmax(li[s]), li[s].shape)
        assert abs(c - u) <= 1.0 and abs(r - v) <= 1.0
