"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any HIP call.

Device pointers here are fake non-NULL addresses: every case is rejected by
host-side validation before the library would touch them."""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

import oracle
from oracle import geometry as og
import workloads as wl

fdk = pytest.importorskip("paper_2104_13248_amd")
from paper_2104_13248_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x10000)
OK, E_INVALID, E_GEOMETRY, E_UNSUPPORTED = 0, -1, -2, -3


def header_functions():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(fdk_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_exports_match_header():
    names = header_functions()
    assert "fdk_backproject" in names and "fdk_forwardproject" in names and "fdk_filter" in names
    for n in names:
        assert hasattr(_lib.lib, n), n
    assert sorted(_lib.EXPORTS) == names


def test_symbols_via_nm():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (fdk_\w+)", out))
    assert set(header_functions()) <= exported


def _geom(cfg):
    vg = _lib.volume_struct(cfg["shape"], cfg["voxel"])
    sg = _lib.stack_struct(cfg["np"], cfg["nh"], cfg["nw"])
    m = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    return vg, sg, np.ascontiguousarray(m)


def call_bp(vg, sg, m, vol=FAKE, proj=FAKE, scale=None):
    return _lib.lib.fdk_backproject(ctypes.byref(vg) if vg is not None else None, vol,
                                    ctypes.byref(sg) if sg is not None else None, proj, scale,
                                    _lib.ptr(m) if m is not None else None, None)


C1 = wl.CONFIGS["c1"]


def test_null_pointers_rejected():
    vg, sg, m = _geom(C1)
    assert call_bp(None, sg, m) == E_INVALID
    assert call_bp(vg, None, m) == E_INVALID
    assert call_bp(vg, sg, None) == E_INVALID
    assert call_bp(vg, sg, m, vol=None) == E_INVALID
    assert call_bp(vg, sg, m, proj=None) == E_INVALID
    assert "NULL" in _lib.lib.fdk_last_error().decode()


def test_bad_sizes_rejected():
    vg, sg, m = _geom(C1)
    for field in ("nx", "ny", "nz"):
        bad = _lib.volume_struct(C1["shape"], C1["voxel"])
        setattr(bad, field, 0)
        assert call_bp(bad, sg, m) == E_INVALID
    bad = _lib.volume_struct(C1["shape"], (1.0, -1.0, 1.0))
    assert call_bp(bad, sg, m) == E_INVALID
    bad = _lib.volume_struct(C1["shape"], (1.0, float("nan"), 1.0))
    assert call_bp(bad, sg, m) == E_INVALID
    for field in ("np", "nh", "nw"):
        s2 = _lib.stack_struct(C1["np"], C1["nh"], C1["nw"])
        setattr(s2, field, -3)
        assert call_bp(vg, s2, m) == E_INVALID


def test_dtype_and_scale_rules():
    vg, sg, m = _geom(C1)
    s_bad = _lib.stack_struct(C1["np"], C1["nh"], C1["nw"], 7)
    assert call_bp(vg, s_bad, m) == E_INVALID
    s16 = _lib.stack_struct(C1["np"], C1["nh"], C1["nw"], _lib.FDK_F16)
    assert call_bp(vg, s16, m, scale=None) == E_INVALID            # f16 needs scales
    assert call_bp(vg, sg, m, scale=FAKE) == E_INVALID             # f32 takes none
    # the forward projector takes float32 only
    assert _lib.lib.fdk_forwardproject(ctypes.byref(vg), FAKE, ctypes.byref(s16), FAKE,
                                       _lib.ptr(m), None) == E_UNSUPPORTED


def test_non_finite_matrix_rejected():
    vg, sg, m = _geom(C1)
    m = m.copy()
    m[3, 1, 2] = np.inf
    assert call_bp(vg, sg, m) == E_INVALID


def test_tilted_detector_rejected():
    """u w or w depending on k breaks the hoisting the kernels rely on."""
    vg, sg, m = _geom(C1)
    m1 = m.copy()
    m1[5, 0, 2] = 1e-3                       # u w depends on z
    assert call_bp(vg, sg, m1) == E_GEOMETRY
    m2 = m.copy()
    m2[0, 2, 2] = 1e-4                       # w depends on z
    assert call_bp(vg, sg, m2) == E_GEOMETRY
    assert "slice index" in _lib.lib.fdk_last_error().decode()
    m3 = m.copy()
    m3[0, 0, 2] = 1e-16                      # round-off sized entries are accepted
    vg2 = _lib.volume_struct(C1["shape"], C1["voxel"])
    out = (ctypes.c_int64 * 12)()
    assert _lib.lib.fdk_bp_plan(ctypes.byref(vg2), ctypes.byref(sg), _lib.ptr(m3),
                                ctypes.cast(out, ctypes.c_void_p)) == OK


def test_voxel_behind_source_rejected():
    cfg = dict(C1, scan=dict(C1["scan"], sod=20.0, sdd=40.0))  # source inside the FOV
    vg, sg, m = _geom(cfg)
    assert call_bp(vg, sg, m) == E_GEOMETRY
    assert "w <= 0" in _lib.lib.fdk_last_error().decode()


def test_slab_range_rejected():
    vg, sg, m = _geom(C1)
    f = _lib.lib.fdk_backproject_slab
    for kb, kc in [(-1, 4), (0, 0), (60, 5), (64, 1)]:
        assert f(ctypes.byref(vg), kb, kc, FAKE, ctypes.byref(sg), FAKE, None, _lib.ptr(m),
                 None) == E_INVALID


def test_filter_quantize_phantom_validation():
    sg = _lib.stack_struct(4, 8, 16)
    L = _lib.lib
    OUT = ctypes.c_void_p(0x20000)
    SC = ctypes.c_void_p(0x30000)
    assert L.fdk_filter(ctypes.byref(sg), None, 0, FAKE, None, 1.0, 1.0, 500.0, 1000.0, 0, 0,
                        6.28, 4, None) == E_INVALID
    assert L.fdk_filter(ctypes.byref(sg), FAKE, 0, FAKE, None, 1.0, 1.0, 500.0, 1000.0, 0, 0,
                        6.28, 4, None) == E_INVALID                 # raw == out
    assert L.fdk_filter(ctypes.byref(sg), FAKE, 0, OUT, None, -1.0, 1.0, 500.0,
                        1000.0, 0, 0, 6.28, 4, None) == E_INVALID
    assert L.fdk_filter(ctypes.byref(sg), FAKE, 0, OUT, None, 1.0, 1.0, 500.0,
                        1000.0, 0, 0, 6.28, 0, None) == E_INVALID
    # output dtype and scale array must agree
    assert L.fdk_filter(ctypes.byref(sg), FAKE, 1, OUT, None, 1.0, 1.0, 500.0,
                        1000.0, 0, 0, 6.28, 4, None) == E_INVALID     # f16 without scale
    assert L.fdk_filter(ctypes.byref(sg), FAKE, 0, OUT, SC, 1.0, 1.0, 500.0,
                        1000.0, 0, 0, 6.28, 4, None) == E_INVALID     # f32 with scale
    assert L.fdk_filter(ctypes.byref(sg), FAKE, 2, OUT, SC, 1.0, 1.0, 500.0,
                        1000.0, 0, 0, 6.28, 4, None) == E_INVALID     # unknown dtype
    assert L.fdk_quantize_f16(0, 8, 16, FAKE, FAKE, FAKE, None) == E_INVALID
    assert L.fdk_quantize_f16(4, 8, 16, FAKE, FAKE, None, None) == E_INVALID
    ell = np.zeros((2, 16))
    ell[:, 3:6] = 1.0
    scan = C1["scan"]
    args = [scan["arc"], scan["theta0"], scan["sod"], scan["sdd"], scan["du"], scan["dv"],
            scan["u_off"], scan["v_off"]]
    assert L.fdk_phantom_project(_lib.ptr(ell), 2, ctypes.byref(sg), FAKE, *args, 2, 5,
                                 None) == E_INVALID             # views past np_total
    bad = ell.copy()
    bad[1, 4] = 0.0
    assert L.fdk_phantom_project(_lib.ptr(bad), 2, ctypes.byref(sg), FAKE, *args, 0, 4,
                                 None) == E_INVALID             # zero semi-axis


def test_noalloc_rejects_more_views_than_its_scratch():
    vg, _, _ = _geom(C1)
    big = 16385
    sg = _lib.stack_struct(big, C1["nh"], C1["nw"])
    m = np.zeros((big, 3, 4))
    assert _lib.lib.fdk_backproject_noalloc(ctypes.byref(vg), FAKE, ctypes.byref(sg), FAKE, None,
                                            _lib.ptr(m), None) == E_UNSUPPORTED
    assert b"16384" in _lib.lib.fdk_last_error()
    vg2, sg2, m2 = _geom(C1)
    assert _lib.lib.fdk_backproject_noalloc(ctypes.byref(vg2), None, ctypes.byref(sg2), FAKE,
                                            None, _lib.ptr(m2), None) == E_INVALID


def test_peak_microbenchmarks_validate():
    L = _lib.lib
    n = ctypes.c_int64(0)
    assert L.fdk_peak_hbm_read(None, 1024, 8, FAKE, None) == E_INVALID
    assert L.fdk_peak_hbm_read(FAKE, 1000, 8, FAKE, None) == E_INVALID          # not 16 * k
    assert L.fdk_peak_hbm_read(ctypes.c_void_p(0x10004), 1024, 8, FAKE, None) == E_INVALID
    assert L.fdk_peak_hbm_read(FAKE, 1024, 0, FAKE, None) == E_INVALID
    assert L.fdk_peak_lds_read(8, 8, 1, FAKE, ctypes.addressof(n), None) == E_INVALID
    assert L.fdk_peak_valu_op(12, 8, 1, FAKE, ctypes.addressof(n), None) == E_INVALID
    assert L.fdk_peak_valu_op(0, 8, 0, FAKE, ctypes.addressof(n), None) == E_INVALID
    assert L.fdk_peak_lds_read(0, 0, 1, FAKE, ctypes.addressof(n), None) == E_INVALID
    assert L.fdk_peak_lds_read(0, 8, 1, None, ctypes.addressof(n), None) == E_INVALID
    assert L.fdk_peak_valu_fma(8, 0, FAKE, ctypes.addressof(n), None) == E_INVALID
    assert L.fdk_peak_valu_fma(8, 1, FAKE, None, None) == E_INVALID


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5):
        assert _lib.lib.fdk_status_string(code).decode()
    assert _lib.lib.fdk_status_string(42).decode() == "unknown status"


def test_circular_matrices_match_ray_plane_geometry():
    """The library's matrix helper against the oracle's ray/plane intersection
    (an independent derivation of the same scanner)."""
    scan = dict(sod=510.0, sdd=990.0, du=0.7, dv=1.1, arc=2 * math.pi, theta0=0.4,
                u_off=1.5, v_off=-2.25)
    npv, nh, nw = 11, 50, 70
    m = fdk.circular_matrices(npv, scan["arc"], scan["theta0"], scan["sod"], scan["sdd"], nh, nw,
                              scan["du"], scan["dv"], scan["u_off"], scan["v_off"])
    th = og.view_angles(npv, scan["arc"], scan["theta0"])
    pts = np.random.default_rng(3).uniform(-60, 60, (40, 3))
    for s in range(npv):
        uvw = oracle.project_points(th[s], scan, nh, nw, pts)
        q = np.concatenate([pts, np.ones((40, 1))], 1) @ m[s].T
        np.testing.assert_allclose(q[:, 0] / q[:, 2], uvw[:, 0], atol=1e-9)
        np.testing.assert_allclose(q[:, 1] / q[:, 2], uvw[:, 1], atol=1e-9)
        np.testing.assert_allclose(q[:, 2], uvw[:, 2], atol=1e-12)
    assert np.all(m[:, 0, 2] == 0) and np.all(m[:, 2, 2] == 0)
    with pytest.raises(fdk.FdkError):
        fdk.circular_matrices(4, scan["arc"], 0.0, -1.0, 990.0, nh, nw, 1.0, 1.0)


@pytest.mark.parametrize("name,f16", [("c1", False), ("c2", False), ("c2", True), ("c3", False),
                                      ("c3", True), ("c4", False), ("c5", False)])
def test_plan_covers_every_footprint(name, f16):
    """The launch plan bounds the footprint of every block and view (checked
    here by brute force over tiles, chunks and views, in FP64, with the
    kernel's own rule): every half-chunk fits the LDS rows, every whole chunk
    fits rows_full, every width fits the pitch."""
    cfg = wl.CONFIGS[name]
    m = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    plan = fdk.bp_plan(cfg["shape"], cfg["voxel"], cfg["np"], cfg["nh"], cfg["nw"], m, f16=f16)
    M = og.index_matrices(m, cfg["shape"], cfg["voxel"])
    nz, ny, nx = cfg["shape"]
    kz = plan["kz"]
    step = max(1, cfg["np"] // 64)
    M = M[::step]
    i0 = np.arange(0, nx, 16)
    j0 = np.arange(0, ny, 16)
    k0 = np.arange(0, nz, kz)
    I = np.stack([i0, np.minimum(i0 + 15, nx - 1)], 1)          # [ntx, 2]
    J = np.stack([j0, np.minimum(j0 + 15, ny - 1)], 1)

    def rows(A, w, ka, kb, Ms):
        v0 = (A + Ms[1, 2] * ka) / w
        v1 = (A + Ms[1, 2] * kb) / w
        vmin = np.minimum(v0, v1).min(axis=(2, 3))
        vmax = np.maximum(v0, v1).max(axis=(2, 3))
        return int((np.floor(vmax) - np.floor(vmin)).max()) + 4

    cols = full = half = 0
    for Ms in M:
        ii = I[:, None, :, None]
        jj = J[None, :, None, :]
        w = Ms[2, 0] * ii + Ms[2, 1] * jj + Ms[2, 3]
        u = (Ms[0, 0] * ii + Ms[0, 1] * jj + Ms[0, 3]) / w
        cols = max(cols, int((np.floor(u.max(axis=(2, 3))) - np.floor(u.min(axis=(2, 3)))).max()) + 4)
        A = Ms[1, 0] * ii + Ms[1, 1] * jj + Ms[1, 3]
        for kc in k0:
            full = max(full, rows(A, w, kc, kc + kz - 1, Ms))
            half = max(half, rows(A, w, kc, kc + kz // 2 - 1, Ms),
                       rows(A, w, kc + kz // 2, kc + kz - 1, Ms))
    assert cols <= plan["lds_pitch"]
    assert half <= plan["lds_rows"]
    assert full <= plan["rows_full"]
    assert plan["lds_bytes"] >= plan["lds_rows"] * plan["lds_pitch"] * 4
    # forward projector: a window of (band rows + 2) x pitch floats within the default
    # budget; chunks of at most 128 columns cover the detector evenly
    fp, rb, cw = plan["fp_lds_bytes"], plan["fp_rows"], plan["fp_cols"]
    chunks = -(-cfg["nw"] // cw)
    assert cw <= 128 and chunks == -(-cfg["nw"] // 128) and (chunks - 1) * cw < cfg["nw"]
    assert fp % (4 * (rb + 2)) == 0 and cw + 4 <= fp // (4 * (rb + 2)) <= 254
    assert 1 <= rb <= min(64, cfg["nh"])
    assert fp <= 10 * 1024


def test_learned_filter_entry_points_validate():
    lib = _lib.lib
    # unsupported channel counts, bad sizes, NULL pointers: rejected on the host
    assert lib.fdk_conv1d_forward(16, 32, 4, 8, FAKE, FAKE, None, None, None, 1.0, 0, FAKE,
                                  None) == E_UNSUPPORTED
    assert lib.fdk_conv1d_forward(1, 32, 0, 8, FAKE, FAKE, None, None, None, 1.0, 0, FAKE,
                                  None) == E_INVALID
    assert lib.fdk_conv1d_forward(1, 32, 4, 8, None, FAKE, None, None, None, 1.0, 0, FAKE,
                                  None) == E_INVALID
    assert lib.fdk_conv1d_forward(1, 32, 4, 8, FAKE, FAKE, None, None, None, math.inf, 0,
                                  ctypes.c_void_p(0x20000), None) == E_INVALID
    assert lib.fdk_conv1d_backward_data(32, 5, 4, 8, FAKE, FAKE, None, FAKE, None) == E_UNSUPPORTED
    assert lib.fdk_conv1d_backward_data(32, 32, 4, 8, FAKE, FAKE, None, FAKE, None) == E_INVALID
    assert lib.fdk_conv1d_backward_weight(32, 32, 4, -1, FAKE, FAKE, FAKE, None, None) == E_INVALID
    assert lib.fdk_conv1d_backward_weight(32, 32, 4, 8, FAKE, FAKE, None, None, None) == E_INVALID
    assert lib.fdk_sqerr(0, FAKE, FAKE, None, 1.0, FAKE, None) == E_INVALID
    assert lib.fdk_sqerr(10, FAKE, FAKE, None, 1.0, None, None) == E_INVALID
    assert lib.fdk_adam(10, FAKE, FAKE, FAKE, FAKE, 1e-3, 0.9, 0.999, 1e-8, 0, None) == E_INVALID
    assert lib.fdk_adam(10, FAKE, FAKE, FAKE, FAKE, 1e-3, 1.0, 0.999, 1e-8, 1, None) == E_INVALID
    assert lib.fdk_adam(10, FAKE, FAKE, FAKE, FAKE, 1e-3, 0.9, 0.999, 0.0, 1, None) == E_INVALID
    sg = _lib.stack_struct(2, 3, 4)
    assert lib.fdk_cosine_weight(ctypes.byref(sg), FAKE, None, 1.0, 1.0, 100.0, 0.0, 0.0,
                                 None) == E_INVALID
    assert lib.fdk_cosine_weight(ctypes.byref(sg), FAKE, FAKE, 1.0, -1.0, 100.0, 0.0, 0.0,
                                 None) == E_INVALID
    bad = _lib.stack_struct(2, 3, 4, _lib.FDK_F16)
    assert lib.fdk_cosine_weight(ctypes.byref(bad), FAKE, FAKE, 1.0, 1.0, 100.0, 0.0, 0.0,
                                 None) != OK


def test_variant_entry_point_validates():
    vg, sg, m = _geom(C1)
    lib = _lib.lib
    assert lib.fdk_backproject_variant(9, 4, ctypes.byref(vg), FAKE, ctypes.byref(sg), FAKE,
                                       _lib.ptr(m), None) == E_INVALID
    assert lib.fdk_backproject_variant(2, 0, ctypes.byref(vg), FAKE, ctypes.byref(sg), FAKE,
                                       _lib.ptr(m), None) == E_INVALID
    assert lib.fdk_backproject_variant(1, 4, ctypes.byref(vg), None, ctypes.byref(sg), FAKE,
                                       _lib.ptr(m), None) == E_INVALID
    s16 = _lib.stack_struct(C1["np"], C1["nh"], C1["nw"], _lib.FDK_F16)
    assert lib.fdk_backproject_variant(1, 4, ctypes.byref(vg), FAKE, ctypes.byref(s16), FAKE,
                                       _lib.ptr(m), None) == E_UNSUPPORTED
    # the symmetric variant needs v(nz-1-k) = nh-1-v(k): rejected (before any HIP
    # call) when the detector's centre row is offset or the volume is off-centre in z
    m_off = np.ascontiguousarray(og.scan_matrices(dict(C1["scan"], v_off=1.5), C1["np"], C1["nh"],
                                                  C1["nw"]))
    assert lib.fdk_backproject_variant(3, 1, ctypes.byref(vg), FAKE, ctypes.byref(sg), FAKE,
                                       _lib.ptr(m_off), None) == E_GEOMETRY
    vz = _lib.volume_struct(C1["shape"], C1["voxel"], (0.0, 0.0, 2.0))
    assert lib.fdk_backproject_variant(3, 1, ctypes.byref(vz), FAKE, ctypes.byref(sg), FAKE,
                                       _lib.ptr(m), None) == E_GEOMETRY


def test_forward_projector_falls_back_for_huge_slices(monkeypatch):
    """The voxel-driven forward projector addresses a tile's slices with 31-bit
    byte offsets; 256 MiB slices (8192^2 voxels) cannot fit even a few, so the
    plan takes the column-owned organisation (256-column chunks); 64 MiB
    slices still fit.  FDK_FP_ALGO=gather forces the fallback."""
    scan = dict(sod=750.0, sdd=1200.0, du=1.0, dv=1.0, arc=2 * math.pi, theta0=0.0,
                u_off=0.0, v_off=0.0)
    mats = og.scan_matrices(scan, 8, 1024, 1024)
    huge = fdk.bp_plan((16, 8192, 8192), (0.05,) * 3, 8, 1024, 1024, mats)
    big = fdk.bp_plan((16, 4096, 4096), (0.1,) * 3, 8, 1024, 1024, mats)
    assert huge["fp_cols"] == 256 and huge["fp_lds_bytes"] == 4 * (huge["fp_rows"] + 2) * 258
    assert big["fp_cols"] == 128
    monkeypatch.setenv("FDK_FP_ALGO", "gather")
    assert fdk.bp_plan((16, 4096, 4096), (0.1,) * 3, 8, 1024, 1024, mats)["fp_cols"] == 256


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_plan_tile_grows_to_four_blocks_per_cu(name, monkeypatch):
    """Past the percentile footprint the back-projector's tile grows while four
    blocks still fit a CU's 160 KiB of LDS (39 KiB each, view table included),
    never beyond the tallest footprint; binary16 tiles take rows = 4 mod 8 so
    that their two pair-word regions (rows x pitch/2 words each) start 16 banks
    (mod 32) apart.  FDK_BP_TILE_BYTES=0 keeps the percentile rows."""
    cfg = wl.CONFIGS[name]
    m = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    args = (cfg["shape"], cfg["voxel"], cfg["np"], cfg["nh"], cfg["nw"], m)
    table = 32 * 24 * 4
    p32, p16 = fdk.bp_plan(*args), fdk.bp_plan(*args, f16=True)
    monkeypatch.setenv("FDK_BP_TILE_BYTES", "0")
    base = fdk.bp_plan(*args)
    assert fdk.bp_plan(*args, f16=True)["lds_rows"] == base["lds_rows"]
    for p in (p32, p16):
        assert (p["kz"], p["lds_pitch"], p["rows_full"]) == (base["kz"], base["lds_pitch"], base["rows_full"])
        assert p["lds_bytes"] == p["lds_rows"] * p["lds_pitch"] * 4 + table <= 39 * 1024
        assert base["lds_rows"] <= p["lds_rows"]
    fit = (39 * 1024 - table) // (base["lds_pitch"] * 4)
    assert p32["lds_rows"] == max(base["lds_rows"], min(fit, base["rows_full"]))
    if p16["lds_rows"] > base["lds_rows"]:
        assert p16["lds_rows"] % 8 == 4 and p16["lds_rows"] <= fit
        assert (p16["lds_rows"] * base["lds_pitch"] // 2) % 32 == 16


def test_plan_takes_direct_taps_when_staging_offsets_could_overflow():
    """The staging loop addresses a window's rows by one signed 32-bit byte
    offset per lane, its first row clamped to [-R, nh]: the plan keeps the LDS
    tile only while (nh + rows + 1) rows of a view stay below 2^31 bytes, and
    otherwise takes the direct organisation (lds_pitch = 0).  Host only."""
    scan = dict(wl.CONFIGS["c1"]["scan"])
    shape, voxel = (32, 32, 32), (1.0, 1.0, 1.0)
    nh = 1024
    ok = 8192                                    # 32 MiB views
    edge = (2 ** 31 - 1) // (4 * nh)             # a float32 view just under 2 GiB
    for nw, direct in ((ok, False), (edge, True)):
        mats = og.scan_matrices(scan, 2, nh, nw)
        plan = fdk.bp_plan(shape, voxel, 2, nh, nw, mats)
        assert (plan["lds_pitch"] == 0) == direct, (nw, plan)
        # binary16 views of the same width are half as large: the tile stays
        plan16 = fdk.bp_plan(shape, voxel, 2, nh, nw, mats, f16=True)
        assert plan16["lds_pitch"] > 0, (nw, plan16)
