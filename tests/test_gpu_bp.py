"""Parity of the HIP back-projector with the FP64 oracle (MI355X).

Every case feeds the same seeded host arrays to both sides.  FP32 tolerance:
rel-L2 <= 1e-5; FP16-stored projections: rel-L2 <= 1e-3 against the oracle on
the float32 stack (and <= 1e-5 against the oracle on the dequantised stack,
which isolates the kernel's own error from the storage rounding).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import geometry as og
import workloads as wl
from helpers import (c1_filtered, gpu_phantom_stacks, log, rel, subblock_errors,
                     whole_rel)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdk = pytest.importorskip("paper_2104_13248_amd")

TOL32 = 1e-5
TOL16 = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def gpu_bp(proj, mats, shape, voxel, centre=(0.0, 0.0, 0.0), vol0=None, scale=None):
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda") if vol0 is None else \
        torch.from_numpy(np.ascontiguousarray(vol0, dtype=np.float32)).cuda()
    p = torch.from_numpy(np.ascontiguousarray(proj)).cuda()
    s = None if scale is None else torch.from_numpy(np.ascontiguousarray(scale)).cuda()
    fdk.backproject(vol, p, mats, voxel, centre, scale=s)
    torch.cuda.synchronize()
    return vol.cpu().numpy()


def test_c1_phantom_f32():
    cfg = wl.CONFIGS["c1"]
    proj, mats = c1_filtered(0)
    log("c1 phantom f32", cfg["shape"], proj.shape)
    got = gpu_bp(proj, mats, cfg["shape"], cfg["voxel"])
    ref = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"])
    e = rel(got, ref)
    log("rel-L2", e)
    assert e <= TOL32


def test_c1_gaussian_f32():
    """White-noise projections: the largest interpolation gradients."""
    cfg = wl.CONFIGS["c1"]
    proj = wl.gaussian(101, (cfg["np"], cfg["nh"], cfg["nw"]))
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    got = gpu_bp(proj, mats, cfg["shape"], cfg["voxel"])
    ref = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"])
    e = rel(got, ref)
    log("c1 gaussian rel-L2", e)
    assert e <= TOL32


RAGGED = [
    # shape (nz, ny, nx), (np, nh, nw), voxel, centre, scan overrides
    ((7, 19, 33), (70, 45, 61), (0.9, 1.1, 1.3), (2.0, -3.0, 1.5),
     dict(theta0=0.3, u_off=1.7, v_off=-2.2)),
    ((1, 16, 16), (1, 40, 40), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), {}),
    ((33, 17, 15), (129, 96, 80), (1.0, 1.0, 0.5), (0.0, 0.0, -4.0), dict(arc=math.pi)),
    ((5, 1, 1), (3, 16, 16), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), {}),
    ((40, 48, 48), (64, 30, 200), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), dict(dv=2.0)),  # volume far off the detector rows
]


@pytest.mark.parametrize("case", range(len(RAGGED)))
def test_ragged_shapes(case):
    shape, (npv, nh, nw), voxel, centre, over = RAGGED[case]
    scan = dict(wl.CONFIGS["c1"]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    proj = wl.gaussian(200 + case, (npv, nh, nw))
    log("ragged", case, shape, (npv, nh, nw))
    got = gpu_bp(proj, mats, shape, voxel, centre)
    ref = oracle.backproject(proj, mats, shape, voxel, centre)
    e = rel(got, ref)
    log("rel-L2", e)
    assert e <= TOL32


def test_accumulates_into_volume():
    cfg = wl.CONFIGS["c1"]
    proj, mats = c1_filtered(0)
    base = wl.gaussian(300, cfg["shape"])
    got = gpu_bp(proj, mats, cfg["shape"], cfg["voxel"], vol0=base)
    ref = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"], vol=base.astype(np.float64))
    assert rel(got, ref) <= TOL32


def test_deterministic_bitwise():
    cfg = wl.CONFIGS["c1"]
    proj, mats = c1_filtered(0)
    a = gpu_bp(proj, mats, cfg["shape"], cfg["voxel"])
    b = gpu_bp(proj, mats, cfg["shape"], cfg["voxel"])
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_slabs_bitwise_equal_full():
    """z-slab decomposition (the multi-device split) reproduces the full call."""
    cfg = wl.shrink(wl.CONFIGS["c1"], shape=(70, 40, 36))
    proj, mats = c1_filtered(0)
    full = gpu_bp(proj, mats, cfg["shape"], cfg["voxel"])
    p = torch.from_numpy(proj).cuda()
    for k0, kc in [(0, 70), (0, 1), (5, 20), (31, 33), (69, 1), (32, 32), (17, 53)]:
        slab = torch.zeros((kc,) + cfg["shape"][1:], dtype=torch.float32, device="cuda")
        fdk.backproject_slab(slab, cfg["shape"], k0, p, mats, cfg["voxel"])
        torch.cuda.synchronize()
        got = slab.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), full[k0:k0 + kc].view(np.uint32)), (k0, kc)


def test_quantizer_bit_exact():
    proj, _ = c1_filtered(0)
    proj = proj.copy()
    proj[3] = 0.0                                   # an all-zero view
    proj[5] *= np.float32(1e-20)                    # tiny values (binary16 subnormals)
    proj[7, 0, :] = np.float32(-0.0)                # negative zeros keep their sign
    h_ref, s_ref = oracle.quantize_f16(proj)
    h, s = fdk.quantize_f16(torch.from_numpy(proj).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy().view(np.uint32), s_ref.view(np.uint32))
    assert np.array_equal(h.cpu().numpy().view(np.uint16), h_ref.view(np.uint16))


def test_c1_f16_storage():
    cfg = wl.CONFIGS["c1"]
    proj, mats = c1_filtered(0)
    h, s = fdk.quantize_f16(torch.from_numpy(proj).cuda())
    vol = torch.zeros(cfg["shape"], dtype=torch.float32, device="cuda")
    fdk.backproject(vol, h, mats, cfg["voxel"], scale=s)
    torch.cuda.synchronize()
    got = vol.cpu().numpy()
    ref32 = oracle.backproject(proj, mats, cfg["shape"], cfg["voxel"])
    h_np, s_np = h.cpu().numpy(), s.cpu().numpy()
    ref16 = oracle.backproject(h_np, mats, cfg["shape"], cfg["voxel"], scale=s_np)
    e32, e16 = rel(got, ref32), rel(got, ref16)
    log("f16: vs oracle(f32) %.3e, vs oracle(dequantised) %.3e, storage-only %.3e"
        % (e32, e16, rel(ref16, ref32)))
    assert e32 <= TOL16
    assert e16 <= TOL32


OFF_DETECTOR = [
    # shape (nz, ny, nx), (np, nh, nw), centre: windows of blocks far above,
    # far below and partly beside the detector rows (a window's first row
    # many window heights outside the detector, where the staging clamps it)
    ((40, 24, 24), (16, 20, 64), (0.0, 0.0, 260.0)),
    ((40, 24, 24), (16, 20, 64), (0.0, 0.0, -260.0)),
    ((70, 24, 24), (16, 20, 64), (0.0, 0.0, 30.0)),
]


@pytest.mark.parametrize("f16", [False, True])
@pytest.mark.parametrize("case", range(len(OFF_DETECTOR)))
def test_windows_off_detector(case, f16):
    shape, (npv, nh, nw), centre = OFF_DETECTOR[case]
    scan = wl.CONFIGS["c1"]["scan"]
    mats = og.scan_matrices(scan, npv, nh, nw)
    proj = wl.gaussian(400 + case, (npv, nh, nw))
    voxel = (1.0, 1.0, 1.0)
    log("off detector", case, shape, centre, "f16" if f16 else "f32")
    if f16:
        h, sc = fdk.quantize_f16(torch.from_numpy(proj).cuda())
        vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
        fdk.backproject(vol, h, mats, voxel, centre, scale=sc)
        torch.cuda.synchronize()
        got = vol.cpu().numpy()
        ref = oracle.backproject(h.cpu().numpy(), mats, shape, voxel, centre, scale=sc.cpu().numpy())
    else:
        got = gpu_bp(proj, mats, shape, voxel, centre)
        ref = oracle.backproject(proj, mats, shape, voxel, centre)
    e = rel(got, ref)
    log("rel-L2", e, "nonzero", int(np.count_nonzero(ref)))
    assert e <= TOL32
    if not np.any(ref):
        assert not np.any(got)


def _sample_voxels(shape, n, seed):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)], 1)
    corners = np.array([[i, j, k] for i in (0, nx - 1) for j in (0, ny - 1) for k in (0, nz - 1)])
    edges = np.array([[nx // 2, 0, nz // 2], [0, ny // 2, 0], [nx - 1, ny - 1, nz // 2],
                      [nx // 2, ny // 2, nz - 1]])
    return np.concatenate([pts, corners, edges]).astype(np.int64)


def test_c2_full_size_sampled():
    """512^3 x 1024 views x 1024^2 (the benchmark's shape) with float32
    storage, Gaussian projections; sampled voxels against the oracle
    evaluated one by one."""
    cfg = wl.CONFIGS["c2"]
    log("c2: generating", (cfg["np"], cfg["nh"], cfg["nw"]))
    proj = wl.gaussian(2001, (cfg["np"], cfg["nh"], cfg["nw"]))
    mats = og.scan_matrices(cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    log("c2: gpu")
    vol = torch.zeros(cfg["shape"], dtype=torch.float32, device="cuda")
    p = torch.from_numpy(proj).cuda()
    fdk.backproject(vol, p, mats, cfg["voxel"])
    torch.cuda.synchronize()
    ijk = _sample_voxels(cfg["shape"], 384, 7)
    got = vol[ijk[:, 2], ijk[:, 1], ijk[:, 0]].cpu().numpy()
    del vol, p
    log("c2: oracle on", len(ijk), "voxels")
    ref = oracle.backproject_points(proj, mats, cfg["shape"], cfg["voxel"], ijk)
    e = rel(got, ref)
    log("c2 sampled rel-L2", e)
    assert e <= TOL32


def test_c2_full_size_sampled_f16():
    """The benchmark launch itself: 512^3 x 1024 views x 1024^2 with binary16
    storage and per-view scales (the plan's grown FP16 tile).  A seeded
    binary16 stack is the input of both sides; sampled voxels against the
    oracle evaluated one by one on the same values, to the FP32 tolerance."""
    cfg = wl.CONFIGS["c2"]
    shape, npv, nh, nw = cfg["shape"], cfg["np"], cfg["nh"], cfg["nw"]
    log("c2 f16: generating", (npv, nh, nw))
    h, s = wl.device_f16_stack(2002, (npv, nh, nw))
    mats = og.scan_matrices(cfg["scan"], npv, nh, nw)
    plan = fdk.bp_plan(shape, cfg["voxel"], npv, nh, nw, mats, f16=True)
    log("c2 f16: plan", plan)
    assert plan["lds_rows"] % 8 == 4
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    fdk.backproject(vol, h, mats, cfg["voxel"], scale=s)
    torch.cuda.synchronize()
    ijk = _sample_voxels(shape, 384, 17)
    got = vol[ijk[:, 2], ijk[:, 1], ijk[:, 0]].cpu().numpy()
    del vol
    h_np, s_np = h.cpu().numpy(), s.cpu().numpy()
    del h
    log("c2 f16: oracle on", len(ijk), "voxels")
    ref = oracle.backproject_points(h_np, mats, shape, cfg["voxel"], ijk, scale=s_np)
    e = rel(got, ref)
    log("c2 f16 sampled rel-L2", e)
    assert e <= TOL32


def test_c3_full_size_sampled_f16():
    """1024^3 (0.5 mm) x 2048 views x 2048^2, binary16 storage with per-view
    scales: the largest workload, in the launch the library makes for it.
    The stored stack (seeded, generated on the GPU) is the input of both
    sides; sampled voxels against the oracle evaluated one by one on the same
    binary16 values, to the FP32 tolerance."""
    cfg = wl.CONFIGS["c3"]
    shape, npv, nh, nw = cfg["shape"], cfg["np"], cfg["nh"], cfg["nw"]
    log("c3: generating", (npv, nh, nw))
    h, s = wl.device_f16_stack(3001, (npv, nh, nw))
    mats = og.scan_matrices(cfg["scan"], npv, nh, nw)
    log("c3: plan", fdk.bp_plan(shape, cfg["voxel"], npv, nh, nw, mats, f16=True))
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    fdk.backproject(vol, h, mats, cfg["voxel"], scale=s)
    torch.cuda.synchronize()
    ijk = _sample_voxels(shape, 384, 11)
    got = vol[ijk[:, 2], ijk[:, 1], ijk[:, 0]].cpu().numpy()
    del vol
    log("c3: copying the stack to the host")
    h_np, s_np = h.cpu().numpy(), s.cpu().numpy()
    del h
    log("c3: oracle on", len(ijk), "voxels")
    ref = oracle.backproject_points(h_np, mats, shape, cfg["voxel"], ijk, scale=s_np)
    e = rel(got, ref)
    log("c3 sampled rel-L2", e)
    assert e <= TOL32


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_benchmark_stack_subblocks(name):
    """The benchmark's own input and launches: GPU phantom line integrals
    filtered into float32 and (same filter call, binary16 output) into
    binary16 + per-view scale, both back-projected at full size.  The binary16
    stack is bit-equal to the stand-alone pre-pass applied to the float32
    one; over eight 64^3 sub-blocks (centre, corners, edges) against the FP64
    oracle on each view's window: float32 storage <= 1e-5, binary16 storage
    <= 1e-3 against the oracle on the float32 stack and <= 1e-5 against the
    oracle on the dequantised stack; binary16 against float32 storage over
    the whole volume <= 1e-3."""
    cfg = wl.CONFIGS[name]
    log(name, "benchmark stacks", cfg["shape"], (cfg["np"], cfg["nh"], cfg["nw"]))
    filt, h, sc, mats = gpu_phantom_stacks(cfg)
    hq, sq = fdk.quantize_f16(filt)
    torch.cuda.synchronize()
    assert torch.equal(hq.view(torch.int16), h.view(torch.int16))
    assert torch.equal(sq.view(torch.int32), sc.view(torch.int32))
    del hq, sq
    vol32 = torch.zeros(cfg["shape"], dtype=torch.float32, device="cuda")
    vol16 = torch.zeros(cfg["shape"], dtype=torch.float32, device="cuda")
    fdk.backproject(vol32, filt, mats, cfg["voxel"])
    fdk.backproject(vol16, h, mats, cfg["voxel"], scale=sc)
    torch.cuda.synchronize()
    whole = whole_rel(vol16, vol32)
    log(name, "binary16 vs float32 storage, whole volume", whole)
    errs = subblock_errors(cfg, mats, filt, h, sc, vol32, vol16)
    log(name, "sub-blocks", errs)
    del filt, h, sc, vol32, vol16
    torch.cuda.empty_cache()
    assert errs["f32"] <= TOL32
    assert errs["f16"] <= TOL16
    assert errs["f16_dequantised"] <= TOL32
    assert whole <= TOL16


def test_binding_rejects_scale_of_wrong_length():
    """A per-view scale array shorter than the stack would be read past its
    end on the device: the binding refuses it."""
    vol = torch.zeros((4, 8, 8), dtype=torch.float32, device="cuda")
    h = torch.zeros((3, 16, 16), dtype=torch.float16, device="cuda")
    mats = og.scan_matrices(wl.CONFIGS["c1"]["scan"], 3, 16, 16)
    for bad in (torch.ones(2, device="cuda"), torch.ones((3, 1), device="cuda")):
        with pytest.raises(ValueError):
            fdk.backproject(vol, h, mats, (1.0, 1.0, 1.0), scale=bad)


def test_p10_1300cube_sampled():
    """The paper's largest problem (Table 3, P10: 1024^2 x 512 views =>
    1300^3, 8.2 GiB of volume), float32: ragged tiles (1300 = 81 x 16 + 4) and
    a ragged last chunk of slices; sampled voxels against the oracle."""
    from paper_2104_13248_amd import problems
    shape, voxel, mats, nh, nw = problems.geometry("P10")
    npv = problems.VIEWS
    log("p10: generating", (npv, nh, nw))
    proj = wl.gaussian(10010, (npv, nh, nw))
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    p = torch.from_numpy(proj).cuda()
    fdk.backproject(vol, p, mats, voxel)
    torch.cuda.synchronize()
    ijk = _sample_voxels(shape, 384, 13)
    got = vol[ijk[:, 2], ijk[:, 1], ijk[:, 0]].cpu().numpy()
    del vol, p
    ref = oracle.backproject_points(proj, mats, shape, voxel, ijk)
    e = rel(got, ref)
    log("p10 sampled rel-L2", e)
    assert e <= TOL32


# Strongly magnified cone geometries: some blocks' footprints are taller than
# the LDS tile and are staged per half-chunk (the tile keeps only the rows of
# 95% of the footprints: FDK_BP_TILE_BYTES=0 turns off its growth to the
# occupancy limit, which would hold every footprint of these small cases).
SPLIT = [
    (dict(sod=120.0, sdd=400.0), (96, 48, 48), (24, 400, 300)),
    (dict(sod=150.0, sdd=450.0), (64, 40, 40), (24, 320, 256)),
]


@pytest.mark.parametrize("kz", [0, 8, 16, 32])
@pytest.mark.parametrize("case", range(len(SPLIT)))
def test_split_footprints(case, kz, monkeypatch):
    over, shape, (npv, nh, nw) = SPLIT[case]
    monkeypatch.setenv("FDK_BP_TILE_BYTES", "0")
    if kz:
        monkeypatch.setenv("FDK_BP_KZ", str(kz))
    scan = dict(wl.CONFIGS["c1"]["scan"], theta0=0.1, **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    voxel = (1.0, 1.0, 1.0)
    plan = fdk.bp_plan(shape, voxel, npv, nh, nw, mats)
    log("split case", case, "kz", kz, plan)
    if kz == 0:
        assert plan["rows_full"] > plan["lds_rows"], "geometry does not exercise the split path"
    proj = wl.gaussian(400 + case, (npv, nh, nw))
    ref = oracle.backproject(proj, mats, shape, voxel)
    got = gpu_bp(proj, mats, shape, voxel)
    e = rel(got, ref)
    log("f32 rel-L2", e)
    assert e <= TOL32
    h, s = fdk.quantize_f16(torch.from_numpy(proj).cuda())
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    fdk.backproject(vol, h, mats, voxel, scale=s)
    torch.cuda.synchronize()
    ref16 = oracle.backproject(h.cpu().numpy(), mats, shape, voxel, scale=s.cpu().numpy())
    e16 = rel(vol.cpu().numpy(), ref16)
    log("f16 rel-L2 vs dequantised", e16)
    assert e16 <= TOL32
    # slabs stay bitwise equal to the full volume where footprints are split
    p = torch.from_numpy(proj).cuda()
    for k0, kc in [(3, 41), (50, shape[0] - 50)]:
        slab = torch.zeros((kc,) + shape[1:], dtype=torch.float32, device="cuda")
        fdk.backproject_slab(slab, shape, k0, p, mats, voxel)
        torch.cuda.synchronize()
        assert np.array_equal(slab.cpu().numpy().view(np.uint32), got[k0:k0 + kc].view(np.uint32))


# Strong magnification: a 16 x 16 x 8 block's footprint is wider than the
# widest LDS tile, so the library reads the taps from memory (the plan
# reports lds_pitch 0).  Up to ~20 detector pixels per voxel near the centre.
MAGNIFIED = [
    # scan overrides, volume shape, voxel, (np, nh, nw)
    (dict(sod=60.0, sdd=240.0, du=0.2, dv=0.2), (20, 20, 24), 1.0, (16, 420, 460)),
    (dict(sod=90.0, sdd=900.0, du=0.5, dv=0.5, theta0=0.4, u_off=3.0), (9, 14, 11), 1.0, (12, 500, 480)),
]


@pytest.mark.parametrize("case", range(len(MAGNIFIED)))
def test_strong_magnification_direct_taps(case):
    over, shape, vox, (npv, nh, nw) = MAGNIFIED[case]
    scan = dict(wl.CONFIGS["c1"]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    voxel = (vox, vox, vox)
    plan = fdk.bp_plan(shape, voxel, npv, nh, nw, mats)
    log("magnified case", case, plan)
    assert plan["lds_pitch"] == 0
    proj = wl.gaussian(1300 + case, (npv, nh, nw))
    ref = oracle.backproject(proj, mats, shape, voxel)
    got = gpu_bp(proj, mats, shape, voxel)
    e = rel(got, ref)
    log("f32 rel-L2", e)
    assert e <= TOL32
    h, s = fdk.quantize_f16(torch.from_numpy(proj).cuda())
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    fdk.backproject(vol, h, mats, voxel, scale=s)
    torch.cuda.synchronize()
    ref16 = oracle.backproject(h.cpu().numpy(), mats, shape, voxel, scale=s.cpu().numpy())
    e16 = rel(vol.cpu().numpy(), ref16)
    log("f16 rel-L2 vs dequantised", e16)
    assert e16 <= TOL32


@pytest.mark.parametrize("kz", [0, 8, 16])
def test_direct_organisation_forced(kz, monkeypatch):
    """The direct organisation on an ordinary geometry (FDK_BP_DIRECT=1):
    parity, binary16 storage, accumulation and z-slabs bitwise equal to the
    full volume."""
    monkeypatch.setenv("FDK_BP_DIRECT", "1")
    if kz:
        monkeypatch.setenv("FDK_BP_KZ", str(kz))
    shape, (npv, nh, nw) = (37, 19, 33), (21, 45, 61)
    scan = dict(wl.CONFIGS["c1"]["scan"], theta0=0.3, u_off=1.7, v_off=-2.2)
    mats = og.scan_matrices(scan, npv, nh, nw)
    voxel, centre = (0.9, 1.1, 1.3), (2.0, -3.0, 1.5)
    assert fdk.bp_plan(shape, voxel, npv, nh, nw, mats, centre)["lds_pitch"] == 0
    proj = wl.gaussian(1400 + kz, (npv, nh, nw))
    base = wl.gaussian(1450 + kz, shape)
    got = gpu_bp(proj, mats, shape, voxel, centre, vol0=base)
    ref = oracle.backproject(proj, mats, shape, voxel, centre, vol=base.astype(np.float64))
    assert rel(got, ref) <= TOL32
    full = gpu_bp(proj, mats, shape, voxel, centre)
    p = torch.from_numpy(proj).cuda()
    for k0, kc in [(0, 37), (3, 11), (36, 1)]:
        slab = torch.zeros((kc,) + shape[1:], dtype=torch.float32, device="cuda")
        fdk.backproject_slab(slab, shape, k0, p, mats, voxel, centre)
        torch.cuda.synchronize()
        assert np.array_equal(slab.cpu().numpy().view(np.uint32), full[k0:k0 + kc].view(np.uint32))
    h, s = fdk.quantize_f16(p)
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    fdk.backproject(vol, h, mats, voxel, centre, scale=s)
    torch.cuda.synchronize()
    ref16 = oracle.backproject(h.cpu().numpy(), mats, shape, voxel, centre, scale=s.cpu().numpy())
    assert rel(vol.cpu().numpy(), ref16) <= TOL32
