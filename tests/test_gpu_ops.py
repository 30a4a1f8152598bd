"""Parity of the forward projector, the FDK filter and the analytic phantom
projector with the FP64 oracle, and the end-to-end FDK pipeline (MI355X)."""
import math

import numpy as np
import pytest

import oracle
from oracle import geometry as og
from oracle import phantom as oph
import workloads as wl
from helpers import c1_filtered, log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdk = pytest.importorskip("paper_2104_13248_amd")

TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def gpu_fp(vol, mats, nh, nw, voxel, centre=(0.0, 0.0, 0.0), proj0=None):
    v = torch.from_numpy(np.ascontiguousarray(vol, dtype=np.float32)).cuda()
    p = torch.zeros((len(mats), nh, nw), dtype=torch.float32, device="cuda") if proj0 is None \
        else torch.from_numpy(np.ascontiguousarray(proj0, dtype=np.float32)).cuda()
    fdk.forwardproject(v, p, mats, voxel, centre)
    torch.cuda.synchronize()
    return p.cpu().numpy()


FP_CASES = [
    # config, shape, (np, nh, nw), scan overrides, centre
    ("c1", (64, 64, 64), (64, 128, 128), {}, (0.0, 0.0, 0.0)),
    ("c1", (9, 21, 17), (37, 50, 70), dict(theta0=0.4, u_off=2.5, v_off=-1.0), (1.0, -2.0, 3.0)),
    ("c1", (96, 48, 48), (24, 400, 300), dict(sod=120.0, sdd=400.0), (0.0, 0.0, 0.0)),
    # odd detector width: a full 256-column chunk and a ragged one of 45
    ("c1", (20, 18, 22), (16, 40, 301), dict(theta0=0.7, u_off=-1.5), (0.5, 0.0, -1.0)),
]


@pytest.mark.parametrize("case", range(len(FP_CASES)))
def test_forward_projection_parity(case):
    name, shape, (npv, nh, nw), over, centre = FP_CASES[case]
    scan = dict(wl.CONFIGS[name]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    x = wl.gaussian(500 + case, shape)
    got = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre)
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, (1.0, 1.0, 1.0), centre)
    e = rel(got, ref)
    log("fp case", case, "rel-L2", e)
    assert e <= TOL32


@pytest.fixture
def small_fp_budget(monkeypatch):
    """Forward-projector LDS budget of a few rows, so that every detector is
    split into many row bands (band boundaries inside every footprint)."""
    monkeypatch.setenv("FDK_FP_LDS_BUDGET", "2600")


@pytest.mark.parametrize("case", range(len(FP_CASES)))
def test_forward_projection_many_bands(case, small_fp_budget):
    name, shape, (npv, nh, nw), over, centre = FP_CASES[case]
    scan = dict(wl.CONFIGS[name]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    rb = fdk.bp_plan(shape, (1.0, 1.0, 1.0), npv, nh, nw, mats, centre)["fp_rows"]
    assert rb < nh // 3
    x = wl.gaussian(540 + case, shape)
    got = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre)
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, (1.0, 1.0, 1.0), centre)
    e = rel(got, ref)
    log("fp many bands case", case, "rb", rb, "rel-L2", e)
    assert e <= TOL32


@pytest.mark.parametrize("chunk", [16, 40])
@pytest.mark.parametrize("case", [1, 2, 3])
def test_forward_projection_narrow_chunks(case, chunk, monkeypatch):
    """Column chunks of 16 or 40 detector columns, so that most voxels have
    their two u-taps in neighbouring chunks (each chunk's window drops the
    tap outside it and the neighbour adds it)."""
    monkeypatch.setenv("FDK_FP_CHUNK", str(chunk))
    name, shape, (npv, nh, nw), over, centre = FP_CASES[case]
    scan = dict(wl.CONFIGS[name]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    cw = fdk.bp_plan(shape, (1.0, 1.0, 1.0), npv, nh, nw, mats, centre)["fp_cols"]
    assert cw <= chunk and -(-nw // cw) >= 2
    x = wl.gaussian(620 + case, shape)
    got = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre)
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, (1.0, 1.0, 1.0), centre)
    e = rel(got, ref)
    log("fp narrow chunks", case, chunk, cw, "rel-L2", e)
    assert e <= TOL32


@pytest.mark.parametrize("theta0", [math.pi / 2 - 0.3, -0.3, 0.25 * math.pi - 0.3])
def test_forward_projection_view_orientations(theta0):
    """Short arcs whose views all run lanes along x (no transposed copy), all
    along y (transposed copy only), and a mix across the 45-degree switch."""
    cfg = wl.CONFIGS["c1"]
    scan = dict(cfg["scan"], arc=0.6, theta0=theta0)
    shape, npv, nh, nw = (40, 36, 44), 20, 64, 96
    mats = og.scan_matrices(scan, npv, nh, nw)
    x = wl.gaussian(560, shape)
    got = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0))
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, (1.0, 1.0, 1.0))
    assert rel(got, ref) <= TOL32


def test_forward_projection_c5_geometry():
    """Magnification-2 sampling of the learned-filter workload (0.25 mm voxels,
    0.25 mm pixels) on a 48^3 crop, 30 views, full 512^2 detector."""
    cfg = wl.CONFIGS["c5"]
    mats = og.scan_matrices(cfg["scan"], 30, cfg["nh"], cfg["nw"])
    x = wl.gaussian(570, (48, 48, 48))
    centre = (1.5, -2.0, 0.75)
    got = gpu_fp(x, mats, cfg["nh"], cfg["nw"], cfg["voxel"], centre)
    ref = oracle.forwardproject(x.astype(np.float64), mats, cfg["nh"], cfg["nw"], cfg["voxel"],
                                centre)
    assert rel(got, ref) <= TOL32


def test_forward_projection_is_deterministic():
    name, shape, (npv, nh, nw), over, centre = FP_CASES[1]
    mats = og.scan_matrices(dict(wl.CONFIGS[name]["scan"], **over), npv, nh, nw)
    x = wl.gaussian(580, shape)
    a = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre)
    b = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre)
    assert np.array_equal(a, b)


def test_forward_projection_accumulates():
    name, shape, (npv, nh, nw), over, centre = FP_CASES[1]
    mats = og.scan_matrices(dict(wl.CONFIGS[name]["scan"], **over), npv, nh, nw)
    x = wl.gaussian(510, shape)
    base = wl.gaussian(511, (npv, nh, nw))
    got = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre, proj0=base)
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, (1.0, 1.0, 1.0), centre,
                                proj=base.astype(np.float64))
    assert rel(got, ref) <= TOL32


@pytest.mark.parametrize("case", range(len(FP_CASES)))
def test_adjoint_identity_on_gpu(case):
    """<BP p, x> = <p, FP x> with both operators from the HIP library."""
    name, shape, (npv, nh, nw), over, centre = FP_CASES[case]
    mats = og.scan_matrices(dict(wl.CONFIGS[name]["scan"], **over), npv, nh, nw)
    p = wl.gaussian(520 + case, (npv, nh, nw))
    x = wl.gaussian(530 + case, shape)
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    fdk.backproject(vol, torch.from_numpy(p).cuda(), mats, (1.0, 1.0, 1.0), centre)
    fpx = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre)
    bp = vol.cpu().numpy().astype(np.float64)
    lhs = float(np.sum(bp * x))
    rhs = float(np.sum(p.astype(np.float64) * fpx))
    scale = np.linalg.norm(bp) * np.linalg.norm(x)
    log("adjoint", case, lhs, rhs, abs(lhs - rhs) / scale)
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_adjoint_identity_precision_workload_scale():
    """<BP p, x> = <p, FP x> at the scale of the 1024^3 precision workload:
    0.5 mm voxels, 64 views over 360 degrees, 2048^2 detector (4 MiB slices,
    nine column chunks of the forward projector, views on both lane axes)."""
    cfg = wl.CONFIGS["c3"]
    npv = 64
    mats = og.scan_matrices(cfg["scan"], npv, cfg["nh"], cfg["nw"])
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    x = torch.randn(cfg["shape"], device="cuda", generator=g)
    p = torch.randn((npv, cfg["nh"], cfg["nw"]), device="cuda", generator=g)
    vol = torch.zeros(cfg["shape"], dtype=torch.float32, device="cuda")
    fdk.backproject(vol, p, mats, cfg["voxel"])
    fpx = torch.zeros_like(p)
    fdk.forwardproject(x, fpx, mats, cfg["voxel"])
    torch.cuda.synchronize()
    lhs = float(torch.sum(vol.double() * x.double()))
    rhs = float(torch.sum(p.double() * fpx.double()))
    scale = float(vol.double().norm() * x.double().norm())
    log("adjoint at 1024^3 x 64 x 2048^2", lhs, rhs, abs(lhs - rhs) / scale)
    assert abs(lhs - rhs) <= 1e-5 * scale
    assert float(fpx.abs().max()) > 0.0


def test_filter_parity():
    cfg = wl.CONFIGS["c1"]
    ell = wl.config_ellipsoids(cfg, 0)
    raw = oph.line_integrals(ell, cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"]).astype(np.float32)
    out = fdk.fdk_filter(torch.from_numpy(raw).cuda(), cfg["scan"])
    torch.cuda.synchronize()
    ref = oracle.fdk_filter(raw.astype(np.float64), cfg["scan"])
    e = rel(out.cpu().numpy(), ref)
    log("filter rel-L2", e)
    assert e <= TOL32


@pytest.mark.parametrize("nw", [1, 2, 7, 300, 1027, 2048, 2049])
def test_filter_ragged_rows(nw):
    scan = dict(sod=600.0, sdd=1100.0, du=0.8, dv=1.2, arc=2 * math.pi, theta0=0.0,
                u_off=1.5, v_off=-0.5)
    raw = wl.gaussian(600 + nw, (3, 5, nw))
    out = fdk.fdk_filter(torch.from_numpy(raw).cuda(), scan, np_total=360)
    torch.cuda.synchronize()
    ref = oracle.fdk_filter(raw.astype(np.float64), scan, np_total=360)
    assert rel(out.cpu().numpy(), ref) <= TOL32


# Both ends of every transform length's row range (M = the power of two
# >= 2 nw - 1, at least 16): nw = M / 2 fills the unpadded half exactly,
# nw = M / 4 + 1 is the narrowest row of that length.
@pytest.mark.parametrize("nw", [8, 9, 16, 17, 32, 33, 64, 65, 128, 129, 256, 257, 512, 513,
                                1024, 1025])
def test_filter_every_transform_length(nw):
    """Float32 output against the FP64 filter, and the binary16 output (the
    kernels that also take the per-view maxima) bit for bit against the
    storage rule applied to that float32 output.  Five rows per view: row
    pairs that span two views."""
    scan = dict(sod=600.0, sdd=1100.0, du=0.8, dv=1.2, arc=2 * math.pi, theta0=0.0,
                u_off=-2.5, v_off=0.5)
    raw = wl.gaussian(800 + nw, (3, 5, nw))
    raw_d = torch.from_numpy(raw).cuda()
    out = fdk.fdk_filter(raw_d, scan, np_total=360)
    h, s = fdk.fdk_filter(raw_d, scan, np_total=360, dtype=torch.float16)
    torch.cuda.synchronize()
    ref = oracle.fdk_filter(raw.astype(np.float64), scan, np_total=360)
    assert rel(out.cpu().numpy(), ref) <= TOL32
    h_ref, s_ref = oracle.quantize_f16(out.cpu().numpy())
    assert np.array_equal(s.cpu().numpy().view(np.uint32), s_ref.view(np.uint32))
    assert np.array_equal(h.cpu().numpy().view(np.uint16), h_ref.view(np.uint16))


F16_FILTER_CASES = [
    # (np, nh, nw), raw: "phantom" (C1 phantom views) or "gaussian"
    ((64, 128, 128), "phantom"),
    ((5, 3, 7), "gaussian"),          # odd rows: a row pair spans two views
    ((6, 9, 2049), "gaussian"),       # direct-convolution rows, odd nh
    ((10, 2048, 2048), "gaussian"),   # three chunks of the 64 MiB workspace (4 + 4 + 2 views)
]


@pytest.mark.parametrize("case", range(len(F16_FILTER_CASES)))
def test_filter_f16_output(case):
    """fdk_filter with binary16 output = the FP16 storage rule applied to its
    own float32 output (bit for bit, both against the library's stand-alone
    pre-pass and against the oracle's rule), and within the binary16 rounding
    of the FP64 filter."""
    (npv, nh, nw), kind = F16_FILTER_CASES[case]
    scan = dict(sod=600.0, sdd=1100.0, du=0.8, dv=1.2, arc=2 * math.pi, theta0=0.0,
                u_off=1.5, v_off=-0.5)
    if kind == "phantom":
        cfg = wl.CONFIGS["c1"]
        scan = cfg["scan"]
        raw = oph.line_integrals(wl.config_ellipsoids(cfg, 0), scan, npv, nh, nw).astype(np.float32)
        raw[3] = 0.0                                 # an all-zero view: scale 1
        raw[5] *= np.float32(1e-20)                  # tiny values: binary16 subnormals
    else:
        raw = wl.gaussian(700 + case, (npv, nh, nw))
    raw_d = torch.from_numpy(raw).cuda()
    out32 = fdk.fdk_filter(raw_d, scan, np_total=360)
    h, s = fdk.fdk_filter(raw_d, scan, np_total=360, dtype=torch.float16)
    hq, sq = fdk.quantize_f16(out32)
    torch.cuda.synchronize()
    assert torch.equal(h.view(torch.int16), hq.view(torch.int16))
    assert torch.equal(s.view(torch.int32), sq.view(torch.int32))
    h_ref, s_ref = oracle.quantize_f16(out32.cpu().numpy())
    assert np.array_equal(s.cpu().numpy().view(np.uint32), s_ref.view(np.uint32))
    assert np.array_equal(h.cpu().numpy().view(np.uint16), h_ref.view(np.uint16))
    nv = min(npv, 2)                                 # FP64 filter on the first views
    ref = oracle.fdk_filter(raw[:nv].astype(np.float64), scan, np_total=360)
    deq = (h[:nv].float() * s[:nv, None, None]).cpu().numpy()
    e = rel(deq, ref)
    log("filter f16 case", case, "rel-L2 of the dequantised output vs FP64 filter", e)
    assert e <= 1e-3
    del raw_d, out32, h, s, hq, sq
    torch.cuda.empty_cache()


def test_phantom_projector_parity():
    cfg = wl.CONFIGS["c1"]
    scan = dict(cfg["scan"], theta0=0.25, u_off=0.5, v_off=-1.5)
    ell = wl.config_ellipsoids(cfg, 3)
    views = 16
    p = torch.zeros((views, cfg["nh"], cfg["nw"]), dtype=torch.float32, device="cuda")
    fdk.phantom_project(ell, scan, p, view_begin=8, np_total=cfg["np"])
    torch.cuda.synchronize()
    ref = oph.line_integrals(ell, scan, cfg["np"], cfg["nh"], cfg["nw"], views=np.arange(8, 8 + views))
    e = rel(p.cpu().numpy(), ref)
    log("phantom rel-L2", e)
    assert e <= 1e-6


def test_fdk_pipeline_on_gpu():
    """GPU phantom -> GPU filter -> GPU back-projection against the oracle
    pipeline (oracle phantom -> oracle filter -> oracle back-projection)."""
    cfg = wl.CONFIGS["c1"]
    scan = cfg["scan"]
    ell = wl.config_ellipsoids(cfg, 1)
    raw = torch.zeros((cfg["np"], cfg["nh"], cfg["nw"]), dtype=torch.float32, device="cuda")
    fdk.phantom_project(ell, scan, raw)
    filt = fdk.fdk_filter(raw, scan)
    mats = fdk.scan_matrices(scan, cfg["np"], cfg["nh"], cfg["nw"])
    vol = torch.zeros(cfg["shape"], dtype=torch.float32, device="cuda")
    fdk.backproject(vol, filt, mats, cfg["voxel"])
    torch.cuda.synchronize()
    ref_proj, ref_mats = c1_filtered(1)
    ref = oracle.backproject(ref_proj, ref_mats, cfg["shape"], cfg["voxel"])
    e = rel(vol.cpu().numpy(), ref)
    log("pipeline rel-L2", e)
    assert e <= 1e-5


def test_forward_projection_c4_full_size_views():
    """The C4 launch itself (256^3 at 0.25 mm, 360 views, 384^2 detector):
    element-wise against the oracle on eight of the 360 views (all quadrants,
    both lane axes of the voxel-driven kernel)."""
    cfg = wl.CONFIGS["c4"]
    npv, nh, nw = cfg["np"], cfg["nh"], cfg["nw"]
    mats = og.scan_matrices(cfg["scan"], npv, nh, nw)
    x = wl.gaussian(4101, cfg["shape"])
    log("c4 fp: gpu")
    got = gpu_fp(x, mats, nh, nw, cfg["voxel"])
    sel = np.array([0, 45, 89, 90, 137, 180, 271, 359])
    log("c4 fp: oracle on views", sel)
    ref = oracle.forwardproject(x.astype(np.float64), mats[sel], nh, nw, cfg["voxel"])
    e = rel(got[sel], ref)
    log("c4 fp: rel-L2 on 8 views", e)
    assert e <= TOL32


@pytest.fixture
def gather_organisation(monkeypatch):
    """The column-owned organisation the library falls back to when the
    voxel-driven kernel's load offsets would not fit (huge slices)."""
    monkeypatch.setenv("FDK_FP_ALGO", "gather")


@pytest.mark.parametrize("case", range(len(FP_CASES)))
def test_forward_projection_gather_organisation(case, gather_organisation):
    name, shape, (npv, nh, nw), over, centre = FP_CASES[case]
    scan = dict(wl.CONFIGS[name]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    assert fdk.bp_plan(shape, (1.0, 1.0, 1.0), npv, nh, nw, mats, centre)["fp_cols"] == min(nw, 256)
    x = wl.gaussian(590 + case, shape)
    got = gpu_fp(x, mats, nh, nw, (1.0, 1.0, 1.0), centre)
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, (1.0, 1.0, 1.0), centre)
    assert rel(got, ref) <= TOL32


@pytest.mark.parametrize("voxel,pitch", [(0.25, 1.4), (2.5, 0.5)])
def test_forward_projection_lane_strides(voxel, pitch):
    """Pixels much wider than the magnified voxel (several voxels per column:
    lane strides of 4 and more) and much narrower (five columns per voxel:
    stride 1), both at a 45-degree view where neither axis dominates."""
    scan = dict(sod=300.0, sdd=600.0, du=pitch, dv=pitch, arc=0.5 * math.pi,
                theta0=0.25 * math.pi, u_off=0.5, v_off=-0.5)
    shape, npv = (24, 40, 36), 9
    nh = nw = int(2.6 * 40 * voxel / pitch) + 8
    mats = og.scan_matrices(scan, npv, nh, nw)
    x = wl.gaussian(600, shape)
    got = gpu_fp(x, mats, nh, nw, (voxel,) * 3)
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, (voxel,) * 3)
    e = rel(got, ref)
    log("fp lane strides", voxel, pitch, nh, "rel-L2", e)
    assert e <= TOL32
