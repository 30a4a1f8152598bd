"""Differentiation through the back-projector (MI355X): the backward of
BackProject is the exact transpose (forward projection).

Checks: the dot-product test on seeded Gaussian x, y; central finite
differences of a loss on 32^3 crops of the differentiation workload's
geometry (256^3 / 0.25 mm, 360 views, 384^2 detector), which, BP being linear,
must equal the directional derivative <backward(g), d> exactly up to rounding;
a batch of volumes; and the mirror pair ForwardProject.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdk = pytest.importorskip("paper_2104_13248_amd")
from paper_2104_13248_amd.autograd import Geometry, back_project, forward_project  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def crop_geometry(offset=(0.0, 0.0, 0.0), n=32, np_views=360):
    """A 32^3 crop of the 256^3 / 0.25 mm differentiation volume, centred at
    ``offset`` (mm), with that workload's scanner."""
    cfg = wl.CONFIGS["c4"]
    return Geometry.circular((n, n, n), cfg["voxel"], cfg["scan"], np_views, cfg["nh"], cfg["nw"],
                             centre=offset)


def test_dot_product_test_c4():
    g = crop_geometry((3.0, -2.0, 4.5))
    x = torch.from_numpy(wl.gaussian(4001, (g.np, g.nh, g.nw))).cuda()
    y = torch.from_numpy(wl.gaussian(4002, g.shape)).cuda()
    bx = back_project(x, g)
    fy = forward_project(y, g)
    lhs = float((bx.double() * y.double()).sum())
    rhs = float((x.double() * fy.double()).sum())
    scale = float(bx.double().norm() * y.double().norm())
    log("dot test", lhs, rhs, abs(lhs - rhs) / scale)
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_backward_is_forward_projection():
    g = crop_geometry()
    p = torch.from_numpy(wl.gaussian(4010, (g.np, g.nh, g.nw))).cuda().requires_grad_(True)
    w = torch.from_numpy(wl.gaussian(4011, g.shape)).cuda()
    loss = (back_project(p, g) * w).sum()
    loss.backward()
    ref = oracle.forwardproject(w.cpu().numpy().astype(np.float64), g.mats, g.nh, g.nw, g.voxel,
                                g.centre)
    e = rel(p.grad.cpu().numpy(), ref)
    log("grad vs oracle FP", e)
    assert e <= 1e-5


def test_central_finite_differences():
    """L(p) = 0.5 |BP(p) - t|^2.  For a random direction d the central
    difference (L(p + h d) - L(p - h d)) / 2h equals <grad L, d> for this
    quadratic (exactly, in exact arithmetic)."""
    g = crop_geometry((-5.0, 6.0, -2.0))
    p0 = torch.from_numpy(wl.gaussian(4020, (g.np, g.nh, g.nw))).cuda()
    t = torch.from_numpy(wl.gaussian(4021, g.shape)).cuda()
    d = torch.from_numpy(wl.gaussian(4022, (g.np, g.nh, g.nw))).cuda()
    p = p0.clone().requires_grad_(True)
    loss = 0.5 * ((back_project(p, g) - t) ** 2).sum()
    loss.backward()
    analytic = float((p.grad.double() * d.double()).sum())
    h = 1e-2

    def L(q):
        with torch.no_grad():
            r = back_project(q, g).double() - t.double()
            return 0.5 * float((r * r).sum())
    fd = (L(p0 + h * d) - L(p0 - h * d)) / (2 * h)
    log("FD", fd, "analytic", analytic)
    assert abs(fd - analytic) <= 2e-4 * abs(analytic)


def test_batched_volumes_and_forward_project_grad():
    g = crop_geometry((0.0, 0.0, 0.0), np_views=90)
    B = 3
    vol = torch.from_numpy(wl.gaussian(4030, (B,) + g.shape)).cuda().requires_grad_(True)
    proj = forward_project(vol, g)
    assert proj.shape == (B, g.np, g.nh, g.nw)
    w = torch.from_numpy(wl.gaussian(4031, (B, g.np, g.nh, g.nw))).cuda()
    (proj * w).sum().backward()
    for b in range(B):
        ref = oracle.backproject(w[b].cpu().numpy(), g.mats, g.shape, g.voxel, g.centre)
        assert rel(vol.grad[b].cpu().numpy(), ref) <= 1e-5


def test_differentiation_workload_full_batch():
    """The differentiation workload at full size through the autograd pair: a
    batch of 8 volumes of 256^3 (0.25 mm), 360 views, 384^2 detector.  With
    vol = BP(p) and p.grad = FP(y) (the backward of <BP p, y>), every item
    satisfies <BP p, y> = <p, FP y>."""
    cfg = wl.CONFIGS["c4"]
    g = Geometry.circular(cfg["shape"], cfg["voxel"], cfg["scan"], cfg["np"], cfg["nh"], cfg["nw"])
    B = cfg["batch"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4040)
    p = torch.randn((B, g.np, g.nh, g.nw), device="cuda", generator=gen).requires_grad_(True)
    y = torch.randn((B,) + g.shape, device="cuda", generator=gen)
    vol = back_project(p, g)
    assert vol.shape == (B,) + tuple(g.shape)
    (vol * y).sum().backward()
    for b in range(B):
        lhs = float((vol[b].detach().double() * y[b].double()).sum())
        rhs = float((p[b].detach().double() * p.grad[b].double()).sum())
        scale = float(vol[b].detach().double().norm() * y[b].double().norm())
        log("batch item", b, lhs, rhs, abs(lhs - rhs) / scale)
        assert abs(lhs - rhs) <= 1e-5 * scale
