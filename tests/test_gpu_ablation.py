"""Back-projection variants of include/fdk_ablation.h against the FP64 oracle
(MI355X): each organisation computes the same operation."""
import numpy as np
import pytest

import oracle
from oracle import geometry as og
import workloads as wl
from helpers import log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdk = pytest.importorskip("paper_2104_13248_amd")
from paper_2104_13248_amd.ablations import backproject_variant  # noqa: E402

CASES = [
    # shape, (np, nh, nw), scan overrides, centre
    ((40, 36, 44), (23, 96, 80), dict(theta0=0.3), (1.0, -2.0, 0.5)),
    ((17, 33, 50), (11, 70, 90), dict(u_off=2.5, v_off=-1.0), (0.0, 0.0, 0.0)),
]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.mark.parametrize("variant,nb", [("production", 5), ("global_taps", None),
                                        ("listing1", 1), ("listing1", 7), ("listing1", None)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_variant_parity(variant, nb, case):
    shape, (npv, nh, nw), over, centre = CASES[case]
    scan = dict(wl.CONFIGS["c1"]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    proj = wl.gaussian(4500 + case, (npv, nh, nw))
    base = wl.gaussian(4600 + case, shape)
    vol = torch.from_numpy(base).cuda()
    backproject_variant(vol, torch.from_numpy(proj).cuda(), mats, (1.0, 1.0, 1.0), variant, nb,
                        centre)
    torch.cuda.synchronize()
    ref = oracle.backproject(proj, mats, shape, (1.0, 1.0, 1.0), centre) + base
    e = rel(vol.cpu().numpy(), ref)
    log(variant, nb, case, "rel-L2", e)
    assert e <= 1e-5


# Symmetric geometries (detector centre row on the orbit plane, volume centred
# on it in z): even nz; odd nz (the middle slice is its own mirror); and a
# magnified cone whose windows exceed one LDS region (staged one at a time).
SYM_CASES = [
    ((40, 36, 44), (23, 96, 80), dict(theta0=0.3), (1.0, -2.0, 0.0)),
    ((17, 33, 50), (11, 70, 91), dict(u_off=2.5), (0.0, 0.0, 0.0)),
    ((96, 48, 48), (24, 400, 300), dict(sod=120.0, sdd=400.0, theta0=0.1), (0.0, 0.0, 0.0)),
]


@pytest.mark.parametrize("case", range(len(SYM_CASES)))
def test_symmetry_variant_parity(case):
    shape, (npv, nh, nw), over, centre = SYM_CASES[case]
    scan = dict(wl.CONFIGS["c1"]["scan"], v_off=0.0, **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    proj = wl.gaussian(4700 + case, (npv, nh, nw))
    base = wl.gaussian(4800 + case, shape)
    vol = torch.from_numpy(base).cuda()
    backproject_variant(vol, torch.from_numpy(proj).cuda(), mats, (1.0, 1.0, 1.0), "symmetry",
                        None, centre)
    torch.cuda.synchronize()
    ref = oracle.backproject(proj, mats, shape, (1.0, 1.0, 1.0), centre) + base
    e = rel(vol.cpu().numpy(), ref)
    log("symmetry", case, "rel-L2", e)
    assert e <= 1e-5


# Sub-line variant: the C1 orbit, a magnified cone (tall windows, long lines),
# a demagnified one (dv < 1: several slices per detector row, short lines),
# ragged tiles and an off-centre detector.
SUBLINE_CASES = [
    ((40, 36, 44), (23, 96, 80), dict(theta0=0.3), (1.0, -2.0, 0.5), None),
    ((96, 48, 48), (24, 400, 300), dict(sod=120.0, sdd=400.0, theta0=0.1), (0.0, 0.0, 0.0), None),
    ((70, 34, 29), (19, 24, 40), dict(du=4.0, dv=4.0, u_off=1.5, v_off=-2.0), (0.0, 0.0, 0.0), None),
    ((33, 17, 15), (13, 60, 70), dict(theta0=1.1), (0.0, 0.0, 2.0), 16),
    ((33, 17, 15), (13, 60, 70), dict(theta0=1.1), (0.0, 0.0, 2.0), 8),
]


@pytest.mark.parametrize("case", range(len(SUBLINE_CASES)))
def test_subline_variant_parity(case, monkeypatch):
    shape, (npv, nh, nw), over, centre, kz = SUBLINE_CASES[case]
    if kz:
        monkeypatch.setenv("FDK_BP_KZ", str(kz))
    scan = dict(wl.CONFIGS["c1"]["scan"], **over)
    mats = og.scan_matrices(scan, npv, nh, nw)
    proj = wl.gaussian(4900 + case, (npv, nh, nw))
    base = wl.gaussian(4950 + case, shape)
    vol = torch.from_numpy(base).cuda()
    backproject_variant(vol, torch.from_numpy(proj).cuda(), mats, (1.0, 1.0, 1.0), "subline",
                        None, centre)
    torch.cuda.synchronize()
    ref = oracle.backproject(proj, mats, shape, (1.0, 1.0, 1.0), centre) + base
    e = rel(vol.cpu().numpy(), ref)
    log("subline", case, "rel-L2", e)
    assert e <= 1e-5
