"""Randomised parity: small random volumes, detectors and circular-orbit
geometries (derandomised Hypothesis examples, so every run draws the same
cases) for the back-projector (float32 and binary16 storage) and the
forward projector, against the oracle.

Every drawn volume fits in a sphere of radius < 50 mm about the isocentre
(<= 40 voxels of <= 1.25 mm, centre offsets <= 3 mm) and the source is at
least 80 mm away, so every voxel is in front of the source (w > 0).
Magnifications reach ~20 detector pixels per voxel near the source, beyond
the widest LDS tile: the back-projector then reads its taps from memory.
Forward-projection cases outside its window plan are not drawn."""
from __future__ import annotations

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
hypothesis = pytest.importorskip("hypothesis")
from hypothesis import assume, given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
from oracle import geometry as og  # noqa: E402
import workloads as wl  # noqa: E402
from helpers import log  # noqa: E402

import paper_2104_13248_amd as fdk  # noqa: E402

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


CASE = st.fixed_dictionaries({
    "shape": st.tuples(st.integers(1, 40), st.integers(1, 40), st.integers(1, 40)),
    "views": st.integers(1, 24),
    "det": st.tuples(st.integers(4, 90), st.integers(4, 90)),
    "voxel": st.tuples(*(st.sampled_from([0.5, 0.75, 1.0, 1.25]) for _ in range(3))),
    "centre": st.tuples(*(st.floats(-3.0, 3.0) for _ in range(3))),
    "theta0": st.floats(0.0, 2.0 * math.pi),
    "arc": st.sampled_from([0.5, math.pi, 2.0 * math.pi]),
    "offsets": st.tuples(st.floats(-3.0, 3.0), st.floats(-3.0, 3.0)),
    "sod": st.floats(80.0, 200.0),
    "mag": st.floats(1.2, 4.0),
    "pitch": st.tuples(st.sampled_from([0.25, 0.6, 1.0, 1.4]),
                       st.sampled_from([0.25, 0.6, 1.0, 1.4])),
    "seed": st.integers(0, 10 ** 6),
})


def _scan(c):
    return dict(sod=c["sod"], sdd=c["sod"] * c["mag"], du=c["pitch"][0], dv=c["pitch"][1],
                arc=c["arc"], theta0=c["theta0"], u_off=c["offsets"][0], v_off=c["offsets"][1])


def _fp_supported(c, mats) -> bool:
    nh, nw = c["det"]
    return fdk.bp_plan(c["shape"], c["voxel"], c["views"], nh, nw, mats, c["centre"])["fp_cols"] > 0


def _rel(got, ref):
    nr = np.linalg.norm(ref)
    if nr == 0.0:
        return float(np.linalg.norm(got))
    return float(np.linalg.norm(got - ref) / nr)


@settings(max_examples=16, deadline=None, derandomize=True, database=None)
@given(CASE)
def test_random_backprojection(c):
    nh, nw = c["det"]
    mats = og.scan_matrices(_scan(c), c["views"], nh, nw)
    plan = fdk.bp_plan(c["shape"], c["voxel"], c["views"], nh, nw, mats, c["centre"])
    proj = wl.gaussian(c["seed"], (c["views"], nh, nw))
    p = torch.from_numpy(proj).cuda()
    vol = torch.zeros(c["shape"], dtype=torch.float32, device="cuda")
    fdk.backproject(vol, p, mats, c["voxel"], c["centre"])
    h, s = fdk.quantize_f16(p)
    vol16 = torch.zeros(c["shape"], dtype=torch.float32, device="cuda")
    fdk.backproject(vol16, h, mats, c["voxel"], c["centre"], scale=s)
    torch.cuda.synchronize()
    ref = oracle.backproject(proj, mats, c["shape"], c["voxel"], c["centre"])
    ref16 = oracle.backproject(h.cpu().numpy(), mats, c["shape"], c["voxel"], c["centre"],
                               scale=s.cpu().numpy())
    e, e16 = _rel(vol.cpu().numpy(), ref), _rel(vol16.cpu().numpy(), ref16)
    log("random bp", c["shape"], (c["views"], nh, nw), "pitch", plan["lds_pitch"], "rel-L2", e,
        "f16 vs dequantised", e16)
    assert e <= TOL32 and e16 <= TOL32


@settings(max_examples=12, deadline=None, derandomize=True, database=None)
@given(CASE)
def test_random_forward_projection(c):
    nh, nw = c["det"]
    mats = og.scan_matrices(_scan(c), c["views"], nh, nw)
    assume(_fp_supported(c, mats))
    x = wl.gaussian(c["seed"] + 1, c["shape"])
    v = torch.from_numpy(x).cuda()
    p = torch.zeros((c["views"], nh, nw), dtype=torch.float32, device="cuda")
    fdk.forwardproject(v, p, mats, c["voxel"], c["centre"])
    torch.cuda.synchronize()
    ref = oracle.forwardproject(x.astype(np.float64), mats, nh, nw, c["voxel"], c["centre"])
    e = _rel(p.cpu().numpy(), ref)
    log("random fp", c["shape"], (c["views"], nh, nw), "rel-L2", e)
    assert e <= TOL32
