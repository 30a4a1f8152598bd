"""fdk_backproject_noalloc (no allocation; fixed per-GPU scratch array)
against fdk_backproject, both called through the C ABI (MI355X): bitwise
equal outputs on consecutive calls, the second with a smaller input (the
shared scratch keeps the previous call's entries), float32 and binary16
storage, and within the oracle's tolerance."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import geometry as og
import workloads as wl
from helpers import log, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdk = pytest.importorskip("paper_2104_13248_amd")
from paper_2104_13248_amd import _lib  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _call(name, shape, voxel, proj, scale, mats):
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    npv, nh, nw = proj.shape
    vg = _lib.volume_struct(shape, voxel)
    sg = _lib.stack_struct(npv, nh, nw, _lib.FDK_F16 if proj.dtype == torch.float16 else _lib.FDK_F32)
    m = np.ascontiguousarray(mats, dtype=np.float64)
    code = getattr(_lib.lib, name)(ctypes.byref(vg), vol.data_ptr(), ctypes.byref(sg),
                                   proj.data_ptr(), None if scale is None else scale.data_ptr(),
                                   _lib.ptr(m), torch.cuda.current_stream().cuda_stream)
    assert code == 0, (name, code, _lib.lib.fdk_last_error())
    torch.cuda.synchronize()
    return vol.cpu().numpy()


# two calls in a row, the second smaller (fewer views, smaller volume and detector)
CASES = [((64, 64, 64), 100, 128, 128, 0.0), ((20, 24, 28), 9, 40, 48, 0.3)]


@pytest.mark.parametrize("f16", [False, True])
def test_noalloc_equals_backproject(f16):
    for q, (shape, npv, nh, nw, theta0) in enumerate(CASES):
        scan = dict(wl.CONFIGS["c1"]["scan"], theta0=theta0)
        mats = og.scan_matrices(scan, npv, nh, nw)
        proj = wl.gaussian(900 + q, (npv, nh, nw))
        p = torch.from_numpy(proj).cuda()
        scale = None
        if f16:
            p, scale = fdk.quantize_f16(p)
        log("noalloc case", q, shape, (npv, nh, nw), "f16" if f16 else "f32")
        ref = _call("fdk_backproject", shape, (1.0, 1.0, 1.0), p, scale, mats)
        got = _call("fdk_backproject_noalloc", shape, (1.0, 1.0, 1.0), p, scale, mats)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), q
        if f16:
            host = oracle.backproject(p.cpu().numpy(), mats, shape, (1.0, 1.0, 1.0),
                                      scale=scale.cpu().numpy())
        else:
            host = oracle.backproject(proj, mats, shape, (1.0, 1.0, 1.0))
        e = rel(got, host)
        log("rel-L2 vs oracle", e)
        assert e <= 1e-5
