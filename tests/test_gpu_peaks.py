"""The ceiling microbenchmarks (include/fdk_peaks.h) run, report the work the
header states, and stay within the hardware's nominal limits (MI355X)."""
import pytest

from helpers import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdk = pytest.importorskip("paper_2104_13248_amd")
from paper_2104_13248_amd import peaks as pk  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def _rate(fn):
    s = torch.cuda.current_stream()
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    work = fn()
    b.record(s)
    torch.cuda.synchronize()
    return work / (a.elapsed_time(b) * 1e-3)


def test_peaks_run_within_nominal_limits():
    dev = torch.device("cuda:0")
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    buf = torch.ones((1 << 30) // 4, dtype=torch.float32, device=dev)        # 1 GiB
    hbm = _rate(lambda: pk.hbm_read(buf, 1 << 30, 4096, sink)) / 1e9
    log("hbm read GB/s", hbm)
    assert 500.0 < hbm < 8000.0 * 1.25
    n = pk.lds_read("b32", 7, 3, dev, sink)
    assert n == 7 * 256 * 3 * 16 * 4
    lds_nominal = 256 * 128 * 2.4e9 / 1e9
    for pat in pk.LDS_PATTERNS:
        g = _rate(lambda: pk.lds_read(pat, 2560, 200, dev, sink)) / 1e9
        log("lds", pat, "GB/s", g)
        assert 1000.0 < g < 2.5 * lds_nominal
    ops = pk.valu_fma(3, 2, dev, sink)
    assert ops == 3 * 256 * 8 * 16 * 2
    t = _rate(lambda: pk.valu_fma(2048, 400, dev, sink)) / 1e12
    log("valu TOP/s", t)
    assert 5.0 < t < 256 * 128 * 2.4e9 / 1e12 * 1.1
    torch.cuda.synchronize()
    assert int(sink.item()) == 0                  # the never-taken write
