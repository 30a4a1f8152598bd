"""bench.py's contract helpers, on the CPU: one GPU only, and the measured HBM
traffic it reports next to the roofline (looked up per workload, and only
while the back-projector's sources are the ones the counters were taken on)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as wl  # noqa: E402


def _fields(path):
    return dict(re.findall(r"^(\w+)\s*=\s*(\S+)\s*$", open(path).read(), flags=re.M))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("path", bench.TRAFFIC_PROFILES)
def test_traffic_summaries_are_of_the_current_kernel_sources(path):
    f = _fields(path)
    assert f["kernel_source_sha256"] == bench.kernel_source_hash()
    for st in ("f16", "f32"):
        v = bench.measured_traffic(f["workload"], st)
        assert v is not None and v == float(f["traffic_bytes_per_launch_" + st]) and v > 0


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_benchmark_workloads_have_traffic_summaries(name):
    """The workload names bench.py builds for the two benchmark configurations
    are the ones the summaries record."""
    cfg = wl.CONFIGS[name]
    nz, ny, nx = cfg["shape"]
    workload = "fdk_backprojection_%dx%dx%d_%dviews_%dx%d" % (nx, ny, nz, cfg["np"], cfg["nh"],
                                                            cfg["nw"])
    assert workload in {_fields(p)["workload"] for p in bench.TRAFFIC_PROFILES}


def test_traffic_lookup_rejects_other_workloads_and_sources(tmp_path, monkeypatch):
    src = bench.TRAFFIC_PROFILES[0]
    f = _fields(src)
    assert bench.measured_traffic("fdk_backprojection_1x1x1_1views_1x1", "f16") is None
    assert bench.measured_traffic(f["workload"], "f64") is None
    stale = tmp_path / "stale.md"
    stale.write_text(open(src).read().replace(f["kernel_source_sha256"], "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", (str(stale),))
    assert bench.measured_traffic(f["workload"], "f16") is None
