"""Build libfdk.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python paper_2104_13248_amd/build.py            # incremental
    python paper_2104_13248_amd/build.py --force    # rebuild everything

(run as a script: importing the package loads the library it builds).

Objects go to ``_build/`` at the repository root; the shared library to
``paper_2104_13248_amd/libfdk.so`` (where the Python binding loads it).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shlex
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfdk.so")
ARCH = os.environ.get("FDK_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + INCLUDE, "-I" + CSRC, "--offload-arch=" + ARCH]
# Packed FP32 (v_pk_*_f32) is switched off for all device code; unsafe FP
# atomics give the hardware float atomic instructions.
DEVICE = ["-x", "hip", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = ["api.cpp", "geometry.cpp", "runtime.cpp", "compose.hip", "bp.hip", "fp.hip",
           "filter.hip", "quantize.hip", "phantom.hip", "learn.hip",
           "ablation.hip", "peaks.hip", "noalloc.hip"]
HEADERS = ["internal.h", "footprint.h"]


def _newer(src_paths, dst):
    if not os.path.exists(dst):
        return True
    t = os.path.getmtime(dst)
    return any(os.path.getmtime(p) > t for p in src_paths)


def _compile(src: str, force: bool, build_dir: str = BUILD, extra=()) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(build_dir, src + ".o")
    deps = [path] + [os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE) if h.endswith(".h")] + \
        [os.path.join(CSRC, h) for h in HEADERS]
    if force or _newer(deps, obj):
        cmd = [HIPCC, "-c"] + COMMON + DEVICE + list(extra) + [path, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(map(shlex.quote, cmd)),
                                                            r.stdout, r.stderr))
    return obj


def build(force: bool = False, jobs: int = 0, lib_path: str = LIB, build_dir: str = BUILD,
          extra=()) -> str:
    """Compile every source into ``build_dir`` and link ``lib_path``.  ``extra``
    are additional hipcc flags for every compile and the link (e.g. host-only
    sanitizers, each ``-fsanitize=`` after ``-Xarch_host``)."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, build_dir, extra), SOURCES))
    if force or _newer(objs, lib_path):
        tmp = lib_path + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + list(extra) + ["-o", tmp] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
        os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
