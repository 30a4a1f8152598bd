"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer.

* the oracle (oracle/oracle.c), built by gcc with -fsanitize=address,undefined,
  runs the oracle's pin suite (tests/test_oracle.py);
* the library's host code (argument validation, FP64 geometry checks, launch
  plans, scratch handling), built by hipcc with the sanitizers on the host
  side only (each -fsanitize= after -Xarch_host; device code unchanged), runs
  the C-ABI suite (tests/test_abi.py), which exercises every host-side
  rejection path without a GPU.

Each suite runs in a child process with the sanitizer runtime preloaded and
halts on the first report.  CPU only."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:verify_asan_link_order=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run_suite(test_file, env_extra, timeout=900):
    env = dict(os.environ, **ENV_SAN, **env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", test_file)],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    gcc_asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                              text=True).stdout.strip()
    if not os.path.isabs(gcc_asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", so, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    out = _run_suite("test_oracle.py", {"ORACLE_LIBRARY": so, "LD_PRELOAD": gcc_asan})
    assert " passed" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_fdk_build_san", os.path.join(ROOT, "paper_2104_13248_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    lib = str(tmp_path / "libfdk_san.so")
    b.build(force=True, lib_path=lib, build_dir=str(tmp_path / "obj"),
            extra=["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
                   "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=undefined"])
    out = _run_suite("test_abi.py", {"FDK_LIBRARY": lib, "LD_PRELOAD": rt[-1]})
    assert " passed" in out
