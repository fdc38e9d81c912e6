"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two programs are built with both sanitizers (host code only; no GPU is
used) and must finish with no report:

- tests/sanitize/host_check.cpp links the library's host sources
  (kp_api.cpp: argument validation and workspace planning of the C ABI;
  grouping.cpp: the grouping of the initial centroids) with stand-in
  kernel launchers, and checks the grouping's invariants on random and
  degenerate inputs;
- tests/sanitize/oracle_check.c links the FP64 oracle (test
  infrastructure) and runs every entry point single- and multi-threaded.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1905_09345_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _build(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert r.returncode == 0, "build failed:\n" + r.stdout


def _run_clean(exe):
    r = subprocess.run([exe], env=ENV, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out and "runtime error" not in out, out
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    _build([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
            # sanitizers on the host side of the compile and link only
            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", exe,
            os.path.join(SAN, "host_check.cpp"), os.path.join(SAN, "launch_stubs.cpp"),
            os.path.join(CSRC, "kp_api.cpp"), os.path.join(CSRC, "grouping.cpp")])
    assert "host checks passed" in _run_clean(exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _build(["gcc", "-std=c99", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
            "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off", "-o", exe,
            os.path.join(SAN, "oracle_check.c"), os.path.join(ROOT, "oracle", "lloyd64.c"), "-lm"])
    assert "oracle checks passed" in _run_clean(exe)
