"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code,
run on the CPU: the oracle (every entry point, serial and threaded) and the
library's host side of the tile path (canonicalisation, fusion, planning with
and without relabeling, lowering, and the host model of the register kernel).
Built with gcc / g++ from the sources (no GPU code involved); any invalid
access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout)
    if r.returncode != 0:
        if "cannot find" in r.stderr and "asan" in r.stderr:
            pytest.skip("sanitizer runtime not installed")
        raise AssertionError("build failed:\n" + r.stderr[-4000:])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=ENV)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert r.stdout.startswith("ok"), r.stdout
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _build_and_run(["gcc", "-std=c99", "-fopenmp", "-ffp-contract=off"] + SAN +
                   [os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
                    os.path.join(ROOT, "oracle", "qsv_oracle.c"), "-lm", "-o", exe], exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_host_planner_and_lowering_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1612_08091_amd", "csrc")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.exists(os.path.join(rocm, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("HIP headers not found")
    exe = str(tmp_path / "planner_check")
    out = _build_and_run(["g++", "-std=c++17"] + SAN +
                         ["-I" + csrc, "-I" + os.path.join(ROOT, "include"),
                          "-I" + os.path.join(rocm, "include"), "-D__HIP_PLATFORM_AMD__",
                          os.path.join(ROOT, "tests", "sanitize", "planner_check.cpp"),
                          os.path.join(csrc, "planner.cpp"), os.path.join(csrc, "tileprog.cpp"),
                          "-o", exe], exe)
    assert "programs" in out
