"""Build libqsv.so for gfx950 with hipcc, in-tree.

Every .hip file is compiled for the device (gfx950) and the host; every
.cpp file is host-only C++.  Objects go to ../_build/, the library next to
this file.  Always compiles (no staleness shortcut) when called with
force=True, which is what the package's build() entry does.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqsv.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# -simplifycfg-sink-common=false: without it LLVM merges the per-register-bit
# cases of the tile kernel into one dynamically indexed access, which moves
# the register-resident amplitudes to scratch memory.
# -amdgpu-atomic-optimizer-strategy=None: every atomic here is one lane's
# claim of a work item; the optimizer turns it into a wave-wide scan whose
# result is needed at once, which puts a full vmcnt(0) wait (on the tile loads
# issued just before) right after the claim.
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-mllvm", "--simplifycfg-sink-common=false",
          "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON
    if src.endswith(".hip"):
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(force: bool = True, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    if not force and os.path.exists(OUT):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(ROOT, "include", "qsv.h")])
        if os.path.getmtime(OUT) >= newest:
            return OUT
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
