"""Builds libhdmd.so (gfx950) in-tree from csrc/ with hipcc.

Every HIP translation unit is compiled with -ffp-contract=off (the list test
must round exactly as written), with packed FP32 arithmetic disabled, and with
matrix-core results in ordinary vector registers (the list build reads their
sign bits with vector instructions).
The dimension-templated kernels are compiled once per d = 2..10 in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhdmd.so")
DIMS = range(2, 11)

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", INC, "-I", CSRC, "-Wno-unused-result"]


def _hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return h


def _compile(src: str, obj: str, extra: list[str]) -> str:
    cmd = [_hipcc(), *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = [(os.path.join(CSRC, "common.hip"), os.path.join(BUILD, "common.o"), []),
             (os.path.join(CSRC, "runtime.hip"), os.path.join(BUILD, "runtime.o"), []),
             (os.path.join(CSRC, "kern_all.hip"), os.path.join(BUILD, "kern_all.o"), [])]
    for d in DIMS:
        units.append((os.path.join(CSRC, "kern_dim.hip"), os.path.join(BUILD, "kern_d%d.o" % d),
                      ["-DHDMD_DIM=%d" % d]))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(*u), units))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
