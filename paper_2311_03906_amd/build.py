"""Builds libsymphase_hip.so in-tree (hipcc, gfx950).

    python -m paper_2311_03906_amd.build
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsymphase_hip.so")

ARCH = os.environ.get("SYMPHASE_ARCH", "gfx950")
HOST_SRCS = ["circuit.cpp", "symbolize.cpp", "api.cpp", "sample_host.cpp"]
HIP_SRCS = ["sample.hip", "batch.hip", "server.hip", "init.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include")]
HOST_FLAGS = ["-pthread"]
# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = [], []
    for s in HOST_SRCS:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["g++"] + COMMON + HOST_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HIP_SRCS:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["hipcc"] + COMMON + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for r, c in zip(ex.map(_run, cmds), cmds):
            if verbose:
                print(" ".join(c))
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-pthread", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
