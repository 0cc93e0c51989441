"""Build ``liblsamg.so`` in-tree for gfx950.

The host setup (``host_setup.cpp``) is compiled with g++; the HIP sources (the
kernels and C-ABI, and the device setup) with hipcc for
``--offload-arch=gfx950``; both are linked into one shared
library next to this file.  Run ``python -m paper_2601_04112_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys
import concurrent.futures as cf

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblsamg.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SRCS = ["host_setup.cpp"]
HIP_SRCS = ["lsamg.hip", "setup_device.hip"]

CXXFLAGS = ["-O3", "-fPIC", "-std=c++17", "-pthread", "-mavx2", "-mfma",
            "-Wall", "-Wno-unused-function"]
HIPFLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n"
                           + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link ``liblsamg.so``; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for s in HOST_SRCS:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append(["g++"] + CXXFLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    for s in HIP_SRCS:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append([HIPCC] + HIPFLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
         + ["-pthread", "-ldl"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
