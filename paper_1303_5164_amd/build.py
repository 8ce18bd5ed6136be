"""Build libkernelet.so (HIP kernels + C++ runtime) for gfx950 with hipcc.

Usage: python -m paper_1303_5164_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libkernelet.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["workloads.hip", "mlp.hip", "model.cpp", "runtime.cpp"]

# Packed FP32 instructions are disabled: the compiler would otherwise form
# them from ordinary float code.
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = ["hipcc", *[f for f in HIP_FLAGS if f != "--offload-arch=gfx950"],
                   "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        out = _run(cmd)
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
          "-lpthread"])
    os.replace(tmp, LIB)
    build_plain()
    return LIB


PLAIN_SOURCE = os.path.join(CSRC, "plain_kernels.hip")
PLAIN_IMAGE = os.path.join(HERE, "plain_kernels_sliced.hsaco")
PLAIN_KERNELS = ["kl_plain_matadd", "kl_plain_visit3d"]


def build_plain() -> str:
    """The kernels written without slicing, made sliceable by rewriting
    their device IR, in one code object."""
    from . import irslice
    tmp = PLAIN_IMAGE + ".tmp"
    irslice.slice_source(PLAIN_SOURCE, PLAIN_KERNELS, tmp)
    os.replace(tmp, PLAIN_IMAGE)
    return PLAIN_IMAGE


if __name__ == "__main__":
    print(build(verbose=True))
