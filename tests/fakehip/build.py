"""Build libkernelet_fake.so: the engine's runtime compiled with g++ against
the host-thread HIP test double in this directory (CPU tests of the
dispatcher)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1303_5164_amd", "csrc")
OUT = os.path.join(HERE, "libkernelet_fake.so")


def build(force=False):
    srcs = [os.path.join(CSRC, "runtime.cpp"), os.path.join(CSRC, "model.cpp"),
            os.path.join(HERE, "fake_hip.cpp")]
    if not force and os.path.exists(OUT) and all(
            os.path.getmtime(OUT) > os.path.getmtime(s) for s in srcs):
        return OUT
    tmp = OUT + ".tmp"
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-Wall",
                           "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           *srcs, "-o", tmp, "-lpthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force=True))
