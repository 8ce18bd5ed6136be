"""Build libkernelet_fake.so: the engine's runtime compiled with g++ against
the host-thread HIP test double in this directory (CPU tests of the
dispatcher).

The environment variable KL_FAKE_SANITIZE selects a sanitized build for the
same tests: "address" (AddressSanitizer and UndefinedBehaviorSanitizer) or
"thread" (ThreadSanitizer).  The sanitizer's runtime must then be preloaded
into the Python process, e.g.

    KL_FAKE_SANITIZE=address ASAN_OPTIONS=detect_leaks=0 \\
    LD_PRELOAD=$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so) \\
    python -m pytest tests/test_runtime_fake.py

    KL_FAKE_SANITIZE=thread LD_PRELOAD=$(gcc -print-file-name=libtsan.so) \\
    python -m pytest tests/test_runtime_fake.py
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1303_5164_amd", "csrc")

SANITIZE = {
    None: ([], "libkernelet_fake.so"),
    "address": (["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                 "-fno-sanitize-recover=undefined"], "libkernelet_fake_asan.so"),
    "thread": (["-fsanitize=thread"], "libkernelet_fake_tsan.so"),
}


def output(sanitize=None):
    return os.path.join(HERE, SANITIZE[sanitize][1])


def build(force=False, sanitize=None):
    if sanitize is None:
        sanitize = os.environ.get("KL_FAKE_SANITIZE") or None
    flags, _ = SANITIZE[sanitize]
    out = output(sanitize)
    srcs = [os.path.join(CSRC, "runtime.cpp"), os.path.join(CSRC, "model.cpp"),
            os.path.join(HERE, "fake_hip.cpp")]
    if not force and os.path.exists(out) and all(
            os.path.getmtime(out) > os.path.getmtime(s) for s in srcs):
        return out
    tmp = out + ".tmp"
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-Wall",
                           *flags, "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           *srcs, "-o", tmp, "-lpthread"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(force=True))
