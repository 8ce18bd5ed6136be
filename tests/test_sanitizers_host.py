"""The dispatcher tests of test_runtime_fake.py again, with the runtime built
under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer (host code only: the runtime against the host-thread HIP
test double).  Each run is a child pytest process with the sanitizer's
runtime preloaded; any sanitizer report fails the run."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "fakehip"))

import build as fake_build  # noqa: E402


def _gcc_lib(name):
    return subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_runtime_under_sanitizer(kind, tmp_path):
    fake_build.build(force=False, sanitize=kind)
    env = dict(os.environ)
    env["KL_FAKE_SANITIZE"] = kind
    log = str(tmp_path / "san")
    if kind == "address":
        env["LD_PRELOAD"] = _gcc_lib("libasan.so") + ":" + _gcc_lib("libubsan.so")
        env["ASAN_OPTIONS"] = f"detect_leaks=0:halt_on_error=1:log_path={log}"
        env["UBSAN_OPTIONS"] = f"halt_on_error=1:print_stacktrace=1:log_path={log}"
    else:
        env["LD_PRELOAD"] = _gcc_lib("libtsan.so")
        env["TSAN_OPTIONS"] = f"halt_on_error=1:report_signal_unsafe=0:log_path={log}"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_runtime_fake.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = [p for p in os.listdir(tmp_path) if p.startswith("san")]
    text = "".join(open(os.path.join(tmp_path, p)).read() for p in reports)
    assert r.returncode == 0 and not reports, (r.stdout[-2000:], r.stderr[-2000:], text[:4000])
    assert "passed" in r.stdout
