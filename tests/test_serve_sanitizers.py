"""The serving loop's host logic under AddressSanitizer + UBSan and under
ThreadSanitizer (host code only; the simulated executor needs no GPU):
concurrent submitters, a poller, close and destroy with work in flight."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1612_06592_amd", "csrc")


def _build(tmp_path, sanitize):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip"))
    exe = str(tmp_path / f"serve_stress_{sanitize.replace(',', '_')}")
    flags = []
    for s in sanitize.split(","):
        flags += ["-Xarch_host", f"-fsanitize={s}"]
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           *flags, "-Xarch_host", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "tests", "native", "serve_stress.cpp"), *srcs,
           "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr[-3000:])
    return exe


@pytest.mark.parametrize("sanitize", ["address,undefined", "thread"])
def test_serving_loop_under_sanitizer(tmp_path, sanitize):
    exe = _build(tmp_path, sanitize)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "serve_stress: ok" in r.stdout
