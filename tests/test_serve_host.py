"""Host-only tests of the serving runtime's scheduler (csrc/serve.cpp).

serve.cpp is compiled with the host compiler against a fake device
(tests/serve_fake/fake_device.cpp: streams are worker threads, device memory
is host memory, the kernel launchers are replaced by small functions of their
inputs) and driven by tests/serve_fake/serve_driver.cpp, under
ThreadSanitizer: per-stream order and the carry of partial sub-intervals,
the HBM budget and no head-of-line blocking, cancel, close while busy,
export / import, an allocation failure (the stream continues), a launch
failure after part of a block was enqueued (the block keeps its slot until
that work has run; its stream fails, others do not), and four threads
submitting, waiting, polling and closing at once. No GPU is used.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INC),
                    reason="needs g++ and the HIP headers")
def test_serving_scheduler_on_fake_device_under_tsan(tmp_path):
    exe = tmp_path / "serve_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-Wno-deprecated-declarations",
           "-D__HIP_PLATFORM_AMD__", f"-I{HIP_INC}", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2512_16278_amd/csrc",
           f"{ROOT}/paper_2512_16278_amd/csrc/serve.cpp",
           f"{ROOT}/tests/serve_fake/fake_device.cpp",
           f"{ROOT}/tests/serve_fake/serve_driver.cpp",
           "-o", str(exe), "-lpthread"]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "ALL OK" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
