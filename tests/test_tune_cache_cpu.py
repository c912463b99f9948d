"""The launch-shape cache file behind VCA_TUNE_CACHE (the TuneCache of
csrc/vca_host.h), built as a host-only program and run on the CPU
(tests/host/tune_cache_check.cpp): six-field and older four-field lines
load, invalid shapes are dropped, put() writes the six-field form."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "tune_cache_check.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_tune_cache_file(tmp_path):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "tune_cache_check"
    build = subprocess.run([HIPCC if os.path.exists(HIPCC) else "hipcc", "-x", "hip", "--offload-arch=gfx950",
                            "-std=c++17", "-O1", SRC, "-o", str(exe)],
                           capture_output=True, text=True, timeout=600)
    assert build.returncode == 0, build.stderr
    cache = tmp_path / "tune_cache.txt"
    env = {k: v for k, v in os.environ.items() if k != "VCA_TUNE_CACHE"}
    run = subprocess.run([str(exe), str(cache)], capture_output=True, text=True, timeout=120, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "tune cache check ok" in run.stdout
