"""The host ingest helpers (vca_ingest.h: raw .yuv reading in row bands on a
worker pool, pitched row copies) built with AddressSanitizer + UBSan and
with ThreadSanitizer, then run on the CPU (tests/host/ingest_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "ingest_check.cpp")


@pytest.mark.parametrize("sanitize", ["address,undefined", "thread"])
def test_ingest_helpers_under_sanitizer(tmp_path, sanitize):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "ingest_check"
    build = subprocess.run([gxx, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}",
                            "-fno-omit-frame-pointer", "-pthread", SRC, "-o", str(exe)],
                           capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ingest check ok" in run.stdout
