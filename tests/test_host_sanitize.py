"""The library's host preprocessing (flatten, pruned-view pass, Algorithm 1
traversal) under AddressSanitizer and UndefinedBehaviorSanitizer: a host-only
build of flatten.cpp with the driver tests/host_sanitize/driver.cpp, run on
random valid trees of all primitive and operator kinds (the three view
constructions must agree) and on malformed ones (refused, never a crash).
Sanitizers instrument the host code only; no device code is built."""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

import pytest

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent


@pytest.mark.slow
def test_host_code_under_address_and_undefined_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = tmp_path / "driver"
    cmd = [hipcc, "--cuda-host-only", "-x", "hip", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           str(HERE / "host_sanitize" / "driver.cpp"), str(ROOT / "paper_2304_09673_amd" / "csrc" / "flatten.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe), "300"], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "failures 0" in r.stdout
