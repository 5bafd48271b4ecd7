"""Host test of the serving scheduler core (no GPU): builds tests/cpp/test_serve_core.cpp
with g++ (thread sanitizer) against the scheduler header and runs it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_13714_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "cpp", "test_serve_core.cpp")


@pytest.mark.parametrize("san", ["thread", "none"])
def test_serve_core(tmp_path, san):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path / f"serve_core_{san}")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", "-I", CSRC, SRC, "-o", exe]
    if san != "none":
        cmd.insert(1, f"-fsanitize={san}")
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
