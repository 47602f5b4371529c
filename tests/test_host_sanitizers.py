"""The host code (preprocessing, partitioner, features, plan files) built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on random matrices:
no memory error, leak or undefined behaviour may be reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_06666_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_host")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(ROOT, "tests", "native", "sanitize_host.cpp"),
           os.path.join(CSRC, "ehyb_host.cpp"), os.path.join(CSRC, "partition.cpp"),
           os.path.join(CSRC, "features.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe, "6", str(tmp_path / "plan.bin")], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "Sanitizer" not in out, out[-4000:]
    assert "fails=0" in out
