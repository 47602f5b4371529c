"""Failure paths of the host code, on the CPU.

* Allocation failures: tests/native/alloc_fail_host.cpp replaces operator new
  with one that fails at a chosen allocation and sweeps that choice over every
  host entry point (preprocessing, re-encoding, features, decode, save, load).
  Built with AddressSanitizer (leak detection on) and UBSan: every call must
  return EHYB_OK or EHYB_ENOMEM, never abort (an exception leaving an OpenMP
  region or task would terminate the process), and leak nothing.
* Threads: the OpenMP preprocessing built with ThreadSanitizer (LLVM's OpenMP
  runtime and its Archer annotations of OpenMP synchronisation) reports no
  data race, and a planted race in a small loop is reported (the detector is
  live)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_06666_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
HOST = [os.path.join(CSRC, f) for f in ("ehyb_host.cpp", "partition.cpp", "features.cpp")]
LLVM = os.environ.get("ROCM_PATH", "/opt/rocm") + "/llvm"
CLANG = os.path.join(LLVM, "bin", "clang++")
ARCHER = os.path.join(LLVM, "lib", "libarcher.so")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_allocation_failures_report_enomem_without_leaks(tmp_path):
    exe = str(tmp_path / "alloc_fail_host")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(NATIVE, "alloc_fail_host.cpp"), *HOST, "-o", exe]
    subprocess.run(cmd, check=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe, "40", str(tmp_path / "plan.bin")], capture_output=True, text=True, timeout=900,
                       env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out and "terminate" not in out, out[-4000:]
    assert "bad=0" in out
    # the sweep reached every phase of preprocessing
    assert "preprocess:" in out and "preprocess_partitioned:" in out and "features:" in out


def _tsan_build(src, exe):
    cmd = [CLANG, "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=thread", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *src, "-o", exe, f"-Wl,-rpath,{LLVM}/lib"]
    subprocess.run(cmd, check=True, timeout=600, capture_output=True)


def _tsan_env():
    return dict(os.environ, OMP_NUM_THREADS="4", OMP_TOOL_LIBRARIES=ARCHER,
                TSAN_OPTIONS="halt_on_error=1 ignore_noninstrumented_modules=1")


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(ARCHER)),
                    reason="needs LLVM clang with its OpenMP runtime and Archer")
def test_openmp_preprocessing_under_thread_sanitizer(tmp_path):
    canary = str(tmp_path / "tsan_canary")
    _tsan_build([os.path.join(NATIVE, "tsan_canary.cpp")], canary)
    r = subprocess.run([canary], capture_output=True, text=True, timeout=300, env=_tsan_env())
    assert "WARNING: ThreadSanitizer: data race" in r.stdout + r.stderr, "the planted race was not reported"
    exe = str(tmp_path / "sanitize_host_tsan")
    _tsan_build([os.path.join(NATIVE, "sanitize_host.cpp"), *HOST], exe)
    r = subprocess.run([exe, "4", str(tmp_path / "plan.bin")], capture_output=True, text=True, timeout=900,
                       env=_tsan_env())
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-6000:]
    assert r.returncode == 0 and "fails=0" in out, out[-4000:]
