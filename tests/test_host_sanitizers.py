"""Sanitizer runs on the CPU (no GPU needed):

* the CPU oracle built with -fsanitize=address,undefined, under its own pin
  tests (the pins exercise every oracle function, including the 64-bit and
  CRT routines);
* the host path of libmont's vector batch (reserve, update, launch, destroy)
  built with the same sanitizers against a host stand-in for the HIP runtime
  (tests/host_sanitize), which checks every staging write, upload length and
  buffer lifetime, and runs the kernel on the host over the uploaded
  descriptors.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
CLANGXX = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")


def _gcc_runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = oracle.build(force=True, out=str(tmp_path / "liboracle_san.so"), extra_flags=SAN)
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=asan + ":" + ubsan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.loaded_path())"], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stdout + probe.stderr
    pins = ["tests/test_oracle_pins.py", "tests/test_oracle64_pins.py", "tests/test_paper_algorithms.py",
            "tests/test_crt_cpu.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *pins], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_vector_batch_host_path_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(CLANGXX) and not shutil.which("clang++"):
        pytest.skip("clang++ not found")
    cxx = CLANGXX if os.path.exists(CLANGXX) else shutil.which("clang++")
    exe = str(tmp_path / "batch_harness")
    src = os.path.join(HERE, "host_sanitize", "batch_harness.cpp")
    cmd = [cxx, "-std=c++17", *SAN, "-I", os.path.join(HERE, "host_sanitize"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1609_00999_amd", "csrc"), src, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " 0 failures" in r.stdout
