"""libmont from plain C: tests/c_abi_demo.c is compiled with gcc against the
headers in include/ and linked with libmont.so, the HIP runtime and the CPU
oracle; the host checks run anywhere, the device checks on a GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1609_00999_amd")
ORACLE = os.path.join(ROOT, "oracle")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def demo(tmp_path_factory):
    if not os.path.exists(os.path.join(PKG, "libmont.so")):
        pytest.skip("libmont.so is not built")
    import oracle
    oracle.build()
    exe = str(tmp_path_factory.mktemp("cabi") / "c_abi_demo")
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_abi_demo.c"), "-o", exe,
           "-L", PKG, "-lmont", "-L", ORACLE, "-loracle", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + PKG, "-Wl,-rpath," + ORACLE, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_abi_host(demo):
    r = subprocess.run([demo, "host"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout


@pytest.mark.gpu
def test_c_abi_device(demo):
    r = subprocess.run([demo, "device"], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
