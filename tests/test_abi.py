"""The C ABI without a GPU: every declared symbol is exported, and host-side
validation rejects bad arguments before anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def declared_symbols():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if fn.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, fn)).read()
            names += re.findall(r"MONT_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)
    return names


@pytest.fixture(scope="module")
def L():
    from paper_1609_00999_amd import mont
    return mont.lib()


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("mont_setup", "mont_to", "mont_from", "mont_mul", "mont_muladd", "mont_pow", "mont_strerror"):
        assert must in names


@pytest.mark.parametrize("name", declared_symbols())
def test_symbol_exported(L, name):
    assert hasattr(L, name), name


def test_no_stray_exports():
    import subprocess
    from paper_1609_00999_amd import mont
    out = subprocess.run(["nm", "-D", "--defined-only", mont.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported <= set(declared_symbols()), exported - set(declared_symbols())


def test_setup_host_only(L):
    from paper_1609_00999_amd import mont
    import oracle
    for P in (3, 15, 17, 469762049, 998244353, 2013265921, 2113929217, 2147483647):
        prm, ref = mont.setup(P), oracle.setup(P)
        assert (prm.Pprime, prm.R1, prm.R2, prm.k) == (ref.Pprime, ref.R1, ref.R2, ref.k)
    for bad in (0, 1, 2, 4, 100, 1 << 31, (1 << 32) - 1):
        with pytest.raises(mont.MontError) as ei:
            mont.setup(bad)
        assert ei.value.status == -1
    assert L.mont_setup(17, None) == -1


def test_validation_without_gpu(L):
    from paper_1609_00999_amd import mont
    prm = mont.setup(2013265921)
    p = ctypes.byref(prm)
    # n == 0 is a no-op even with NULL pointers
    assert L.mont_mul(p, None, None, None, 0, None) == 0
    assert L.mont_to(p, None, None, 0, None) == 0
    # NULL device pointers with n > 0
    assert L.mont_mul(p, None, None, None, 5, None) == -1
    assert L.mont_muladd(p, 16, 16, None, 16, 5, None) == -1
    assert L.mont_pow(p, 16, None, 16, 5, None) == -1
    assert L.mont_from(p, None, 16, 5, None) == -1
    # a parameter block that mont_setup did not produce
    bad = mont.MontParams(P=2013265921, Pprime=1, R1=0, R2=0, k=0)
    assert L.mont_mul(ctypes.byref(bad), 16, 16, 16, 5, None) == -1
    even = mont.MontParams(P=10, Pprime=0, R1=0, R2=0, k=0)
    assert L.mont_to(ctypes.byref(even), 16, 16, 5, None) == -1
    assert L.mont_mul(None, 16, 16, 16, 5, None) == -1


def test_strerror(L):
    from paper_1609_00999_amd import mont
    for s in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(mont.strerror(s), str) and mont.strerror(s)


def test_elem_tune(L):
    from paper_1609_00999_amd import mont
    old = mont.elem_tune_get("mul")
    try:
        mont.elem_tune_set("mul", 512, 2, False)
        assert mont.elem_tune_get("mul") == (512, 2, False)
        with pytest.raises(mont.MontError):
            mont.elem_tune_set("mul", 96, 2, False)
        assert L.mont_elem_tune_set(9, 256, 1, 1) == -1
    finally:
        mont.elem_tune_set("mul", *old)


def test_ntt_host_validation(L):
    import ctypes as C
    from paper_1609_00999_amd import ntt  # noqa: F401  (registers argument types)
    h = C.c_void_p()
    arr = (C.c_uint32 * 1)(2013265921)
    assert L.ntt_ctx_create(arr, 0, 23, C.byref(h)) == -1
    assert L.ntt_ctx_create(arr, 1, 0, C.byref(h)) == -1
    assert L.ntt_ctx_create(arr, 1, 28, C.byref(h)) == -1
    # transforms are capped at 2^23: a longer table is refused before any HIP call
    for bad_log in (24, 25, 27):
        assert L.ntt_ctx_create(arr, 1, bad_log, C.byref(h)) == -1
    assert L.ntt_ctx_create(None, 1, 23, C.byref(h)) == -1
    assert L.ntt_ctx_create(arr, 1, 23, None) == -1
    assert L.ntt_ctx_destroy(None) == -1
    assert L.ntt_forward(None, 0, 16, 4, None) == -1
    assert L.ntt_polymul(None, 0, 16, 1, 16, 1, 16, None, 0, None) == -1
    assert L.ntt_plan_create(None, None, 0, 0, C.byref(h)) == -1
    assert L.ntt_plan_execute(None, None, None, None, 0, 0, 0, None) == -1
    assert L.ntt_plan_destroy(None) == -1
    # scratch sizing is pure host arithmetic
    assert L.ntt_polymul_scratch_bytes(0, 0) == 0
    assert L.ntt_polymul_scratch_bytes(4095, 4096) == 0          # N = 2^13: one workgroup
    assert L.ntt_polymul_scratch_bytes(4096, 4096) == 8 << 14    # N = 2^14: two arrays of N words
    assert L.ntt_polymul_scratch_bytes((1 << 20) - 1, (1 << 20) - 1) == 8 << 21


def test_validation_of_the_next_rows_without_gpu(L):
    """64-bit residues, CRT products, the range check, Algorithms 3 and 1 and
    plan queries reject bad arguments on the host (nothing is enqueued)."""
    from paper_1609_00999_amd import crt, mont, mont64
    EINVAL = mont.EINVAL
    c_vp = ctypes.c_void_p
    dummy = c_vp(0x10000)                       # never dereferenced: validation fails first
    # 64-bit setup and parameter checks
    q = mont64.setup(9223372036854775783)
    assert (q.P * q.Pprime) % (1 << 64) == (1 << 64) - 1
    for bad in (0, 2, 1 << 63, (1 << 64) - 1):
        with pytest.raises(mont.MontError):
            mont64.setup(bad)
    bad = mont64.Mont64Params()
    bad.P, bad.Pprime = 17, 3
    L64 = mont64.lib()
    assert L64.mont64_mul(ctypes.byref(bad), dummy, dummy, dummy, 8, None) == EINVAL
    assert L64.mont64_mul(ctypes.byref(q), None, dummy, dummy, 8, None) == EINVAL
    assert L64.mont64_pow(ctypes.byref(q), dummy, None, dummy, 8, None) == EINVAL
    assert L64.mont64_mul(ctypes.byref(q), None, None, None, 0, None) == mont.OK     # n = 0
    # CRT
    Lc = crt.lib()
    prm = crt.setup([2013265921, 1811939329, 2113929217])
    assert Lc.crt_reduce(None, dummy, 8, dummy, dummy, dummy, None) == EINVAL
    assert Lc.crt_reduce(ctypes.byref(prm), dummy, 8, None, dummy, dummy, None) == EINVAL
    assert Lc.crt_combine(ctypes.byref(prm), dummy, dummy, None, 8, dummy, None) == EINVAL
    assert Lc.crt_combine(ctypes.byref(prm), None, None, None, 0, None, None) == mont.OK
    broken = crt.setup([2013265921, 1811939329, 2113929217])
    broken.m[1].Pprime ^= 2                     # no longer -P^-1
    assert Lc.crt_reduce(ctypes.byref(broken), dummy, 8, dummy, dummy, dummy, None) == EINVAL
    # range check
    L.mont_check_range.argtypes = [ctypes.c_uint32, c_vp, ctypes.c_size_t, c_vp, c_vp]
    assert L.mont_check_range(0, dummy, 8, dummy, None) == EINVAL
    assert L.mont_check_range(17, dummy, 8, None, None) == EINVAL
    assert L.mont_check_range(17, dummy, 8, c_vp(0x10002), None) == EINVAL     # misaligned status
    assert L.mont_check_range(17, None, 0, dummy, None) == mont.OK
    # Algorithms 3 and 1
    p17 = mont.setup(17)
    assert L.mont_mul_fourier(ctypes.byref(p17), dummy, dummy, dummy, 8, None) == EINVAL   # v2(16) < 16
    assert L.modmul_barrett(4, dummy, dummy, dummy, 8, None) == EINVAL
    assert L.modpow_barrett(1 << 31, dummy, dummy, dummy, 8, None) == EINVAL
    # plan queries
    L.ntt_plan_work.argtypes = [c_vp, c_vp, c_vp]
    assert L.ntt_plan_work(None, None, None) == EINVAL
    L.ntt_plan_shape.argtypes = [c_vp, c_vp, c_vp, c_vp]
    assert L.ntt_plan_shape(None, None, None, None) == EINVAL
    L.ntt_plan_task_count.restype = ctypes.c_uint32
    assert L.ntt_plan_task_count(0xFFFFFFFF, 0xFFFFFFFF) == 0                 # too long
