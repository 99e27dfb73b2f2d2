"""Host-side CRT constants (crt_setup runs on the host, no GPU needed)."""
import pytest

from paper_1609_00999_amd import workloads as wl

R = 1 << 32


@pytest.fixture(scope="module")
def C():
    from paper_1609_00999_amd import crt
    try:
        crt.lib()
    except Exception as e:                       # library not built here
        pytest.skip("libmont not loadable: %s" % e)
    return crt


@pytest.mark.parametrize("primes", [wl.PRIMES_NTT[:3], wl.PRIMES_NTT[3:6], wl.PRIMES_NTT[5:8][::-1]])
def test_garner_constants(C, primes):
    prm = C.setup(primes)
    P1, P2, P3 = primes
    assert prm.primes == tuple(primes)
    # Montgomery forms: c_bar = c R mod P
    assert prm.inv12 == pow(P1, -1, P2) * R % P2
    assert prm.p1_mod3 == P1 % P3 * R % P3
    assert prm.inv123 == pow(P1 * P2, -1, P3) * R % P3
    for j, P in enumerate(primes):
        assert prm.m[j].P == P and (P * prm.m[j].Pprime) % R == R - 1


def test_setup_errors(C):
    from paper_1609_00999_amd import mont
    for bad in ([wl.PRIMES_NTT[0]] * 3, [998244353, wl.PRIMES_NTT[1], wl.PRIMES_NTT[2]],
                [wl.PRIMES_NTT[0], wl.PRIMES_NTT[1], 1 << 31], [wl.PRIMES_NTT[0], wl.PRIMES_NTT[1], 2147483646]):
        with pytest.raises(mont.MontError):
            C.setup(bad)
    assert C.scratch_bytes(0, 0) > 0
    # the scratch holds three residue copies of both operands and of the product, plus the transform's
    a, b = 5000, 7000
    assert C.scratch_bytes(a, b) >= 3 * 4 * (a + b + 2 + a + b + 1)
