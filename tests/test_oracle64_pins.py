"""Pins of the 64-bit-residue and Chinese-remainder oracle routines (CPU).

Each check is against something the oracle does not compute itself: brute
force over tiny moduli, Python's arbitrary-precision integers and built-in
modular power, closed forms of section 3.1, Fermat's little theorem and
Euler's criterion, and exhaustive search for the CRT.
"""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

R64 = 1 << 64
SMALL_ODD = [3, 5, 15, 17, 21, 63, 97, 255, 257]
BIG = list(wl.PRIMES64) + [(1 << 61) - 1, (1 << 63) - 1 - 2 * 3, 2 ** 62 + 135]   # primes and odd composites


def edges64(P):
    v = [0, 1, 2, 3, P - 1, P - 2, (P - 1) // 2, (P + 1) // 2, R64 % P, (R64 * R64) % P, 1 << 32, (1 << 32) - 1,
         (1 << 32) + 1, 1 << 62]
    return np.array(sorted({x % P for x in v}), dtype=np.uint64)


@pytest.mark.parametrize("P", BIG + SMALL_ODD)
def test_setup_closed_forms(P):
    prm = oracle.setup64(P)
    assert R64 * prm.Rinv - P * prm.Pprime == 1
    assert 0 < prm.Rinv < P and 0 < prm.Pprime < R64
    assert (P * prm.Pprime) % R64 == R64 - 1
    assert (prm.R1 * prm.Rinv) % P == 1 % P
    assert (prm.R2 * prm.Rinv * prm.Rinv) % P == 1 % P
    k = 0
    while (P - 1) % (1 << (k + 1)) == 0:
        k += 1
    assert prm.k == k


def test_fourier_prime_identity_64():
    """For P = c 2^k + 1 with 2k >= 64, P^-1 = 1 - c 2^k mod 2^64, so P' = P - 2."""
    for P in wl.PRIMES64[:3]:
        assert oracle.setup64(P).Pprime == P - 2


@pytest.mark.parametrize("P,r", [(17, 5), (15, 5), (21, 6), (63, 7), (97, 8), (255, 9), (257, 10)])
def test_bruteforce_tiny(P, r):
    """Montgomery product with R = 2^r: z in [0, P) with z R = a b (mod P), by search."""
    R = 1 << r
    xs = np.arange(P, dtype=np.uint64)
    a, b = (m.ravel() for m in np.meshgrid(xs, xs, indexing="ij"))
    got = oracle.mont_mul64(P, a, b, r=r)
    for x, y, g in zip(a.tolist(), b.tolist(), got.tolist()):
        z = [z for z in range(P) if (z * R - x * y) % P == 0]
        assert z == [g]
    # conversions: residue i R mod P, and back
    t = oracle.to_mont64(P, xs, r=r)
    assert t.tolist() == [(i * R) % P for i in range(P)]
    assert oracle.from_mont64(P, t, r=r).tolist() == list(range(P))


@pytest.mark.parametrize("P", BIG)
def test_product_identity_and_roundtrip(P):
    rng = np.random.default_rng(P % 10007)
    a = np.concatenate([edges64(P), wl.uniform64(rng, 0, P, 3000)])
    b = np.concatenate([edges64(P)[::-1], wl.uniform64(rng, 0, P, 3000)])
    ta, tb = oracle.to_mont64(P, a), oracle.to_mont64(P, b)
    # REDC(aR bR) = abR, with the ordinary product from Python integers
    prod = oracle.mont_mul64(P, ta, tb)
    want = [(x * y * R64) % P for x, y in zip(a.tolist(), b.tolist())]
    assert prod.tolist() == want
    assert oracle.from_mont64(P, prod).tolist() == [(x * y) % P for x, y in zip(a.tolist(), b.tolist())]
    # mul-add reduces to mul when c = 0, and adds residues otherwise
    z = np.zeros_like(a)
    assert np.array_equal(oracle.mont_muladd64(P, ta, tb, z), prod)
    c = wl.uniform64(rng, 0, P, a.size)
    assert oracle.mont_muladd64(P, ta, tb, c).tolist() == [(p + q) % P for p, q in zip(want, c.tolist())]
    # conversions are total on uint64
    x = np.concatenate([rng.integers(0, 1 << 64, 2000, dtype=np.uint64),
                        np.array([P, P + 1, R64 - 1, 1 << 63], dtype=np.uint64)])
    assert oracle.from_mont64(P, oracle.to_mont64(P, x)).tolist() == [v % P for v in x.tolist()]


@pytest.mark.parametrize("P", wl.PRIMES64 + ((1 << 61) - 1,))
def test_pow_against_python_and_fermat(P):
    rng = np.random.default_rng(P % 7919)
    base = wl.uniform64(rng, 1, P, 500)
    e = rng.integers(0, 1 << 64, 500, dtype=np.uint64)
    e[:6] = [0, 1, 2, 3, (1 << 64) - 1, 1 << 63]
    tb = oracle.to_mont64(P, base)
    got = oracle.from_mont64(P, oracle.mont_pow64(P, tb, e))
    assert got.tolist() == [pow(x, y, P) for x, y in zip(base.tolist(), e.tolist())]
    f = oracle.mont_pow64(P, tb, np.full(base.size, P - 1, dtype=np.uint64))
    assert np.all(f == oracle.setup64(P).R1)
    h = oracle.from_mont64(P, oracle.mont_pow64(P, tb, np.full(base.size, (P - 1) // 2, dtype=np.uint64)))
    assert set(h.tolist()) <= {1, P - 1}
    zero = oracle.mont_pow64(P, np.zeros(1, np.uint64), np.zeros(1, np.uint64))
    assert zero[0] == oracle.setup64(P).R1          # 0^0 = 1


def test_crt_bruteforce_tiny():
    primes = [5, 7, 11]
    M = 5 * 7 * 11
    res = np.array([[x % p for x in range(M)] for p in primes], dtype=np.uint32)
    out = oracle.crt(primes, res, 1)
    assert out[:, 0].tolist() == list(range(M))


def test_crt_random_big():
    rng = np.random.default_rng(99)
    primes = list(wl.PRIMES_NTT[:3])
    M = primes[0] * primes[1] * primes[2]
    xs = [int(rng.integers(0, 1 << 62)) * (1 << 30) % M for _ in range(500)] + [0, 1, M - 1, M // 2]
    res = np.array([[x % p for x in xs] for p in primes], dtype=np.uint32)
    out = oracle.crt(primes, res, 3)
    got = [int(w[0]) | (int(w[1]) << 32) | (int(w[2]) << 64) for w in out]
    assert got == xs
    with pytest.raises(ValueError):
        oracle.crt(primes, res, 2)                  # M needs 93 bits
