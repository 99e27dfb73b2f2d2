"""The paper's Algorithms 1 and 3 written out step by step in Python integers,
checked against plain modular arithmetic (CPU).  They pin the readings of
section 3.1 that the device kernels rely on, and the new oracle routines."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

R = 1 << 32
FOURIER = sorted(set(wl.PRIMES_BW) | set(wl.PRIMES_NTT))


def i32(x):
    """Two's-complement 32-bit reading of an integer."""
    x &= 0xFFFFFFFF
    return x - (1 << 32) if x & 0x80000000 else x


def fourier_parts(a, b, P):
    """q1, q2, q3 of Algorithm 3 with K = c 2^k = P - 1, and the dropped r3."""
    K = P - 1
    T = a * b
    q1, r1 = T // R, T % R
    q2, r2 = (K * r1) // R, (K * r1) % R
    q3, r3 = (K * r2) // R, (K * r2) % R
    return q1, q2, q3, r3


def alg3_as_printed(a, b, P):
    """Algorithm 3 with its 32-bit signed sign-mask corrections."""
    q1, q2, q3, _ = fourier_parts(a, b, P)
    t = i32(q1 - q2 + q3)
    t = i32(t + ((t >> 31) & P))          # Python >> on a negative int is arithmetic
    t = i32(t - P)
    t = i32(t + ((t >> 31) & P))
    return t


def alg3_borrow(a, b, P):
    """Algorithm 3 with the sign taken from an explicit borrow (the device form)."""
    q1, q2, q3, _ = fourier_parts(a, b, P)
    s = q1 + q3
    if s < q2:
        return s - q2 + P
    d = s - q2
    return d - P if d >= P else d


def samples(P, n=3000, seed=0):
    rng = np.random.default_rng(seed)
    e = [x % P for x in (0, 1, 2, P - 1, P - 2, (P - 1) // 2, 1 << 16, (1 << 16) - 1)]
    a = np.concatenate([np.repeat(e, len(e)), rng.integers(0, P, n)]).tolist()
    b = np.concatenate([np.tile(e, len(e)), rng.integers(0, P, n)]).tolist()
    return a, b


@pytest.mark.parametrize("P", FOURIER)
def test_alg3_lemma_and_range(P):
    """r3 = 0 when R = 2^32 <= 2^(2k), and q1 - q2 + q3 lies in (-(P-1), 2(P-1))."""
    assert oracle.setup(P).k >= 16
    a, b = samples(P)
    for x, y in zip(a, b):
        q1, q2, q3, r3 = fourier_parts(x, y, P)
        assert r3 == 0
        t = q1 - q2 + q3
        assert -(P - 1) < t < 2 * (P - 1)
        assert (t * R - x * y) % P == 0                # t = a b R^-1 mod P


@pytest.mark.parametrize("P", FOURIER)
def test_alg3_borrow_form_matches_redc(P):
    a, b = samples(P, seed=1)
    ref = oracle.mont_mul(P, np.array(a, dtype=np.uint32), np.array(b, dtype=np.uint32)).tolist()
    assert [alg3_borrow(x, y, P) for x, y in zip(a, b)] == ref


def test_alg3_as_printed_overflows_for_31_bit_primes():
    """The printed corrections are exact while 2(P-1) < 2^31 and fail beyond."""
    for P in (469762049, 998244353):                   # 29- and 30-bit
        a, b = samples(P, seed=2)
        ref = oracle.mont_mul(P, np.array(a, dtype=np.uint32), np.array(b, dtype=np.uint32)).tolist()
        assert [alg3_as_printed(x, y, P) for x, y in zip(a, b)] == ref
    for P in (2013265921, 2113929217):                 # 31-bit: q1 - q2 + q3 can exceed 2^31
        a, b = samples(P, seed=3)
        ref = oracle.mont_mul(P, np.array(a, dtype=np.uint32), np.array(b, dtype=np.uint32)).tolist()
        bad = sum(alg3_as_printed(x, y, P) != r for x, y, r in zip(a, b, ref))
        assert bad > 0


def barrett_as_printed(a, b, P):
    """Algorithm 1; returns the result and the number of correction loops."""
    k = P.bit_length()                                 # ceil(log2 P) for P not a power of two
    Pb = (1 << (2 * k)) // P
    m = (a * b) >> k
    q = (m * Pb) >> k
    t = a * b - q * P
    assert 0 <= t < 4 * P
    loops = 0
    while t >= P:
        t -= P
        loops += 1
    return t, loops


@pytest.mark.parametrize("P", FOURIER + [3, 17, 65537, (1 << 31) - 1, 1000003])
def test_barrett_matches_plain_product(P):
    a, b = samples(P, seed=4)
    got = [barrett_as_printed(x, y, P) for x, y in zip(a, b)]
    assert [g[0] for g in got] == [x * y % P for x, y in zip(a, b)]
    assert max(g[1] for g in got) <= 3


def test_oracle_plain_routines():
    rng = np.random.default_rng(5)
    for P in (17, 998244353, 2113929217):
        a = rng.integers(0, P, 2000, dtype=np.uint32)
        b = rng.integers(0, P, 2000, dtype=np.uint32)
        assert oracle.modmul(P, a, b).tolist() == [int(x) * int(y) % P for x, y in zip(a, b)]
        e = rng.integers(0, 1 << 32, 2000, dtype=np.uint64).astype(np.uint32)
        assert oracle.modpow(P, a, e).tolist() == [pow(int(x), int(y), P) for x, y in zip(a, e)]
    assert oracle.modpow(7, np.array([0], np.uint32), np.array([0], np.uint32))[0] == 1
