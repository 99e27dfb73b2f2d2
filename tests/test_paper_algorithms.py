"""Facts of section 3.1 behind Algorithms 1 and 3, stated from the
mathematics in Python integers and checked against plain modular arithmetic
(CPU): the quantities the algorithms form, the ranges they stay in and the
congruences they satisfy.  They pin the readings the device kernels rely on
(the borrow form of Algorithm 3, the two-subtraction form of Algorithm 1) and
the oracle's plain routines."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

R = 1 << 32
FOURIER = sorted(set(wl.PRIMES_BW) | set(wl.PRIMES_NTT))


def fourier_parts(a, b, P):
    """q1, q2, q3 of Algorithm 3 with K = c 2^k = P - 1, and the dropped r3."""
    K = P - 1
    T = a * b
    q1, r1 = T // R, T % R
    q2, r2 = (K * r1) // R, (K * r1) % R
    q3, r3 = (K * r2) // R, (K * r2) % R
    return q1, q2, q3, r3


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


def test_alg3_sum_fits_a_signed_word_only_below_31_bits():
    """Algorithm 3 decides its corrections from the sign of q1 - q2 + q3 (and
    of that sum minus P) held in one signed 32-bit word.  The sum's range
    (-(P-1), 2(P-1)) fits a signed word only when 2(P-1) <= 2^31 - 1: for the
    29- and 30-bit primes every sum and every sum minus P is representable,
    while for the 31-bit primes sums of 2^31 and more occur, which a signed
    32-bit word would read as negative.  Hence the kernel's unsigned borrow
    form."""
    lim = 1 << 31
    for P in (469762049, 998244353):
        a, b = samples(P, seed=2)
        for x, y in zip(a, b):
            q1, q2, q3, _ = fourier_parts(x, y, P)
            t = q1 - q2 + q3
            assert -lim <= t < lim and -lim <= t - P < lim
    for P in (2013265921, 2113929217):
        a, b = samples(P, seed=3)
        tops = [sum(fourier_parts(x, y, P)[i] * (1, -1, 1)[i] for i in range(3)) for x, y in zip(a, b)]
        assert max(tops) >= lim
        assert 2 * (P - 1) > lim - 1


def barrett_quantities(a, b, P):
    """Algorithm 1's quantities from their definitions: k the bit length of P,
    the precomputed floor(2^2k / P), the quotient estimate q = floor(floor(ab /
    2^k) floor(2^2k / P) / 2^k) and the remainder t = ab - qP."""
    k = P.bit_length()                                 # ceil(log2 P) for P not a power of two
    inv = (1 << (2 * k)) // P
    q = (((a * b) >> k) * inv) >> k
    return q, a * b - q * P


@pytest.mark.parametrize("P", FOURIER + [3, 17, 65537, (1 << 31) - 1, 1000003])
def test_barrett_quotient_bound(P):
    """The quotient estimate undershoots floor(ab / P) by at most 3, so the
    remainder t = ab - qP lies in [0, 4P) and is congruent to ab: at most three
    subtractions of P finish the reduction (one of 2P and one of P in the
    kernel's form), and t < 4P < 2^33 bounds the intermediate."""
    a, b = samples(P, seed=4)
    for x, y in zip(a, b):
        q, t = barrett_quantities(x, y, P)
        assert 0 <= (x * y) // P - q <= 3
        assert 0 <= t < 4 * P and t % P == x * y % P
        r = t - 2 * P if t >= 2 * P else t                 # the kernel's two conditional subtractions
        r = r - P if r >= P else r
        assert r == x * y % P


def test_oracle_plain_routines():
    rng = np.random.default_rng(5)
    for P in (17, 998244353, 2113929217):
        a = rng.integers(0, P, 2000, dtype=np.uint32)
        b = rng.integers(0, P, 2000, dtype=np.uint32)
        assert oracle.modmul(P, a, b).tolist() == [int(x) * int(y) % P for x, y in zip(a, b)]
        e = rng.integers(0, 1 << 32, 2000, dtype=np.uint64).astype(np.uint32)
        assert oracle.modpow(P, a, e).tolist() == [pow(int(x), int(y), P) for x, y in zip(a, e)]
    assert oracle.modpow(7, np.array([0], np.uint32), np.array([0], np.uint32))[0] == 1
