"""Pins for the CPU oracle (no GPU).

The oracle computes plain definitions; these tests tie it to facts that do not
come from the oracle itself: exhaustive search at tiny moduli, the paper's own
algorithm run step by step in Python big integers, closed forms of the
precomputation, Fermat's little theorem and Euler's criterion, Python's
built-in modular power, the direct O(N^2) transform, schoolbook convolution in
pure Python, binomial coefficients, and Horner evaluation (Schwartz-Zippel).
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

ALL_PRIMES = sorted(set(wl.PRIMES_BW) | set(wl.PRIMES_NTT))


# --------------------------------------------------------------------------
# Precomputation (section 3.1: R R^-1 - P P' = 1, 0 < R^-1 < P, 0 < P' < R)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("P", ALL_PRIMES + [3, 5, 15, 17, 65537, (1 << 31) - 1])
def test_setup_closed_forms(P):
    prm = oracle.setup(P)
    R = 1 << 32
    assert R * prm.Rinv - P * prm.Pprime == 1
    assert 0 < prm.Rinv < P and 0 < prm.Pprime < R
    assert (P * prm.Pprime) % R == R - 1            # P' = -P^-1 mod R
    assert (prm.R1 * prm.Rinv) % P == 1 and prm.R1 < P
    assert (prm.R2 * prm.Rinv * prm.Rinv) % P == 1 and prm.R2 < P
    assert (P - 1) % (1 << prm.k) == 0 and ((P - 1) >> prm.k) & 1 == 1


@pytest.mark.parametrize("P", ALL_PRIMES)
def test_fourier_prime_pprime(P):
    # P = 1 + c 2^k with 2k >= 32: (1 + c 2^k)^-1 = 1 - c 2^k mod 2^32, so
    # P' = -P^-1 = c 2^k - 1 = P - 2 (the Fourier-prime shortcut of section 3.1).
    prm = oracle.setup(P)
    assert prm.k >= 16
    assert prm.Pprime == P - 2


def test_setup_tiny():
    prm = oracle.setup(17, r=5)
    assert (prm.Pprime, prm.Rinv, prm.R1) == (15, 8, 15)


@pytest.mark.parametrize("bad", [0, 1, 2, 4, 1 << 31, (1 << 32) - 2])
def test_setup_rejects(bad):
    with pytest.raises(ValueError):
        oracle.setup(bad)


# --------------------------------------------------------------------------
# Montgomery product at tiny moduli, exhaustively
# --------------------------------------------------------------------------

def redc_alg2(a, b, P, Pp, R):
    """Algorithm 2 step by step in Python integers, asserting the range facts
    stated beside it: T + mP is divisible by R and 0 <= t < 2P."""
    T = a * b
    m = ((T % R) * Pp) % R
    assert (T + m * P) % R == 0
    t = (T + m * P) // R
    assert 0 <= t < 2 * P
    return t - P if t >= P else t


def by_search(a, b, P, R):
    """The unique z in [0, P) with z R = a b (mod P), by search."""
    hits = [z for z in range(P) if (z * R - a * b) % P == 0]
    assert len(hits) == 1
    return hits[0]


def test_bruteforce_p17_r32():
    P, r = 17, 5
    R = 1 << r
    prm = oracle.setup(P, r)
    a, b = np.meshgrid(np.arange(P, dtype=np.uint32), np.arange(P, dtype=np.uint32), indexing="ij")
    got = oracle.mont_mul(P, a.ravel(), b.ravel(), r=r).reshape(P, P)
    for x in range(P):
        for y in range(P):
            want = by_search(x, y, P, R)
            assert got[x, y] == want
            assert redc_alg2(x, y, P, prm.Pprime, R) == want


@pytest.mark.parametrize("r", [6, 8])
def test_bruteforce_all_odd_moduli(r):
    R = 1 << r
    hit_t_equals_p = 0
    for P in range(3, 64, 2):
        prm = oracle.setup(P, r)
        xs = np.arange(P, dtype=np.uint32)
        a, b = np.meshgrid(xs, xs, indexing="ij")
        got = oracle.mont_mul(P, a.ravel(), b.ravel(), r=r).reshape(P, P)
        table = {}
        for z in range(P):
            table.setdefault((z * R) % P, z)
        for x in range(P):
            for y in range(P):
                want = table[(x * y) % P]
                assert got[x, y] == want, (P, x, y)
                assert redc_alg2(x, y, P, prm.Pprime, R) == want
                T = x * y
                m = ((T % R) * prm.Pprime) % R
                hit_t_equals_p += (T + m * P) // R == P
    # composite moduli reach t == P before the final subtraction
    assert hit_t_equals_p > 0


def test_t_equals_p_count_p15():
    # For the composite modulus P = 15 with R = 2^5, Algorithm 2's value t
    # before the final comparison equals P for 16 of the 225 operand pairs, so
    # the comparison must be t >= P (not t > P) for a canonical result.
    P, R = 15, 32
    prm = oracle.setup(P, 5)
    cnt = 0
    for x in range(P):
        for y in range(P):
            T = x * y
            m = ((T % R) * prm.Pprime) % R
            cnt += (T + m * P) // R == P
    assert cnt == 16


# --------------------------------------------------------------------------
# Montgomery product at R = 2^32
# --------------------------------------------------------------------------

def edge_values(P):
    prm = oracle.setup(P)
    v = [0, 1, 2, P - 1, P - 2, (P - 1) // 2, (P + 1) // 2, prm.R1, prm.R2, 1 << 16, (1 << 16) + 1]
    return np.array(sorted({x % P for x in v}), dtype=np.uint32)


@pytest.mark.parametrize("P", wl.PRIMES_BW + (17, 65537, 2130706433, 15))
def test_alg2_matches_oracle_r32(P):
    prm = oracle.setup(P)
    rng = np.random.default_rng(11)
    e = edge_values(P)
    a = np.concatenate([np.repeat(e, e.size), rng.integers(0, P, 4000, dtype=np.uint32)])
    b = np.concatenate([np.tile(e, e.size), rng.integers(0, P, 4000, dtype=np.uint32)])
    got = oracle.mont_mul(P, a, b)
    for x, y, g in zip(a.tolist(), b.tolist(), got.tolist()):
        assert redc_alg2(x, y, P, prm.Pprime, 1 << 32) == g


@pytest.mark.parametrize("P", wl.PRIMES_BW)
def test_roundtrip_and_identity(P):
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.integers(0, 1 << 32, 1 << 18, dtype=np.uint32),
                        np.array([0, 1, P - 1, P, P + 1, (1 << 32) - 1, (1 << 31), 1 << 16], dtype=np.uint32)])
    # round trip from(to(a)) = a mod P for any uint32 a
    assert np.array_equal(oracle.from_mont(P, oracle.to_mont(P, a)), a % np.uint32(P))
    # REDC(aR * bR) = abR: the Montgomery product of residues is the residue of ab
    x = rng.integers(0, P, 1 << 16, dtype=np.uint32)
    y = rng.integers(0, P, 1 << 16, dtype=np.uint32)
    prod = oracle.from_mont(P, oracle.mont_mul(P, oracle.to_mont(P, x), oracle.to_mont(P, y)))
    want = (x.astype(np.uint64) * y.astype(np.uint64)) % np.uint64(P)
    assert np.array_equal(prod, want.astype(np.uint32))
    # to(1) is the residue of 1; from() of it is 1
    assert oracle.to_mont(P, np.array([1], dtype=np.uint32))[0] == oracle.setup(P).R1


def test_roundtrip_strided_full_range():
    # every 251st uint32 (the whole 32-bit range is walked on the GPU)
    P = wl.P_PLAIN
    a = np.arange(0, 1 << 32, 251, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(oracle.from_mont(P, oracle.to_mont(P, a)), a % np.uint32(P))


@pytest.mark.parametrize("P", wl.PRIMES_BW)
def test_muladd(P):
    rng = np.random.default_rng(6)
    a, b, c = (rng.integers(0, P, 1 << 14, dtype=np.uint32) for _ in range(3))
    zero = np.zeros_like(c)
    assert np.array_equal(oracle.mont_muladd(P, a, b, zero), oracle.mont_mul(P, a, b))
    # residues add like ordinary values (section 3.1)
    got = oracle.from_mont(P, oracle.mont_muladd(P, oracle.to_mont(P, a), oracle.to_mont(P, b),
                                                  oracle.to_mont(P, c)))
    want = (a.astype(object) * b.astype(object) + c.astype(object)) % P
    assert np.array_equal(got.astype(object), want)


# --------------------------------------------------------------------------
# Powers
# --------------------------------------------------------------------------

@pytest.mark.parametrize("P", [wl.P_POW, 2013265921, 2113929217])
def test_pow_fermat_euler_builtin(P):
    rng = np.random.default_rng(7)
    a = rng.integers(1, P, 2000, dtype=np.uint32)
    abar = oracle.to_mont(P, a)
    one = oracle.setup(P).R1
    # Fermat: a^(P-1) = 1
    ef = np.full(a.size, P - 1, dtype=np.uint32)
    assert np.all(oracle.mont_pow(P, abar, ef) == one)
    # Euler's criterion: a^((P-1)/2) is +-1
    eh = np.full(a.size, (P - 1) // 2, dtype=np.uint32)
    h = oracle.from_mont(P, oracle.mont_pow(P, abar, eh))
    assert np.all((h == 1) | (h == P - 1))
    assert np.any(h == 1) and np.any(h == P - 1)
    # Python's built-in modular power
    e = rng.integers(0, 1 << 32, a.size, dtype=np.uint64).astype(np.uint32)
    got = oracle.from_mont(P, oracle.mont_pow(P, abar, e))
    assert [int(g) for g in got] == [pow(int(x), int(y), P) for x, y in zip(a, e)]


def test_pow_conventions():
    P = wl.P_POW
    prm = oracle.setup(P)
    rng = np.random.default_rng(8)
    abar = rng.integers(0, P, 500, dtype=np.uint32)
    z = np.zeros_like(abar)
    assert np.all(oracle.mont_pow(P, abar, z) == prm.R1)          # x^0 = 1, including 0^0
    assert np.array_equal(oracle.mont_pow(P, abar, z + 1), abar)  # x^1 = x
    e = rng.integers(0, 1 << 20, abar.size, dtype=np.uint32)
    f = rng.integers(0, 1 << 20, abar.size, dtype=np.uint32)
    lhs = oracle.mont_pow(P, abar, e + f)
    rhs = oracle.mont_mul(P, oracle.mont_pow(P, abar, e), oracle.mont_pow(P, abar, f))
    assert np.array_equal(lhs, rhs)
    # small exponents against repeated products
    acc = np.full(abar.size, prm.R1, dtype=np.uint32)
    for k in range(6):
        assert np.array_equal(oracle.mont_pow(P, abar, np.full(abar.size, k, dtype=np.uint32)), acc)
        acc = oracle.mont_mul(P, acc, abar)


# --------------------------------------------------------------------------
# Primitive roots and the plain transform
# --------------------------------------------------------------------------

def prime_factors(n):
    out, f = [], 2
    while f * f <= n:
        if n % f == 0:
            out.append(f)
            while n % f == 0:
                n //= f
        f += 1
    if n > 1:
        out.append(n)
    return out


@pytest.mark.parametrize("P", ALL_PRIMES)
def test_primitive_root_smallest(P):
    g = oracle.primitive_root(P)
    qs = prime_factors(P - 1)
    assert all(pow(g, (P - 1) // q, P) != 1 for q in qs)
    for h in range(2, g):
        assert any(pow(h, (P - 1) // q, P) == 1 for q in qs)


@pytest.mark.parametrize("P", wl.PRIMES_NTT[:3])
@pytest.mark.parametrize("logn", [0, 1, 2, 3, 5, 6])
def test_ntt_is_the_dft(P, logn):
    n = 1 << logn
    g = oracle.primitive_root(P)
    w = pow(g, (P - 1) // n, P)
    assert pow(w, n, P) == 1
    if n >= 2:
        assert pow(w, n // 2, P) == P - 1
    rng = np.random.default_rng(logn)
    a = rng.integers(0, P, n, dtype=np.uint32)
    got = oracle.ntt(P, a, w)
    want = [sum(int(a[j]) * pow(w, j * k, P) for j in range(n)) % P for k in range(n)]
    assert got.tolist() == want
    # inverse with w^-1 and n^-1 returns the input
    back = oracle.ntt(P, got, pow(w, P - 2, P))
    ninv = pow(n, P - 2, P)
    assert [(int(x) * ninv) % P for x in back] == a.tolist()


# --------------------------------------------------------------------------
# Polynomial products
# --------------------------------------------------------------------------

def py_convolve(a, b, P):
    c = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            c[i + j] = (c[i + j] + int(x) * int(y)) % P
    return c


@pytest.mark.parametrize("da,db", [(0, 0), (0, 5), (1, 1), (7, 3), (31, 32), (63, 64)])
def test_schoolbook_vs_python(da, db):
    P = wl.PRIMES_NTT[0]
    rng = np.random.default_rng(da * 100 + db)
    a = rng.integers(0, P, da + 1, dtype=np.uint32)
    b = rng.integers(0, P, db + 1, dtype=np.uint32)
    assert oracle.polymul_schoolbook(P, a, b).tolist() == py_convolve(a, b, P)


@pytest.mark.parametrize("P", wl.PRIMES_NTT)
def test_ntt_polymul_vs_schoolbook(P):
    rng = np.random.default_rng(P % 1000)
    for da, db in [(0, 0), (1, 0), (5, 9), (255, 256), (1023, 1023), (2047, 1000)]:
        a = rng.integers(0, P, da + 1, dtype=np.uint32)
        b = rng.integers(0, P, db + 1, dtype=np.uint32)
        c = np.empty(da + db + 1, dtype=np.uint32)
        need = da + db + 1
        n = 1 << (need - 1).bit_length()
        work = np.empty(2 * n, dtype=np.uint32)
        lib = oracle._load()
        rc = lib.orc_polymul_ntt(P, oracle.primitive_root(P), oracle._p(a), da, oracle._p(b), db,
                                 oracle._p(c), oracle._p(work))
        assert rc == 0
        assert np.array_equal(c, oracle.polymul_schoolbook(P, a, b))


def test_polymul_special_cases():
    P = wl.PRIMES_NTT[1]
    rng = np.random.default_rng(9)
    for d in [1, 100, 3000, 5000]:
        b = rng.integers(0, P, d + 1, dtype=np.uint32)
        one = np.array([1], dtype=np.uint32)
        assert np.array_equal(oracle.polymul(P, one, b), b)              # 1 * b = b
        k = 7
        xk = np.zeros(k + 1, dtype=np.uint32)
        xk[k] = 1
        c = oracle.polymul(P, xk, b)                                      # x^k * b = shift
        assert np.all(c[:k] == 0) and np.array_equal(c[k:], b)
        ones = np.ones(d + 1, dtype=np.uint32)
        c = oracle.polymul(P, ones, ones)                                 # all-ones
        kk = np.arange(2 * d + 1)
        assert np.array_equal(c, (np.minimum(kk, 2 * d - kk) + 1).astype(np.uint32))
    for d in [3, 50, 2500]:
        binom = np.array([math.comb(d, k) % P for k in range(d + 1)], dtype=np.uint32)
        c = oracle.polymul(P, binom, binom)                               # (1+x)^d (1+x)^d
        assert c.tolist() == [math.comb(2 * d, k) % P for k in range(2 * d + 1)]


def test_horner_vs_python():
    P = wl.PRIMES_NTT[2]
    rng = np.random.default_rng(10)
    a = rng.integers(0, P, 40, dtype=np.uint32)
    for x in [0, 1, 2, P - 1, 123456789]:
        assert oracle.horner(P, a, x) == sum(int(c) * pow(x, i, P) for i, c in enumerate(a)) % P


@pytest.mark.parametrize("d", [4095, 20000, 70000])
def test_polymul_schwartz_zippel(d):
    P = wl.PRIMES_NTT[3]
    rng = np.random.default_rng(d)
    a = rng.integers(0, P, d + 1, dtype=np.uint32)
    b = rng.integers(0, P, d + 1, dtype=np.uint32)
    c = oracle.polymul(P, a, b)
    assert c.size == 2 * d + 1
    for x in rng.integers(2, P, 4).tolist():
        assert oracle.horner(P, c, x) == (oracle.horner(P, a, x) * oracle.horner(P, b, x)) % P


def test_golden_fixtures():
    """Fixtures under tests/golden were written by tests/golden/make_golden.py,
    which calls only the oracle; re-derive them here."""
    path = os.path.join(GOLDEN, "polymul_small.txt")
    with open(path) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert lines
    for ln in lines:
        P, da, db = int(ln[0]), int(ln[1]), int(ln[2])
        a = np.array(ln[3:4 + da], dtype=np.uint64).astype(np.uint32)
        b = np.array(ln[4 + da:5 + da + db], dtype=np.uint64).astype(np.uint32)
        c = [int(x) for x in ln[5 + da + db:]]
        assert py_convolve(a, b, P) == c
