"""GPU parity of the 64-bit-residue kernels (R = 2^64) against the CPU oracle;
every comparison is bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

R64 = 1 << 64
MODULI = list(wl.PRIMES64) + [3, 5, 15, 17, 65537, (1 << 61) - 1, (1 << 63) - 7, (1 << 62) + 135, (1 << 32) + 15,
                              (1 << 31) - 1]


@pytest.fixture(scope="module")
def M64():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1609_00999_amd import mont64
    mont64.lib()
    return mont64


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64)).to("cuda")


def host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def edges64(P):
    v = [0, 1, 2, 3, P - 1, P - 2, (P - 1) // 2, (P + 1) // 2, R64 % P, (R64 * R64) % P, 1 << 32, (1 << 32) - 1,
         (1 << 32) + 1, 1 << 62, (1 << 63) - 1]
    return np.array(sorted({x % P for x in v}), dtype=np.uint64)


def test_setup_matches_oracle(M64):
    from paper_1609_00999_amd import mont
    for P in MODULI:
        prm, ref = M64.setup(P), oracle.setup64(P)
        assert (prm.P, prm.Pprime, prm.R1, prm.R2, prm.k) == (P, ref.Pprime, ref.R1, ref.R2, ref.k)
    for bad in (0, 1, 2, 4, 1 << 63, (1 << 63) + 1, (1 << 64) - 1):
        with pytest.raises(mont.MontError):
            M64.setup(bad)


@pytest.mark.parametrize("P", MODULI)
def test_ops_edges_and_random(M64, P):
    prm = M64.setup(P)
    rng = np.random.default_rng(P % 9973)
    e = edges64(P)
    a = np.concatenate([np.repeat(e, e.size), wl.uniform64(rng, 0, P, 20001)])
    b = np.concatenate([np.tile(e, e.size), wl.uniform64(rng, 0, P, 20001)])
    c = wl.uniform64(rng, 0, P, a.size)
    da, db, dc = dev(a), dev(b), dev(c)
    assert np.array_equal(host(M64.mul(prm, da, db)), oracle.mont_mul64(P, a, b))
    assert np.array_equal(host(M64.muladd(prm, da, db, dc)), oracle.mont_muladd64(P, a, b, c))
    x = np.concatenate([rng.integers(0, 1 << 64, 20001, dtype=np.uint64),
                        np.array([0, 1, P - 1, P, P + 1, R64 - 1, 1 << 63, (1 << 63) - 1], dtype=np.uint64)])
    dx = dev(x)
    assert np.array_equal(host(M64.to_mont(prm, dx)), oracle.to_mont64(P, x))
    assert np.array_equal(host(M64.from_mont(prm, dx)), oracle.from_mont64(P, x))
    ex = rng.integers(0, 1 << 64, a.size, dtype=np.uint64)
    ex[:4] = [0, 1, (1 << 64) - 1, 1 << 63]
    assert np.array_equal(host(M64.pow(prm, da, dev(ex))), oracle.mont_pow64(P, a, ex))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 63, 64, 65, 127, 129, 4097, (1 << 18) + 3])
def test_ragged_sizes(M64, n):
    P = wl.PRIMES64[0]
    prm = M64.setup(P)
    rng = np.random.default_rng(n + 5)
    a, b, c = (wl.uniform64(rng, 0, P, n) for _ in range(3))
    assert np.array_equal(host(M64.mul(prm, dev(a), dev(b))), oracle.mont_mul64(P, a, b))
    assert np.array_equal(host(M64.muladd(prm, dev(a), dev(b), dev(c))), oracle.mont_muladd64(P, a, b, c))
    assert np.array_equal(host(M64.pow(prm, dev(a), dev(b))), oracle.mont_pow64(P, a, b))


def test_misaligned_and_in_place(M64):
    P = wl.PRIMES64[3]
    prm = M64.setup(P)
    rng = np.random.default_rng(21)
    n = 10001
    a, b, c = (wl.uniform64(rng, 0, P, n + 1) for _ in range(3))
    da, db = dev(a), dev(b)
    out = torch.empty(n + 1, dtype=torch.int64, device="cuda")[1:]          # 8 bytes off a 16-byte boundary
    M64.mul(prm, da[1:], db[1:], out=out)
    assert np.array_equal(host(out), oracle.mont_mul64(P, a[1:], b[1:]))
    dc = dev(c)
    M64.muladd(prm, da, db, dc, out=dc)
    assert np.array_equal(host(dc), oracle.mont_muladd64(P, a, b, c))
    dx = dev(a)
    M64.to_mont(prm, dx, out=dx)
    M64.from_mont(prm, dx, out=dx)
    assert np.array_equal(host(dx), a)


def test_argument_errors(M64):
    from paper_1609_00999_amd import mont
    prm = M64.setup(wl.PRIMES64[0])
    x = dev(np.ones(8, dtype=np.uint64))
    with pytest.raises(TypeError):
        M64.mul(prm, x.to(torch.int32), x.to(torch.int32))
    with pytest.raises(ValueError):
        M64.mul(prm, x, x[:4])
    bad = M64.Mont64Params()
    bad.P, bad.Pprime = 17, 1
    with pytest.raises(mont.MontError):
        M64.mul(bad, x, x)


@pytest.mark.parametrize("pi", range(4))
def test_bandwidth64_full_size(M64, pi):
    """2^27 residues per array: mul and in-place mul-add, every element
    compared with the oracle."""
    P, a, b, c = wl.bandwidth_triple64(pi)
    prm = M64.setup(P)
    da, db, dc = dev(a), dev(b), dev(c)
    got = host(M64.mul(prm, da, db))
    bad = np.flatnonzero(got != oracle.mont_mul64(P, a, b))
    assert bad.size == 0, (bad.size, bad[:8].tolist())
    del got
    M64.muladd(prm, da, db, dc, out=dc)
    got = host(dc)
    bad = np.flatnonzero(got != oracle.mont_muladd64(P, a, b, c))
    assert bad.size == 0, (bad.size, bad[:8].tolist())


def test_pow64_config(M64):
    """2^22 bases and 64-bit exponents modulo 2^63 - 25: every power compared
    with the oracle, and Fermat on the first 2^14 bases."""
    P = wl.PRIMES64[3]
    prm = M64.setup(P)
    base, e = wl.pow64_inputs()
    out = host(M64.pow(prm, dev(base), dev(e)))
    bad = np.flatnonzero(out != oracle.mont_pow64(P, base, e))
    assert bad.size == 0, (bad.size, bad[:8].tolist())
    sub = base[: 1 << 14]
    f = host(M64.pow(prm, dev(sub), dev(np.full(sub.size, P - 1, dtype=np.uint64))))
    assert np.all(f == prm.R1)
