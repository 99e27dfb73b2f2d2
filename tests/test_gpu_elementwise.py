"""GPU parity of the elementwise Montgomery kernels against the CPU oracle.

Every comparison is bit-exact (integer arithmetic, unique canonical results).
"""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1609_00999_amd import mont
    mont.lib()
    return mont


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to("cuda")


def host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def edge_values(P):
    prm = oracle.setup(P)
    v = [0, 1, 2, 3, P - 1, P - 2, (P - 1) // 2, (P + 1) // 2, prm.R1, prm.R2, 1 << 16, (1 << 16) + 1,
         (1 << 16) - 1]
    return np.array(sorted({x % P for x in v}), dtype=np.uint32)


MODULI = list(wl.PRIMES_BW) + [3, 15, 17, 65537, 2130706433, (1 << 31) - 1, 2147483647 - 2]


def test_setup_matches_oracle(M):
    for P in MODULI + list(wl.PRIMES_NTT):
        prm, ref = M.setup(P), oracle.setup(P)
        assert (prm.P, prm.Pprime, prm.R1, prm.R2, prm.k) == (P, ref.Pprime, ref.R1, ref.R2, ref.k)
    for bad in (0, 1, 2, 4, 1 << 31, (1 << 32) - 1):
        with pytest.raises(M.MontError):
            M.setup(bad)


@pytest.mark.parametrize("P", MODULI)
def test_ops_edges_and_random(M, P):
    prm = M.setup(P)
    rng = np.random.default_rng(P % 9973)
    e = edge_values(P)
    a = np.concatenate([np.repeat(e, e.size), rng.integers(0, P, 50000, dtype=np.uint32)])
    b = np.concatenate([np.tile(e, e.size), rng.integers(0, P, 50000, dtype=np.uint32)])
    c = rng.integers(0, P, a.size, dtype=np.uint32)
    da, db, dc = dev(a), dev(b), dev(c)
    assert np.array_equal(host(M.mul(prm, da, db)), oracle.mont_mul(P, a, b))
    assert np.array_equal(host(M.muladd(prm, da, db, dc)), oracle.mont_muladd(P, a, b, c))
    # conversions accept every uint32
    x = np.concatenate([rng.integers(0, 1 << 32, 50000, dtype=np.uint64).astype(np.uint32),
                        np.array([0, 1, P - 1, P, P + 1, (1 << 32) - 1, 1 << 31, (1 << 31) - 1], dtype=np.uint32)])
    dx = dev(x)
    assert np.array_equal(host(M.to_mont(prm, dx)), oracle.to_mont(P, x))
    assert np.array_equal(host(M.from_mont(prm, dx)), oracle.from_mont(P, x))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 7, 8, 63, 64, 65, 1023, 1025, 4097 * 3, 256 * 1024 + 3,
                               (1 << 20) + 1])
def test_ragged_sizes(M, n):
    P = wl.P_PLAIN
    prm = M.setup(P)
    rng = np.random.default_rng(n)
    a = rng.integers(0, P, n, dtype=np.uint32)
    b = rng.integers(0, P, n, dtype=np.uint32)
    c = rng.integers(0, P, n, dtype=np.uint32)
    got = host(M.mul(prm, dev(a), dev(b)))
    assert np.array_equal(got, oracle.mont_mul(P, a, b))
    got = host(M.muladd(prm, dev(a), dev(b), dev(c)))
    assert np.array_equal(got, oracle.mont_muladd(P, a, b, c))
    got = host(M.pow(prm, dev(a), dev(b)))
    assert np.array_equal(got, oracle.mont_pow(P, a, b))


@pytest.mark.parametrize("off", [1, 2, 3])
def test_misaligned_views(M, off):
    P = wl.PRIMES_BW[3]
    prm = M.setup(P)
    rng = np.random.default_rng(off)
    n = 10000 + off
    a = rng.integers(0, P, n + off, dtype=np.uint32)
    b = rng.integers(0, P, n + off, dtype=np.uint32)
    da, db = dev(a), dev(b)
    va, vb = da[off:], db[off:]
    out = torch.empty(n + off, dtype=torch.int32, device="cuda")[off:]
    M.mul(prm, va, vb, out=out)
    assert np.array_equal(host(out), oracle.mont_mul(P, a[off:], b[off:]))
    M.to_mont(prm, va, out=out)
    assert np.array_equal(host(out), oracle.to_mont(P, a[off:]))


def test_in_place(M):
    P = wl.PRIMES_BW[2]
    prm = M.setup(P)
    rng = np.random.default_rng(12)
    a, b, c = (rng.integers(0, P, 100003, dtype=np.uint32) for _ in range(3))
    dc = dev(c)
    M.muladd(prm, dev(a), dev(b), dc, out=dc)
    assert np.array_equal(host(dc), oracle.mont_muladd(P, a, b, c))
    da = dev(a)
    M.mul(prm, da, dev(b), out=da)
    assert np.array_equal(host(da), oracle.mont_mul(P, a, b))
    dx = dev(a)
    M.to_mont(prm, dx, out=dx)
    M.from_mont(prm, dx, out=dx)
    assert np.array_equal(host(dx), a)


def test_plain_pipeline_full_size(M):
    """n = 2^20 pairs, P = 15*2^27+1: to, to, mul, from returns a*b mod P."""
    P = wl.P_PLAIN
    prm = M.setup(P)
    a, b = wl.plain_pairs()
    ta, tb = M.to_mont(prm, dev(a)), M.to_mont(prm, dev(b))
    c = host(M.from_mont(prm, M.mul(prm, ta, tb)))
    want = (a.astype(np.uint64) * b.astype(np.uint64)) % np.uint64(P)
    assert np.array_equal(c, want.astype(np.uint32))
    assert np.array_equal(c, oracle.from_mont(P, oracle.mont_mul(P, oracle.to_mont(P, a), oracle.to_mont(P, b))))


def test_roundtrip_all_uint32(M):
    """from(to(x)) = x mod P for every 32-bit x, checked on the device in 2^28 chunks."""
    P = wl.P_PLAIN
    prm = M.setup(P)
    chunk = 1 << 28
    x = torch.empty(chunk, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    idx = torch.arange(chunk, dtype=torch.int64, device="cuda")
    for k in range((1 << 32) // chunk):
        vals = idx + k * chunk                      # int64 values 0 .. 2^32-1
        x.copy_(vals.to(torch.int32))               # wraps to the same bit pattern
        M.to_mont(prm, x, out=y)
        M.from_mont(prm, y, out=y)
        want = torch.remainder(vals, P).to(torch.int32)
        assert torch.equal(y, want), "chunk %d" % k
    torch.cuda.synchronize()


@pytest.mark.parametrize("pi", range(4))
def test_bandwidth_config_full_size(M, pi):
    """n = 2^28 Montgomery residues per prime: mul and in-place muladd,
    compared element by element with the oracle."""
    P, a, b, c = wl.bandwidth_triple(pi)
    prm = M.setup(P)
    da, db, dc = dev(a), dev(b), dev(c)
    out = M.mul(prm, da, db)
    got = host(out)
    assert np.array_equal(got, oracle.mont_mul(P, a, b))
    del got
    M.muladd(prm, da, db, dc, out=dc)
    got = host(dc)
    assert np.array_equal(got, oracle.mont_muladd(P, a, b, c))


def test_pow_config(M):
    """n = 2^24 bases, 31-bit exponents, P = 998244353: every power compared
    with the oracle, and Fermat a^(P-1) = 1 on the first 2^16 bases."""
    P = wl.P_POW
    prm = M.setup(P)
    base, e = wl.pow_inputs()
    out = host(M.pow(prm, dev(base), dev(e)))
    want = oracle.mont_pow(P, base, e)
    bad = np.flatnonzero(out != want)
    assert bad.size == 0, (bad.size, bad[:8].tolist())
    sub = base[: 1 << 16]
    f = host(M.pow(prm, dev(sub), dev(np.full(sub.size, P - 1, dtype=np.uint32))))
    assert np.all(f == prm.R1)
    # Euler's criterion and exponent edges
    h = host(M.from_mont(prm, M.pow(prm, dev(sub), dev(np.full(sub.size, (P - 1) // 2, dtype=np.uint32)))))
    assert np.all((h == 1) | (h == P - 1))
    for ev in (0, 1, 2, 3, (1 << 32) - 1, 1 << 31):
        ee = np.full(sub.size, ev, dtype=np.uint32)
        assert np.array_equal(host(M.pow(prm, dev(sub), dev(ee))), oracle.mont_pow(P, sub, ee))


def test_exhaustive_tiny_modulus(M):
    """All pairs (a, b) in [0, P)^2 for small moduli with R = 2^32."""
    for P in (3, 5, 15, 17, 97, 255, 257):
        prm = M.setup(P)
        xs = np.arange(P, dtype=np.uint32)
        a, b = np.meshgrid(xs, xs, indexing="ij")
        a, b = a.ravel().copy(), b.ravel().copy()
        assert np.array_equal(host(M.mul(prm, dev(a), dev(b))), oracle.mont_mul(P, a, b))
        assert np.array_equal(host(M.pow(prm, dev(a), dev(b))), oracle.mont_pow(P, a, b))


@pytest.mark.parametrize("P", sorted(set(wl.PRIMES_BW) | set(wl.PRIMES_NTT)))
def test_fourier_redc_matches_alg2(M, P):
    """Algorithm 3 (Fourier-prime REDC, borrow form) gives Algorithm 2's results."""
    prm = M.setup(P)
    rng = np.random.default_rng(P % 7919)
    e = edge_values(P)
    a = np.concatenate([np.repeat(e, e.size), rng.integers(0, P, 100003, dtype=np.uint32)])
    b = np.concatenate([np.tile(e, e.size), rng.integers(0, P, a.size - e.size * e.size, dtype=np.uint32)])
    da, db = dev(a), dev(b)
    assert np.array_equal(host(M.mul_fourier(prm, da, db)), oracle.mont_mul(P, a, b))
    ex = rng.integers(0, 1 << 32, a.size, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(host(M.pow_fourier(prm, da, dev(ex))), oracle.mont_pow(P, a, ex))
    assert np.array_equal(host(M.pow_fourier(prm, da, dev(ex))), host(M.pow(prm, da, dev(ex))))


@pytest.mark.parametrize("P", [3, 17, 65537, 1000003, 2147483647] + list(wl.PRIMES_BW))
def test_barrett_matches_plain(M, P):
    """Algorithm 1 (Barrett) on ordinary residues against the plain product."""
    rng = np.random.default_rng(P % 6007)
    n = 50001
    a = rng.integers(0, P, n, dtype=np.uint32)
    b = rng.integers(0, P, n, dtype=np.uint32)
    a[:4] = [0, 1, P - 1, P - 1]
    b[:4] = [P - 1, P - 1, P - 1, 1]
    da, db = dev(a), dev(b)
    assert np.array_equal(host(M.mul_barrett(P, da, db)), oracle.modmul(P, a, b))
    ex = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(host(M.pow_barrett(P, da, dev(ex))), oracle.modpow(P, a, ex))


def test_alt_reduction_errors(M):
    prm = M.setup(2013265921)
    x = dev(np.ones(8, dtype=np.uint32))
    with pytest.raises(M.MontError):
        M.mul_fourier(M.setup(17), x, x)        # v2(16) = 4 < 16: not a usable Fourier prime
    with pytest.raises(M.MontError):
        M.mul_barrett(10, x, x)
    assert np.array_equal(host(M.mul_fourier(prm, x[1:], x[1:])), oracle.mont_mul(2013265921, np.ones(7, np.uint32),
                                                                                 np.ones(7, np.uint32)))


def test_checked_mode(M):
    """mont_check_range flags operands outside [0, P) on the device; the
    checked() block raises MONT_ERANGE and leaves in-range work untouched."""
    P = wl.PRIMES_BW[1]
    prm = M.setup(P)
    rng = np.random.default_rng(77)
    for n in (1, 3, 4, 5, 4097, 100003):
        for off in (0, 1):
            x = rng.integers(0, P, n + off, dtype=np.uint32)
            st = torch.zeros(1, dtype=torch.int32, device="cuda")
            dx = dev(x)[off:]
            M.check_range(P, dx, st)
            assert int(st.item()) == 0
            bad = x.copy()
            bad[off + (n - 1) // 2] = P               # the first value out of range
            M.check_range(P, dev(bad)[off:], st)
            assert int(st.item()) == M.ERANGE
    a = rng.integers(0, P, 4096, dtype=np.uint32)
    b = a.copy()
    b[4095] = 0xFFFFFFFF
    with M.checked():
        got = host(M.mul(prm, dev(a), dev(a)))
    assert np.array_equal(got, oracle.mont_mul(P, a, a))
    with pytest.raises(M.MontError) as ei:
        with M.checked():
            M.mul(prm, dev(a), dev(b))
    assert ei.value.status == M.ERANGE
    with pytest.raises(M.MontError):
        with M.checked():
            M.pow(prm, dev(b), dev(a))              # the base is checked, the exponent is not
    with M.checked():
        M.pow(prm, dev(a), dev(b))
    assert M.checked_status() == 0
    with pytest.raises(M.MontError):
        M.check_range(0, dev(a), torch.zeros(1, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("P", [3, 5, 15, 17, 65537, 469762049, 998244353, (1 << 30) - 35, (1 << 30) - 1,
                               (1 << 30) + 1, (1 << 30) + 3, 2013265921, 2147483647])
def test_pow_both_reduction_paths(M, P):
    """Powers for moduli on both sides of 2^30: below it the power chain keeps
    its values in [0, 2P) and reduces once at the end; above it every product
    is reduced.  Edge bases and exponents, against the oracle."""
    prm = M.setup(P)
    rng = np.random.default_rng(P % 65521)
    e = edge_values(P)
    base = np.concatenate([np.repeat(e, 8), rng.integers(0, P, 30000, dtype=np.uint32)])
    ex = rng.integers(0, 1 << 32, base.size, dtype=np.uint64).astype(np.uint32)
    ex[: 8 * e.size] = np.tile(np.array([0, 1, 2, 3, 0xFFFFFFFF, 0xAAAAAAAA, 0x55555555, P - 1], dtype=np.uint64)
                               .astype(np.uint32), e.size)
    assert np.array_equal(host(M.pow(prm, dev(base), dev(ex))), oracle.mont_pow(P, base, ex))


@pytest.mark.parametrize("P", MODULI)
def test_fused_modmul_ordinary_values(M, P):
    """mont_modmul: a*b mod P of ordinary uint32 values (not reduced, not
    residues) in one pass, against the plain product."""
    prm = M.setup(P)
    rng = np.random.default_rng(P % 8191)
    x = rng.integers(0, 1 << 32, 60001, dtype=np.uint64).astype(np.uint32)
    y = rng.integers(0, 1 << 32, 60001, dtype=np.uint64).astype(np.uint32)
    ed = np.array([0, 1, P - 1, P, P + 1, 0xFFFFFFFF, 1 << 31, (1 << 31) - 1], dtype=np.uint64).astype(np.uint32)
    x = np.concatenate([np.repeat(ed, ed.size), x])
    y = np.concatenate([np.tile(ed, ed.size), y])
    want = oracle.modmul(P, x, y)
    assert np.array_equal(host(M.modmul(prm, dev(x), dev(y))), want)
    for off, n in ((1, 1), (1, 1001), (3, 4099), (0, 7)):           # misaligned views and ragged tails
        assert np.array_equal(host(M.modmul(prm, dev(x)[off:off + n], dev(y)[off:off + n])), want[off:off + n])
    dx = dev(x)
    M.modmul(prm, dx, dev(y), out=dx)                             # in place
    assert np.array_equal(host(dx), want)


def test_fused_modmul_pipeline_config(M):
    """The plain pipeline config (2^20 pairs, P = 15*2^27+1) through the fused
    call equals the to / mul / from path and the plain product."""
    P = wl.P_PLAIN
    prm = M.setup(P)
    a, b = wl.plain_pairs()
    da, db = dev(a), dev(b)
    fused = host(M.modmul(prm, da, db))
    staged = host(M.from_mont(prm, M.mul(prm, M.to_mont(prm, da), M.to_mont(prm, db))))
    assert np.array_equal(fused, staged)
    assert np.array_equal(fused, ((a.astype(np.uint64) * b) % P).astype(np.uint32))
