"""GPU parity of the exact integer polynomial products (three NTT primes and
Garner's reconstruction) against exact integer convolution and the CPU oracle;
all comparisons are bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRIMES3 = wl.PRIMES_NTT[:3]
MAXC = (1 << 32) - 1


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1609_00999_amd import crt, ntt
    ctx = ntt.Context(wl.PRIMES_NTT, 23)
    prm = crt.setup(PRIMES3)
    yield crt, ntt, ctx, prm
    ctx.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint32).view(np.int32)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint32)


def exact_conv(a, b):
    """Integer convolution in Python integers (small sizes)."""
    return np.convolve(np.asarray(a, dtype=object), np.asarray(b, dtype=object)).tolist()


def oracle_exact(a, b):
    """The oracle's products modulo each prime, joined by the oracle's CRT."""
    res = [oracle.polymul(P, a % np.uint32(P), b % np.uint32(P)) for P in PRIMES3]
    return oracle.crt(PRIMES3, np.stack(res), 3)


def test_reduce_and_combine(env):
    crt, _, _, prm = env
    rng = np.random.default_rng(1)
    x = np.concatenate([np.array([0, 1, MAXC, MAXC - 1, 1 << 31, (1 << 30) + 1] + list(PRIMES3) +
                                 [2 * p for p in PRIMES3] + [3 * p - 1 for p in PRIMES3[:1]], dtype=np.uint64)
                        .astype(np.uint32), rng.integers(0, 1 << 32, 100003, dtype=np.uint64).astype(np.uint32)])
    r = host(crt.reduce(prm, dev(x))).reshape(3, -1)
    for j, P in enumerate(PRIMES3):
        assert np.array_equal(r[j], (x.astype(np.uint64) % P).astype(np.uint32))
    # combine: random residue triples plus the extremes
    res = np.stack([rng.integers(0, P, 50001, dtype=np.uint32) for P in PRIMES3])
    res[:, 0] = 0
    res[:, 1] = [P - 1 for P in PRIMES3]
    out = host(crt.combine(prm, dev(res[0]), dev(res[1]), dev(res[2]))).reshape(-1, 3)
    assert np.array_equal(out, oracle.crt(PRIMES3, res, 3))
    M = PRIMES3[0] * PRIMES3[1] * PRIMES3[2]
    assert crt.limbs_to_int(out[1:2])[0] == M - 1


@pytest.mark.parametrize("da,db", [(0, 0), (1, 0), (7, 5), (100, 37), (300, 300), (1000, 3), (4095, 4096)])
def test_small_exact(env, da, db):
    crt, _, ctx, prm = env
    rng = np.random.default_rng(da * 131 + db)
    a = rng.integers(0, 1 << 32, da + 1, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << 32, db + 1, dtype=np.uint64).astype(np.uint32)
    a[0] = MAXC
    out = host(crt.polymul(ctx, prm, dev(a), dev(b))).reshape(-1, 3)
    want = exact_conv(a, b) if (da + 1) * (db + 1) <= 400000 else None
    if want is not None:
        assert crt.limbs_to_int(out) == want
    assert np.array_equal(out, oracle_exact(a, b))


@pytest.mark.parametrize("d", [(1 << 13) + 5, (1 << 16) - 1, (1 << 19) + 77])
def test_two_pass_lengths(env, d):
    """Lengths that take the column/row passes: against the oracle's CRT of
    its modular products."""
    crt, _, ctx, prm = env
    rng = np.random.default_rng(d)
    a = rng.integers(0, 1 << 32, d + 1, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 1 << 32, d // 3 + 1, dtype=np.uint64).astype(np.uint32)
    out = host(crt.polymul(ctx, prm, dev(a), dev(b))).reshape(-1, 3)
    assert np.array_equal(out, oracle_exact(a, b))


def test_all_max_coefficients_closed_form(env):
    """a = b = all (2^32 - 1), degree 2^21 - 1: c_k = (min(k, 2d-k) + 1) (2^32 - 1)^2,
    up to 2^21 (2^32-1)^2 ~ 2^85: the largest values the three primes must hold here."""
    crt, _, ctx, prm = env
    d = (1 << 21) - 1
    a = np.full(d + 1, MAXC, dtype=np.uint32)
    out = host(crt.polymul(ctx, prm, dev(a), dev(a))).reshape(-1, 3)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.arange(64), np.arange(2 * d - 63, 2 * d + 1), [d - 1, d, d + 1],
                                    rng.integers(0, 2 * d + 1, 4000)]))
    got = crt.limbs_to_int(out[idx])
    want = [(min(int(k), 2 * d - int(k)) + 1) * MAXC * MAXC for k in idx]
    assert got == want


def test_batch_matches_single_and_oracle(env):
    """A packed batch of uneven integer products in one persistent launch."""
    crt, _, ctx, prm = env
    batch = wl.int_products(count=48, lo_log2=4, hi_log2=16, seed=11)
    cb = crt.Batch.from_batch(ctx, prm, batch)
    work = cb.buffers()
    out = torch.empty((batch.out_len, 3), dtype=torch.int32, device="cuda")
    cb.run(dev(batch.coeffs), out, work)
    got = host(out).reshape(-1, 3)
    for i in range(batch.count):
        _, a, b = batch.operands(i)
        c0 = int(batch.c_off[i])
        part = got[c0: c0 + a.size + b.size - 1]
        assert np.array_equal(part, oracle_exact(a, b)), "product %d" % i
    # a second run on the same buffers gives the same bytes
    out2 = torch.empty_like(out)
    cb.run(dev(batch.coeffs), out2, work, grid=7)
    assert torch.equal(out, out2)
    cb.close()


def test_batch_run_reports_a_timeout(env):
    """A one-sleep wait limit on the modular products' launch: the waits of
    long products give up (every kernel still exits), run() raises
    MONT_ETIMEOUT, and the next run on the same buffers is exact."""
    crt, _, ctx, prm = env
    from paper_1609_00999_amd import mont
    batch = wl.int_products(count=6, lo_log2=17, hi_log2=18, seed=12)
    cb = crt.Batch.from_batch(ctx, prm, batch)
    work = cb.buffers()
    out = torch.empty((batch.out_len, 3), dtype=torch.int32, device="cuda")
    din = dev(batch.coeffs)
    with pytest.raises(mont.MontError) as ei:
        cb.run(din, out, work, spin_limit=1)
    assert ei.value.status == -6
    cb.run(din, out, work)
    assert cb.status(work) == 0
    got = host(out).reshape(-1, 3)
    for i in (0, batch.count - 1):
        _, a, b = batch.operands(i)
        c0 = int(batch.c_off[i])
        assert np.array_equal(got[c0: c0 + a.size + b.size - 1], oracle_exact(a, b)), i
    cb.close()


def test_errors(env):
    crt, ntt, ctx, prm = env
    from paper_1609_00999_amd import mont
    a = dev(np.ones(10, dtype=np.uint32))
    other = crt.setup(wl.PRIMES_NTT[3:6])
    other.P[0] = wl.PRIMES_NTT[0]            # constants no longer match the primes
    with pytest.raises(mont.MontError):
        crt.polymul(ctx, other, a, a)
    small = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(mont.MontError):
        crt.polymul(ctx, prm, a, a, scratch=small)
