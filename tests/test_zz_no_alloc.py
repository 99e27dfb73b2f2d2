"""ntt_polymul_noalloc, the allocation-free product (static device scratch),
through the C ABI: bit-exact against ntt_polymul (the entry point it is a
variant of) and the oracle, on calls in a row whose second input is
smaller, and its size limit."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRIMES = wl.PRIMES_NTT


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1609_00999_amd import mont, ntt
    ctx = ntt.Context(PRIMES, 23)
    yield mont, ntt, ctx
    ctx.close()


def test_noalloc_matches_polymul_on_calls_in_a_row(env):
    mont, ntt, ctx = env
    rng = np.random.default_rng(4242)
    # the longest product the static scratch holds (N = 2^21), then smaller
    # ones: a two-pass product, a one-workgroup product, a split-length one
    shapes = [((1 << 20) - 1, (1 << 20) - 1), (40000, 30001), (3000, 2000), (8200, 8200)]
    for i, (da, db) in enumerate(shapes):
        pid = i % len(PRIMES)
        P = PRIMES[pid]
        a = rng.integers(0, P, da + 1, dtype=np.uint32)
        b = rng.integers(0, P, db + 1, dtype=np.uint32)
        ga, gb = dev(a), dev(b)
        out = torch.full((da + db + 1,), -1, dtype=torch.int32, device="cuda")
        ntt.polymul_noalloc(ctx, pid, ga, gb, out)
        want = ntt.polymul(ctx, pid, ga, gb)           # the existing entry point, caller scratch
        got = host(out)
        assert got.tobytes() == host(want).tobytes(), (da, db)
        assert np.array_equal(got, oracle.polymul(P, a, b)), (da, db)


def test_noalloc_limit_and_errors(env):
    mont, ntt, ctx = env
    x = dev(np.ones((1 << 20) + 1, dtype=np.uint32))
    out = torch.empty(2 * x.numel() - 1, dtype=torch.int32, device="cuda")
    with pytest.raises(mont.MontError) as ei:             # da + db + 1 = 2^21 + 1
        ntt.polymul_noalloc(ctx, 0, x, x, out)
    assert ei.value.status == -4
    y = dev(np.ones(8, dtype=np.uint32))
    with pytest.raises(mont.MontError) as ei:
        ntt.polymul_noalloc(ctx, 99, y, y, torch.empty(15, dtype=torch.int32, device="cuda"))
    assert ei.value.status == -1
