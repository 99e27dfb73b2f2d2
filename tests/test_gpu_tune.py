"""Every launch shape the autotuner may pick gives the oracle's results."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1609_00999_amd import mont, ntt, tune
    return mont, ntt, tune


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint32)


def test_elementwise_shapes(mods):
    mont, _, tune = mods
    P = wl.PRIMES_BW[3]
    prm = mont.setup(P)
    rng = np.random.default_rng(4)
    n = 3 * 4096 * 4 + 7                        # several tiles of every shape and a ragged tail
    a, b, c = (rng.integers(0, P, n, dtype=np.uint32) for _ in range(3))
    da, db, dc = dev(a), dev(b), dev(c)
    refs = {"to": oracle.to_mont(P, a), "from": oracle.from_mont(P, a), "mul": oracle.mont_mul(P, a, b),
            "muladd": oracle.mont_muladd(P, a, b, c), "pow": oracle.mont_pow(P, a, b)}
    calls = {"to": lambda: mont.to_mont(prm, da), "from": lambda: mont.from_mont(prm, da),
             "mul": lambda: mont.mul(prm, da, db), "muladd": lambda: mont.muladd(prm, da, db, dc),
             "pow": lambda: mont.pow(prm, da, db)}
    for op in calls:
        old = mont.elem_tune_get(op)
        try:
            for shape in tune.ELEM_SHAPES:
                mont.elem_tune_set(op, *shape)
                assert np.array_equal(host(calls[op]()), refs[op]), (op, shape)
        finally:
            mont.elem_tune_set(op, *old)


def test_transform_shapes(mods):
    mont, ntt, tune = mods
    ctx = ntt.Context(wl.PRIMES_NTT, 23)
    rng = np.random.default_rng(5)
    batch = wl.pack_products(wl.PRIMES_NTT, rng.integers(0, 8, 40), wl.log_uniform(rng, 0, 17, 40),
                             wl.log_uniform(rng, 0, 17, 40), rng)
    ref = np.concatenate(oracle.polymul_many([batch.operands(i) for i in range(batch.count)]))
    din = dev(batch.coeffs)
    old = ntt.tune_get()
    try:
        for threads, radix in tune.NTT_SHAPES:
            for gm in tune.GRID_MULTS:
                ntt.tune_set(threads, radix, gm)
                plan = ntt.Plan.from_batch(ctx, batch)
                out = torch.zeros(batch.out_len, dtype=torch.int32, device="cuda")
                scr = plan.alloc_scratch()
                plan.execute(din, out, scr)
                assert plan.status(scr) == 0
                assert np.array_equal(host(out), ref), (threads, radix, gm)
                plan.close()
            for logn in (3, 13, 16):
                P = wl.PRIMES_NTT[logn % 8]
                x = rng.integers(0, P, 1 << logn, dtype=np.uint32)
                dx = dev(x)
                ntt.forward(ctx, logn % 8, dx)
                w = pow(oracle.primitive_root(P), (P - 1) >> logn, P)
                r = np.zeros(1 << logn, dtype=np.int64)
                for bit in range(logn):
                    r |= ((np.arange(1 << logn) >> bit) & 1) << (logn - 1 - bit)
                assert np.array_equal(host(dx), oracle.ntt(P, x, w)[r]), (threads, radix, logn)
                ntt.inverse(ctx, logn % 8, dx)
                assert np.array_equal(host(dx), x)
    finally:
        ntt.tune_set(*old)
        ctx.close()


def test_per_length_shapes_keep_results(mods):
    """Different launch shapes for different transform lengths (plain
    launches by their length, a plan by its dominant length) leave every
    product exact."""
    mont, ntt, tune = mods
    ctx = ntt.Context(wl.PRIMES_NTT, 23)
    rng = np.random.default_rng(6)
    batch = wl.pack_products(wl.PRIMES_NTT, rng.integers(0, 8, 30), wl.log_uniform(rng, 0, 19, 30),
                             wl.log_uniform(rng, 0, 19, 30), rng)
    ref = np.concatenate(oracle.polymul_many([batch.operands(i) for i in range(batch.count)]))
    din = dev(batch.coeffs)
    saved = [ntt.tune_get_length(n) for n in range(24)]
    try:
        shapes = [(256, 3, 1), (1024, 4, 2), (512, 3, 1), (256, 4, 2), (1024, 3, 1), (512, 4, 2)]
        for rep in range(3):
            for n in range(24):
                ntt.tune_set_length(n, *shapes[(n + rep) % len(shapes)])
            plan = ntt.Plan.from_batch(ctx, batch)
            out = torch.zeros(batch.out_len, dtype=torch.int32, device="cuda")
            scr = plan.alloc_scratch()
            plan.execute(din, out, scr)
            assert plan.status(scr) == 0
            assert np.array_equal(host(out), ref), rep
            plan.close()
            for i in (0, batch.count // 2, batch.count - 1):
                P, a, b = batch.operands(i)
                got = host(ntt.polymul(ctx, wl.PRIMES_NTT.index(P), dev(a), dev(b)))
                assert np.array_equal(got, oracle.polymul(P, a, b)), (rep, i)
    finally:
        for n in range(24):
            ntt.tune_set_length(n, 0)
        for n, sh in enumerate(saved):
            if sh != ntt.tune_get():
                ntt.tune_set_length(n, *sh)
        ctx.close()


def test_plan_shape_follows_dominant_length(mods):
    """A plan with at least 90 % of its butterflies at one transform length
    takes that length's launch shape, any other plan the default shape
    (ntt_plan_shape), for created and for reserved plans alike; both give
    the oracle's products."""
    _, ntt, _ = mods
    ctx = ntt.Context(wl.PRIMES_NTT, 23)
    rng = np.random.default_rng(12)
    old = ntt.tune_get()
    saved = [ntt.tune_get_length(n) for n in range(24)]
    reserved = ntt.Plan.reserve(ctx, 16, 1 << 14)
    try:
        for n in range(24):
            ntt.tune_set_length(n, 0)
        ntt.tune_set(512, 4, 1)
        ntt.tune_set_length(16, 1024, 3, 2)
        # degrees 30000 .. 32000: products of length 2^16, none split
        one = wl.pack_products(wl.PRIMES_NTT, rng.integers(0, 8, 6), rng.integers(30000, 32000, 6),
                               rng.integers(30000, 32000, 6), rng)
        # lengths 2^11 .. 2^17, none with 90 % of the work
        mixed = wl.pack_products(wl.PRIMES_NTT, rng.integers(0, 8, 4), [1000, 8000, 30000, 60000],
                                 [1000, 8000, 30000, 60000], rng)
        for batch, want in ((one, (1024, 3, 2)), (mixed, (512, 4, 1))):
            ref = np.concatenate(oracle.polymul_many([batch.operands(i) for i in range(batch.count)]))
            desc = ntt.make_descs(batch.prime_id, batch.da, batch.db, batch.a_off, batch.b_off, batch.c_off)
            reserved.update(desc)
            for plan in (ntt.Plan.from_batch(ctx, batch), reserved):
                assert plan.shape() == want
                out = torch.zeros(batch.out_len, dtype=torch.int32, device="cuda")
                scr = plan.alloc_scratch()
                plan.execute(dev(batch.coeffs), out, scr)
                assert plan.status(scr) == 0
                assert np.array_equal(host(out), ref), want
                if plan is not reserved:
                    plan.close()
    finally:
        reserved.close()
        ntt.tune_set(*old)
        for n in range(24):
            ntt.tune_set_length(n, 0)
        for n, sh in enumerate(saved):
            if sh != ntt.tune_get():
                ntt.tune_set_length(n, *sh)
        ctx.close()
