"""GPU parity of the batched elementwise launch, reusable plans and the
serving loop (bit-exact against the oracle; alone equals in the mix)."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRIMES = wl.PRIMES_NTT


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1609_00999_amd import mont, ntt, serve
    return mont, ntt, serve


@pytest.fixture(scope="module")
def ctx(mods):
    c = mods[1].Context(PRIMES, 23)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint32)


def test_vector_batch_uneven(mods):
    mont = mods[0]
    rng = np.random.default_rng(1)
    sizes = [0, 1, 3, 4095, 4096, 4097, 10000, 123457, 1 << 20, 5, 0, 70000]
    b = mont.Batch(len(sizes) + 4)
    items, refs = [], []
    for i, n in enumerate(sizes):
        P = (list(wl.PRIMES_BW) + list(PRIMES))[i % 12]
        prm = mont.setup(P)
        a = rng.integers(0, P, n + 1, dtype=np.uint32)
        c = rng.integers(0, P, n + 1, dtype=np.uint32)
        off = i % 2                      # odd vectors start 4 bytes in: not 16-byte aligned
        da, dc = dev(a)[off:off + n], dev(c)[off:off + n]
        out = torch.empty(n + 1, dtype=torch.int32, device="cuda")[off:off + n]
        items.append((prm, da, dc, out))
        refs.append(oracle.mont_mul(P, a[off:off + n], c[off:off + n]))
    b.update(items)
    b.mul()
    for (prm, _, _, out), ref in zip(items, refs):
        assert np.array_equal(host(out), ref)
    # a second, smaller batch through the same object
    b.update(items[3:6])
    for _, _, _, out in items[3:6]:
        out.zero_()
    b.mul()
    for (prm, _, _, out), ref in zip(items[3:6], refs[3:6]):
        assert np.array_equal(host(out), ref)
    b.close()


def test_vector_batch_uploaded_uneven_and_misaligned(mods):
    """Above 16 vectors the descriptors are uploaded and a workgroup takes two
    adjacent tiles: pairs that straddle two vectors, partial last tiles,
    empty vectors, vectors not 16-byte aligned (offsets of 1-3 words) and an
    odd tile count, against the oracle."""
    mont = mods[0]
    rng = np.random.default_rng(11)
    base = [0, 1, 3, 4095, 4096, 4097, 8192, 10000, 123457, 1 << 20, 5, 0, 70000, 12288, 3 * 4096 + 1, 2]
    sizes = base + base[::-1] + [4096]
    assert sum((n + 4095) // 4096 for n in sizes) % 2 == 1
    b = mont.Batch(len(sizes))
    items, refs = [], []
    for i, n in enumerate(sizes):
        P = (list(wl.PRIMES_BW) + list(PRIMES))[i % 12]
        prm = mont.setup(P)
        a = rng.integers(0, P, n + 3, dtype=np.uint32)
        c = rng.integers(0, P, n + 3, dtype=np.uint32)
        off = (i * 3) % 4
        da, dc = dev(a)[off:off + n], dev(c)[off:off + n]
        out = torch.empty(n + 3, dtype=torch.int32, device="cuda")[off:off + n]
        items.append((prm, da, dc, out))
        refs.append(oracle.mont_mul(P, a[off:off + n], c[off:off + n]))
    b.update(items)
    b.mul()
    for i, ((_, _, _, out), ref) in enumerate(zip(items, refs)):
        assert np.array_equal(host(out), ref), (i, sizes[i])
    b.close()


def test_vector_batch_large_and_small_in_turn(mods):
    """Batches above 16 vectors upload their descriptors; smaller ones pass
    them in the launch.  One object alternates between the two."""
    mont = mods[0]
    rng = np.random.default_rng(7)
    sizes = [int(x) for x in rng.integers(0, 20000, 40)] + [0, 1, 4096, 70000]
    b = mont.Batch(len(sizes))
    items, refs = [], []
    for i, n in enumerate(sizes):
        P = PRIMES[i % len(PRIMES)]
        prm = mont.setup(P)
        a = rng.integers(0, P, n, dtype=np.uint32)
        c = rng.integers(0, P, n, dtype=np.uint32)
        out = torch.empty(max(1, n), dtype=torch.int32, device="cuda")[:n]
        items.append((prm, dev(a), dev(c), out))
        refs.append(oracle.mont_mul(P, a, c))
    for sel in (slice(0, 44), slice(40, 43), slice(3, 44), slice(41, 42), slice(0, 17), slice(0, 16)):
        for _, _, _, out in items[sel]:
            out.zero_()
        b.update(items[sel])
        b.mul()
        for (_, _, _, out), ref in zip(items[sel], refs[sel]):
            assert np.array_equal(host(out), ref), sel
    b.close()


def test_vector_batch_errors(mods):
    mont = mods[0]
    b = mont.Batch(2)
    x = torch.zeros(8, dtype=torch.int32, device="cuda")
    prm = mont.setup(PRIMES[0])
    with pytest.raises(mont.MontError) as ei:
        b.update([(prm, x, x, x)] * 3)
    assert ei.value.status == -2
    bad = mont.MontParams(P=PRIMES[0], Pprime=7, R1=0, R2=0, k=0)
    with pytest.raises(mont.MontError) as ei:
        b.update([(bad, x, x, x)])
    assert ei.value.status == -1
    b.close()


def test_reserved_plan_updates(mods, ctx):
    ntt = mods[1]
    rng = np.random.default_rng(2)
    plan = ntt.Plan.reserve(ctx, 64, 1 << 16)
    # batches of at most 4 products (and no split ones) travel in the launch
    # arguments, larger ones are uploaded: alternate between the two
    shapes = [(2, 16, 40), (12, 16, 3), (10, 18, 12), (13, 14, 1), (0, 6, 64), (8, 12, 4), (14, 17, 2)]
    for rep, (lo, hi, count) in enumerate(shapes):
        da = wl.log_uniform(rng, lo, hi, count)
        pid = rng.integers(0, len(PRIMES), count)
        batch = wl.pack_products(PRIMES, pid, da, da, rng)
        desc = ntt.make_descs(batch.prime_id, batch.da, batch.db, batch.a_off, batch.b_off, batch.c_off)
        plan.update(desc, order_seed=rep)
        din = dev(batch.coeffs)
        out = torch.zeros(batch.out_len, dtype=torch.int32, device="cuda")
        scr = plan.alloc_scratch()
        plan.execute(din, out, scr)
        assert plan.status(scr) == 0
        got = host(out)
        for i in range(batch.count):
            P, a, b = batch.operands(i)
            ref = oracle.polymul(P, a, b)
            assert np.array_equal(got[batch.c_off[i]: batch.c_off[i] + ref.size], ref), (rep, i)
    big = np.zeros(65, dtype=ntt.DESC_DTYPE)
    with pytest.raises(Exception):
        plan.update(big)
    plan.close()


def serve_setup(mods, ctx, count=48, seed=11):
    serve = mods[2]
    reqs = wl.request_stream(count, 1e6, seed=seed, mul_log2=(4, 17), poly_log2=(3, 15))
    for r in reqs:
        r.t_arrival = 0.0
    inputs = serve.DeviceInputs(reqs, PRIMES)
    return serve, reqs, inputs


def oracle_result(inputs, r):
    P = PRIMES[r.prime_id]
    a, b = inputs.host_operands(r.rid)
    return oracle.mont_mul(P, a, b) if r.kind == "mul" else oracle.polymul(P, a, b)


def test_serving_batches_exact_and_alone_equals_mix(mods, ctx):
    serve, reqs, inputs = serve_setup(mods, ctx)
    ex = serve.GpuBatchExecutor(ctx, inputs, slots=3, max_batch=16)
    stats = serve.Scheduler(ex, slots=3, budget_bytes=1 << 30, max_batch=16).run(serve.jobs_from_requests(reqs))
    assert all(j.status == serve.OK for j in stats.jobs)
    assert stats.batches < len(reqs)
    mix = {j.rid: host(j.result) for j in stats.jobs}
    for r in reqs:
        assert np.array_equal(mix[r.rid], oracle_result(inputs, r)), r.rid
    # every request alone through the same executor gives the same bytes (a
    # one-product batch takes the plain launches, a mixed one the persistent
    # launch)
    for r in reqs[::5]:
        st = serve.Scheduler(ex, slots=3, budget_bytes=1 << 30).run(serve.jobs_from_requests([r]))
        assert st.jobs[0].status == serve.OK
        assert host(st.jobs[0].result).tobytes() == mix[r.rid].tobytes()
    # the per-request plain-launch baseline agrees too
    plain = serve.GpuPlainExecutor(ctx, inputs)
    st = serve.Scheduler(plain, slots=1, budget_bytes=1 << 30, max_batch=1).run(serve.jobs_from_requests(reqs))
    for j in st.jobs:
        assert host(j.result).tobytes() == mix[j.rid].tobytes()
    ex.close()


def test_serving_under_tight_budget(mods, ctx):
    serve, reqs, inputs = serve_setup(mods, ctx, count=30, seed=12)
    ex = serve.GpuBatchExecutor(ctx, inputs, slots=2, max_batch=8)
    fps = [ex.footprint(j) for j in serve.jobs_from_requests(reqs)]
    budget = 2 * max(fps)
    stats = serve.Scheduler(ex, slots=2, budget_bytes=budget, max_batch=8).run(serve.jobs_from_requests(reqs))
    assert stats.max_inflight_bytes <= budget
    assert all(j.status == serve.OK for j in stats.jobs)
    for j in stats.jobs:
        r = reqs[j.rid]
        assert np.array_equal(host(j.result), oracle_result(inputs, r))
    ex.close()


def test_serving_arena_fallback_and_kept_set(mods, ctx):
    """Batches carve outputs and scratch from per-slot arenas; a batch that
    does not fit falls back to torch allocations, and results kept for a set
    of requests are copied out of the arena before the slot is reused."""
    serve, reqs, inputs = serve_setup(mods, ctx, count=40, seed=13)
    # arenas too small for any batch: every batch falls back
    ex = serve.GpuBatchExecutor(ctx, inputs, slots=2, max_batch=8, arena_bytes=4096)
    st = serve.Scheduler(ex, slots=2, budget_bytes=1 << 30, max_batch=8).run(serve.jobs_from_requests(reqs))
    assert ex.fallback_batches == st.batches > 0
    for j in st.jobs:
        assert np.array_equal(host(j.result), oracle_result(inputs, reqs[j.rid]))
    ex.close()
    # one slot, default arena, only some results kept: every kept result is
    # exact although later batches reused the arena
    keep = set(range(0, 40, 3))
    ex = serve.GpuBatchExecutor(ctx, inputs, slots=1, max_batch=4, keep_results=keep)
    st = serve.Scheduler(ex, slots=1, budget_bytes=1 << 30, max_batch=4).run(serve.jobs_from_requests(reqs))
    assert ex.fallback_batches == 0 and st.batches >= 10
    summary = st.summary()
    assert summary["launch_ms_max"] >= summary["launch_ms_p50"] >= 0
    for j in st.jobs:
        if j.rid in keep:
            assert np.array_equal(host(j.result), oracle_result(inputs, reqs[j.rid])), j.rid
        else:
            assert j.result is None
    ex.close()


def test_serving_full_size_stream(mods, ctx):
    """The first 300 requests of the serving workload at its full sizes
    (elementwise n log-uniform in 2^10..2^24, polynomial degree in
    2^10..2^22, eight primes, Poisson arrivals at 20k requests/s, seed 5),
    served by the batching loop: every element of every result against the
    oracle, and the longest polynomial requests alone equal to the mix."""
    serve = mods[2]
    reqs = wl.request_stream(300, 20000.0, seed=wl.SEED_SERVE)
    assert max(r.size for r in reqs if r.kind == "polymul") > 1 << 21
    assert max(r.size for r in reqs if r.kind == "mul") > 1 << 23
    inputs = serve.DeviceInputs(reqs, PRIMES)
    for r in reqs:
        a0, b0, _ = inputs.offs[r.rid]
        assert a0 % 4 == 0 and b0 % 4 == 0          # both operands 16-byte aligned
    ex = serve.GpuBatchExecutor(ctx, inputs, slots=4, max_batch=64)
    stats = serve.Scheduler(ex, slots=4, budget_bytes=16 << 30, max_batch=64).run(serve.jobs_from_requests(reqs))
    assert all(j.status == serve.OK for j in stats.jobs)
    mix = {j.rid: host(j.result) for j in stats.jobs}
    from concurrent.futures import ThreadPoolExecutor

    def check(r):
        return -1 if np.array_equal(mix[r.rid], oracle_result(inputs, r)) else r.rid

    order = sorted(reqs, key=lambda r: -r.size if r.kind == "polymul" else 0)
    with ThreadPoolExecutor(oracle.default_threads()) as pool:
        bad = [rid for rid in pool.map(check, order) if rid >= 0]
    assert not bad, bad[:10]
    longest = sorted((r for r in reqs if r.kind == "polymul"), key=lambda r: -r.size)[:3]
    st = serve.Scheduler(ex, slots=4, budget_bytes=16 << 30).run(serve.jobs_from_requests(longest))
    for j in st.jobs:
        assert j.status == serve.OK
        assert host(j.result).tobytes() == mix[j.rid].tobytes()
    ex.close()


def test_serving_executor_reports_device_timeouts(mods, ctx):
    """The batching executor with a one-sleep bound on the transform tasks'
    dependency waits: batches holding long products time out on the device
    (every kernel still exits), and exactly their polynomial requests come
    back FAILED with MONT_ETIMEOUT, while elementwise requests stay exact.
    The same executor then serves the stream exactly with the normal bound."""
    serve = mods[2]
    reqs = wl.request_stream(12, 1e6, seed=21, mul_log2=(10, 14), poly_log2=(17, 19))
    for r in reqs:
        r.t_arrival = 0.0
    inputs = serve.DeviceInputs(reqs, PRIMES)
    # every batch through the persistent launch (one-product batches would
    # otherwise take the plain launches, which have no dependency waits)
    ex = serve.GpuBatchExecutor(ctx, inputs, slots=2, max_batch=4, spin_limit=1, single_plain=False)
    st = serve.Scheduler(ex, slots=2, budget_bytes=1 << 32, max_batch=4).run(serve.jobs_from_requests(reqs))
    failed = [j for j in st.jobs if j.status == serve.FAILED]
    assert failed, "long products with a one-sleep wait bound should time out"
    for j in st.jobs:
        if j.status == serve.FAILED:
            assert j.kind == "polymul" and "MONT_ETIMEOUT" in j.error and j.result is None
        else:
            assert j.status == serve.OK
            assert np.array_equal(host(j.result), oracle_result(inputs, reqs[j.rid])), j.rid
    assert all(j.status == serve.OK for j in st.jobs if j.kind == "mul")
    ex.spin_limit = 0
    st = serve.Scheduler(ex, slots=2, budget_bytes=1 << 32, max_batch=4).run(serve.jobs_from_requests(reqs))
    assert all(j.status == serve.OK for j in st.jobs)
    for j in st.jobs:
        assert np.array_equal(host(j.result), oracle_result(inputs, reqs[j.rid])), j.rid
    ex.close()
