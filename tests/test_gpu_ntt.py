"""GPU parity of the transforms, single polynomial products and the persistent
batch against the CPU oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import workloads as wl
from test_unit_twiddles import unit_twiddle_butterflies

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRIMES = wl.PRIMES_NTT


@pytest.fixture(scope="module")
def N():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1609_00999_amd import ntt
    return ntt


@pytest.fixture(scope="module")
def ctx(N):
    c = N.Context(PRIMES, 23)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to("cuda")


def host(t):
    return t.cpu().numpy().view(np.uint32)


def bitrev(n_log2):
    n = 1 << n_log2
    r = np.zeros(n, dtype=np.int64)
    for b in range(n_log2):
        r |= ((np.arange(n) >> b) & 1) << (n_log2 - 1 - b)
    return r


def test_context_roots_and_tables(ctx):
    for pid, P in enumerate(PRIMES):
        prm, root, lmax, _, _ = ctx.prime(pid)
        ref = oracle.setup(P)
        assert (prm.P, prm.Pprime, prm.R1, prm.R2) == (P, ref.Pprime, ref.R1, ref.R2)
        assert lmax == 23
        g = oracle.primitive_root(P)
        assert root == pow(g, (P - 1) >> lmax, P)
        assert pow(root, 1 << lmax, P) == 1 and pow(root, 1 << (lmax - 1), P) == P - 1
        f, iv = ctx.twiddles(pid)
        rng = np.random.default_rng(pid)
        xs = np.unique(np.concatenate([np.arange(1, 70), rng.integers(1, 1 << lmax, 3000),
                                       (1 << np.arange(lmax)), (1 << np.arange(1, lmax)) - 1]))
        R = 1 << 32
        for x in xs.tolist():
            s = x.bit_length() - 1
            i = x - (1 << s)
            e = i << (lmax - 1 - s)
            assert int(f[x]) == pow(root, e, P) * R % P, (pid, x)
            assert int(iv[x]) == pow(root, (1 << lmax) - e, P) * R % P, (pid, x)


@pytest.mark.parametrize("logn", [0, 1, 2, 5, 10, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23])
def test_forward_inverse_vs_oracle(N, ctx, logn):
    pid = logn % len(PRIMES)
    P = PRIMES[pid]
    n = 1 << logn
    rng = np.random.default_rng(logn)
    x = rng.integers(0, P, n, dtype=np.uint32)
    dx = dev(x)
    N.forward(ctx, pid, dx)
    got = host(dx)
    g = oracle.primitive_root(P)
    w = pow(g, (P - 1) >> logn, P)
    want = oracle.ntt(P, x, w)                 # natural order
    assert np.array_equal(got, want[bitrev(logn)])
    N.inverse(ctx, pid, dx)
    assert np.array_equal(host(dx), x)
    # inverse alone vs the oracle's transform with w^-1 and N^-1
    y = rng.integers(0, P, n, dtype=np.uint32)
    dy = dev(y)
    N.inverse(ctx, pid, dy)
    inv = oracle.ntt(P, y[bitrev(logn)], pow(w, P - 2, P)).astype(np.uint64)
    inv = (inv * np.uint64(pow(n, P - 2, P))) % np.uint64(P)
    assert np.array_equal(host(dy), inv.astype(np.uint32))


SHAPES = [(0, 0), (0, 7), (5, 0), (1, 1), (255, 256), (2047, 2048), (4095, 4096), (4096, 4095),
          (8191, 0), (4096, 4096), (6000, 2191), (8191, 8191), (12345, 54321), (65535, 65536), (100000, 3)]


@pytest.mark.parametrize("da,db", SHAPES)
def test_polymul_vs_oracle(N, ctx, da, db):
    pid = (da + 3 * db) % len(PRIMES)
    P = PRIMES[pid]
    rng = np.random.default_rng(da * 7 + db)
    a = rng.integers(0, P, da + 1, dtype=np.uint32)
    b = rng.integers(0, P, db + 1, dtype=np.uint32)
    got = host(N.polymul(ctx, pid, dev(a), dev(b)))
    assert np.array_equal(got, oracle.polymul(P, a, b))


def test_polymul_golden(N, ctx):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "polymul_small.txt")
    for ln in open(path):
        if ln.startswith("#") or not ln.strip():
            continue
        v = [int(x) for x in ln.split()]
        P, da, db = v[:3]
        a = np.array(v[3:4 + da], dtype=np.uint32)
        b = np.array(v[4 + da:5 + da + db], dtype=np.uint32)
        c = np.array(v[5 + da + db:], dtype=np.uint32)
        got = host(N.polymul(ctx, PRIMES.index(P), dev(a), dev(b)))
        assert np.array_equal(got, c)


def test_polymul_special_cases(N, ctx):
    import math
    P = PRIMES[4]
    d = 20000
    rng = np.random.default_rng(3)
    b = rng.integers(0, P, d + 1, dtype=np.uint32)
    one = np.array([1], dtype=np.uint32)
    assert np.array_equal(host(N.polymul(ctx, 4, dev(one), dev(b))), b)
    xk = np.zeros(1001, dtype=np.uint32)
    xk[1000] = 1
    c = host(N.polymul(ctx, 4, dev(xk), dev(b)))
    assert np.all(c[:1000] == 0) and np.array_equal(c[1000:], b)
    ones = np.ones(d + 1, dtype=np.uint32)
    kk = np.arange(2 * d + 1)
    assert np.array_equal(host(N.polymul(ctx, 4, dev(ones), dev(ones))),
                          (np.minimum(kk, 2 * d - kk) + 1).astype(np.uint32))
    dd = 3000
    binom = np.array([math.comb(dd, k) % P for k in range(dd + 1)], dtype=np.uint32)
    got = host(N.polymul(ctx, 4, dev(binom), dev(binom)))
    assert got.tolist() == [math.comb(2 * dd, k) % P for k in range(2 * dd + 1)]


@pytest.mark.parametrize("da,db", [((1 << 22) - 1, (1 << 22) - 1), (1500000, 1500000), ((1 << 21) - 1, 1 << 20)])
def test_polymul_largest_length(N, ctx, da, db):
    """N = 2^23, the longest transform the tables support, and N = 2^22
    (column tiles of 32 columns): every coefficient against the oracle."""
    pid = 1
    P = PRIMES[pid]
    rng = np.random.default_rng(da + db)
    a = rng.integers(0, P, da + 1, dtype=np.uint32)
    b = rng.integers(0, P, db + 1, dtype=np.uint32)
    c = host(N.polymul(ctx, pid, dev(a), dev(b)))
    assert c.size == da + db + 1
    want = oracle.polymul(P, a, b)
    bad = np.flatnonzero(c != want)
    assert bad.size == 0, (bad.size, bad[:8].tolist())


def test_lengths_above_the_cap_are_refused(N, ctx):
    """Transforms are capped at 2^23: a product of length 2^23 + 1 and a
    2^24-point transform return MONT_ENOROOT (the tables end at 2^23), and no
    context holds longer tables."""
    from paper_1609_00999_amd import mont
    x = dev(np.ones((1 << 22) + 1, dtype=np.uint32))
    with pytest.raises(mont.MontError) as ei:
        N.polymul(ctx, 0, x, x)                    # da + db + 1 = 2^23 + 1
    assert ei.value.status == -3
    z = dev(np.zeros(1 << 24, dtype=np.uint32))
    with pytest.raises(mont.MontError) as ei:
        N.forward(ctx, 0, z)
    assert ei.value.status == -3
    with pytest.raises(mont.MontError) as ei:
        N.Context([2013265921], 24)                # v2(P - 1) = 27, but the cap is 23
    assert ei.value.status == -1


def test_polymul_errors(N, ctx):
    from paper_1609_00999_amd import mont
    P = PRIMES[0]
    a = dev(np.ones(10, dtype=np.uint32))
    with pytest.raises(mont.MontError):
        N.polymul(ctx, 99, a, a)
    # a prime whose 2-adic valuation is too small for the length
    small = N.Context([998244353, 469762049], 23)     # k = 23 and 26
    try:
        prm, _, lmax, _, _ = small.prime(0)
        assert lmax == 23
    finally:
        small.close()
    c2 = N.Context([2013265921], 12)
    try:
        x = dev(np.ones(1 << 13, dtype=np.uint32))
        with pytest.raises(mont.MontError) as ei:
            N.forward(c2, 0, x)
        assert ei.value.status == -3
        with pytest.raises(mont.MontError) as ei:
            N.polymul(c2, 0, x, x)
        assert ei.value.status == -3
    finally:
        c2.close()


def small_batch(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    da = wl.log_uniform(rng, lo, hi, count)
    db = np.maximum(0, da + rng.integers(-3, 4, count))
    pid = rng.integers(0, len(PRIMES), count)
    return wl.pack_products(PRIMES, pid, da, db, rng)


def run_plan(N, ctx, batch, grid=0, order_seed=0, spin_limit=0):
    plan = N.Plan.from_batch(ctx, batch, order_seed)
    din = dev(batch.coeffs)
    out = torch.zeros(max(1, batch.out_len), dtype=torch.int32, device="cuda")
    scr = plan.alloc_scratch()
    plan.execute(din, out, scr, grid=grid, spin_limit=spin_limit)
    st = plan.status(scr)
    res = host(out)
    plan.close()
    return st, res


def assert_batch_exact(batch, got):
    """Every coefficient of every product of the batch against the oracle,
    products spread over host threads (longest first)."""
    from concurrent.futures import ThreadPoolExecutor

    def check(i):
        P, a, b = batch.operands(i)
        c0 = int(batch.c_off[i])
        ref = oracle.polymul(P, a, b)
        return -1 if np.array_equal(got[c0:c0 + ref.size], ref) else i

    order = np.argsort(-(batch.da + batch.db), kind="stable")
    with ThreadPoolExecutor(oracle.default_threads()) as ex:
        bad = [i for i in ex.map(check, order.tolist()) if i >= 0]
    assert not bad, bad[:10]


def oracle_batch(batch):
    jobs = [batch.operands(i) for i in range(batch.count)]
    res = oracle.polymul_many(jobs)
    return np.concatenate(res)


def test_batch_vs_oracle(N, ctx):
    batch = small_batch(96, 0, 17, 41)
    st, got = run_plan(N, ctx, batch)
    assert st == 0
    assert np.array_equal(got, oracle_batch(batch))


def test_batch_grid_and_order_invariance(N, ctx):
    batch = small_batch(64, 4, 18, 42)
    ref = oracle_batch(batch)
    outs = []
    for grid, seed in [(0, 0), (1, 0), (3, 0), (0, 12345), (7, 999)]:
        st, got = run_plan(N, ctx, batch, grid=grid, order_seed=seed)
        assert st == 0
        outs.append(got)
        assert np.array_equal(got, ref), (grid, seed)
    for o in outs[1:]:
        assert o.tobytes() == outs[0].tobytes()


def test_batch_pipelined_order(N, ctx):
    """A batch with enough multi-pass products for the software-pipelined
    task order (smaller batches are ordered phase by phase): exact for several
    grids and shuffled orders within the pipeline's lists."""
    batch = small_batch(160, 13, 15, 43)
    assert int(np.sum(batch.da + batch.db + 1 > 8192)) >= 128
    ref = oracle_batch(batch)
    for grid, seed in [(0, 0), (3, 0), (0, 777)]:
        st, got = run_plan(N, ctx, batch, grid=grid, order_seed=seed)
        assert st == 0
        assert np.array_equal(got, ref), (grid, seed)


def test_batch_empty_and_tiny(N, ctx):
    b = wl.pack_products(PRIMES, [0], [0], [0], np.random.default_rng(0))
    st, got = run_plan(N, ctx, b)
    assert st == 0 and np.array_equal(got, oracle_batch(b))
    empty = N.Plan(ctx, [], [], [], [], [], [])
    assert empty.ntasks == 0
    empty.close()


def test_batch_timeout_path_drains(N, ctx):
    """A one-sleep wait limit: waits that do not finish at once record a
    timeout and the launch still drains; if no wait was needed the result is
    exact."""
    batch = small_batch(4, 17, 19, 43)
    ref = oracle_batch(batch)
    st, got = run_plan(N, ctx, batch, grid=0, spin_limit=1)
    assert st in (0, -6)
    if st == 0:
        assert np.array_equal(got, ref)
    # the next normal execution is exact again
    st, got = run_plan(N, ctx, batch)
    assert st == 0 and np.array_equal(got, ref)


def run_one_call(N, ctx, batch, scratch=None):
    """The batch through ntt_polymul_batch (descriptors planned on the device)."""
    descs = N.make_descs(batch.prime_id, batch.da, batch.db, batch.a_off, batch.b_off, batch.c_off)
    if scratch is None:
        scratch = torch.empty((N.batch_scratch_bytes(ctx, descs) + 3) // 4, dtype=torch.int32, device="cuda")
    out = torch.zeros(max(1, batch.out_len), dtype=torch.int32, device="cuda")
    N.polymul_batch(ctx, N.descs_to_device(descs), batch.count, dev(batch.coeffs), out, scratch)
    return N.batch_status(scratch), host(out)


def test_batch_config_full_size(N, ctx):
    """2048 products, degrees log-uniform in [2^8, 2^20), eight primes, one
    persistent launch: every coefficient of every product compared with the
    oracle (host threads over products); the one-call batch planned on the
    device gives the same bytes."""
    batch = wl.polymul_batch()
    plan = N.Plan.from_batch(ctx, batch)
    din = dev(batch.coeffs)
    out = torch.empty(batch.out_len, dtype=torch.int32, device="cuda")
    scr = plan.alloc_scratch()
    plan.execute(din, out, scr)
    assert plan.status(scr) == 0
    got = host(out)
    plan.close()
    del scr, din, out
    assert_batch_exact(batch, got)
    st, one = run_one_call(N, ctx, batch)
    assert st == 0
    assert one[:batch.out_len].tobytes() == got.tobytes()


def test_batch_longest_lengths(N, ctx):
    """One persistent launch holding unsplit products of transform lengths
    2^22 and 2^23 (the longest compile-time column tiles) beside short ones:
    every coefficient against the oracle."""
    # none of these is computed in two parts: each length lies above 3N/4
    # (no truncated-transform block) and its top product would be longer
    # than N/4 (no split)
    da = np.array([1600000, (1 << 22) - 1, (1 << 21) - 1, 3000, 120000, 14000], dtype=np.int64)
    db = np.array([1600000, (1 << 22) - 1, (1 << 20) + 10, 2000, 120000, 14100], dtype=np.int64)
    rng = np.random.default_rng(2223)
    pid = rng.integers(0, len(PRIMES), da.size)
    batch = wl.pack_products(PRIMES, pid, da, db, rng)
    plan = N.Plan.from_batch(ctx, batch)
    executed, nsplit = plan.work()
    plan.close()
    assert nsplit == 0
    st, got = run_plan(N, ctx, batch)
    assert st == 0
    assert_batch_exact(batch, got)


def test_batch_graph_replay(N, ctx):
    """The batch captured in a graph (fill kernel + persistent launch) gives the
    eager result on every replay, with eager work and synchronizations in
    between."""
    batch = small_batch(48, 6, 18, 44)
    ref = oracle_batch(batch)
    plan = N.Plan.from_batch(ctx, batch)
    din = dev(batch.coeffs)
    out = torch.zeros(batch.out_len, dtype=torch.int32, device="cuda")
    scr = plan.alloc_scratch()
    plan.execute(din, out, scr)
    assert plan.status(scr) == 0
    eager = host(out)
    assert np.array_equal(eager, ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(din, out, scr)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(din, out, scr)
    for r in range(4):
        out.zero_()
        scr.fill_(-1)                      # eager work that dirties the scratch header
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert plan.status(scr) == 0, r
        assert np.array_equal(host(out), eager), r
    del g
    plan.close()


@pytest.mark.parametrize("off", [1, 2, 3])
def test_polymul_misaligned_operands(N, ctx, off):
    """Operands that do not start on a 16-byte boundary take the element-load path."""
    P = PRIMES[off]
    rng = np.random.default_rng(100 + off)
    da, db = 9000 + off, 7000 - off
    a = rng.integers(0, P, da + 1 + off, dtype=np.uint32)
    b = rng.integers(0, P, db + 1 + off, dtype=np.uint32)
    out = torch.zeros(da + db + 1 + off, dtype=torch.int32, device="cuda")[off:]
    got = host(N.polymul(ctx, off, dev(a)[off:], dev(b)[off:], out=out))
    assert np.array_equal(got, oracle.polymul(P, a[off:], b[off:]))


def test_batch_unaligned_offsets(N, ctx):
    """A hand-packed batch whose operands sit at odd offsets."""
    rng = np.random.default_rng(46)
    da = np.array([5000, 20000, 3, 17000, 70000])
    db = np.array([6000, 19999, 9000, 2, 65000])
    pid = np.array([0, 3, 5, 7, 1])
    a_off, b_off, c_off, pos, cpos = [], [], [], 1, 0
    for x, y in zip(da, db):
        a_off.append(pos)
        pos += int(x) + 2
        b_off.append(pos)
        pos += int(y) + 1
        c_off.append(cpos)
        cpos += int(x + y + 1)
    coeffs = np.zeros(pos, dtype=np.uint32)
    for i in range(da.size):
        P = PRIMES[pid[i]]
        coeffs[a_off[i]: a_off[i] + da[i] + 1] = rng.integers(0, P, da[i] + 1, dtype=np.uint32)
        coeffs[b_off[i]: b_off[i] + db[i] + 1] = rng.integers(0, P, db[i] + 1, dtype=np.uint32)
    plan = N.Plan(ctx, pid, da, db, a_off, b_off, c_off)
    out = torch.zeros(cpos, dtype=torch.int32, device="cuda")
    scr = plan.alloc_scratch()
    plan.execute(dev(coeffs), out, scr)
    assert plan.status(scr) == 0
    got = host(out)
    for i in range(da.size):
        P = PRIMES[pid[i]]
        ref = oracle.polymul(P, coeffs[a_off[i]: a_off[i] + da[i] + 1], coeffs[b_off[i]: b_off[i] + db[i] + 1])
        assert np.array_equal(got[c_off[i]: c_off[i] + ref.size], ref), i


# Shapes around the split rule: a product of length L just above N/2 = h runs
# as its cyclic part of length h plus the product of the top m = L - h
# coefficients of each operand, joined by a fix-up kernel after the launch.
SPLIT_SHAPES = [(1, 1), (2, 1), (2, 2), (4, 4), (16, 16), (32, 31), (33, 30), (64, 64), (100, 60),
                (2048, 2048), (2049, 2047), (4096, 4096), (4100, 4100), (4097, 4095), (4095, 4097),
                (5000, 3300), (6000, 6000), (8192, 8192), (8200, 8200), (8191, 100), (16384, 10),
                (9000, 9100), (20000, 20000), (40000, 30000), (70000, 70000), (65600, 65400),
                ((1 << 19) + 3, (1 << 19) + 1), ((1 << 20) + 100, (1 << 20) - 100), (300000, 900)]

# Shapes the two-block truncated transform takes (N >= 2^18, both operands
# below h = N/2, N/16 < m = L - h <= N/4): block of N/8 points for m <= N/8,
# of N/4 above; unbalanced operands fold four terms.  Edges of each range.
TFT_SHAPES = [(75535, 75535), (81919, 65537), (73728, 73728), (90111, 90112), (98303, 98304),
              (131071, 32768), (700000, 700000), (1000000, 200000), (1048575, 262144), (600000, 600000),
              (4000000, 2000000), (3000000, 2000000), ((1 << 21) + 1, (1 << 21) + 1), (2621440, 2621440)]


def test_split_rule_is_used(N):
    """The plan splits products just above a power of two (fewer tasks than
    the plain two-pass product) and leaves the others whole."""
    assert N.task_count(4100, 4100) == 2            # 2^13 cyclic + a 32-point top product
    assert N.task_count(20000, 20000) < 3 * 4 + 8   # below the unsplit 2^16 product's 3 ntiles + nblocks
    assert N.task_count(6000, 6000) == N.task_count(8191, 8191)   # m too large to pay: unsplit


def test_batch_split_shapes_vs_oracle(N, ctx):
    rng = np.random.default_rng(77)
    da = [s[0] for s in SPLIT_SHAPES]
    db = [s[1] for s in SPLIT_SHAPES]
    pid = rng.integers(0, len(PRIMES), len(da))
    batch = wl.pack_products(PRIMES, pid, da, db, rng)
    ref = oracle_batch(batch)
    outs = []
    for grid, seed in [(0, 0), (5, 31337)]:
        st, got = run_plan(N, ctx, batch, grid=grid, order_seed=seed)
        assert st == 0
        for i in range(batch.count):
            c0, n = int(batch.c_off[i]), int(batch.da[i] + batch.db[i] + 1)
            assert np.array_equal(got[c0:c0 + n], ref[c0:c0 + n]), (grid, seed, SPLIT_SHAPES[i])
        outs.append(got)
    assert outs[0].tobytes() == outs[1].tobytes()


def test_split_special_values(N, ctx):
    """All-(P-1) operands, whose top coefficients are largest, and the binomial
    square (1+x)^d (1+x)^d = (1+x)^2d, at split lengths."""
    def binomials_mod(n, P):
        """C(n, k) mod P for k = 0 .. n from factorials mod P (n < P)."""
        f = [1] * (n + 1)
        for i in range(1, n + 1):
            f[i] = f[i - 1] * i % P
        inv_fn = pow(f[n], P - 2, P)
        inv = [1] * (n + 1)
        inv[n] = inv_fn
        for i in range(n, 0, -1):
            inv[i - 1] = inv[i] * i % P
        return [f[n] * inv[k] % P * inv[n - k] % P for k in range(n + 1)]

    for d in (4100, 20000, 65600):
        P = PRIMES[d % len(PRIMES)]
        full = np.full(d + 1, P - 1, dtype=np.uint32)
        b = wl.pack_products(PRIMES, [PRIMES.index(P)], [d], [d], np.random.default_rng(0))
        b.coeffs[b.a_off[0]:b.a_off[0] + d + 1] = full
        b.coeffs[b.b_off[0]:b.b_off[0] + d + 1] = full
        st, got = run_plan(N, ctx, b)
        assert st == 0
        k = np.arange(2 * d + 1, dtype=np.int64)
        want = ((np.minimum(k, 2 * d - k) + 1) % P).astype(np.uint64)   # (P-1)^2 = 1 mod P
        assert np.array_equal(got[:2 * d + 1].astype(np.uint64), want)
        binom = np.array(binomials_mod(d, P), dtype=np.uint32)
        b.coeffs[b.a_off[0]:b.a_off[0] + d + 1] = binom
        b.coeffs[b.b_off[0]:b.b_off[0] + d + 1] = binom
        st, got = run_plan(N, ctx, b)
        assert st == 0
        idx = np.unique(np.concatenate([np.arange(0, 2 * d + 1, 997), np.arange(2 * d - 40, 2 * d + 1),
                                        np.arange(40), [1 << (2 * d).bit_length() - 1]]))
        c2 = binomials_mod(2 * d, P)
        assert all(int(got[i]) == c2[int(i)] for i in idx)


def planned_work(da, db, rm=4):
    """The planning rules restated: (executed REDC, 1 if computed in two
    parts).  Two-block truncated transform when N >= 2^18, both operands
    below h = N/2 and N/16 < m = L - h <= N/4 (block of N/8 points for m <=
    N/8, N/4 above); otherwise the split when the product is multi-pass, both
    operands are below h and the top product's length 2^nt >= 2m - 1 is at
    most N/4; otherwise whole.  A product costs three transforms, less their
    butterflies by a unit twiddle at radix 2^rm, N pointwise products and db+1
    scalings; a block scales all its N points and adds its fold and twist
    products, and its fix-up m (h/s + 1)."""
    def cost(n, dbb):
        return 3 * (1 << n) // 2 * n - unit_twiddle_butterflies(n, rm) + (1 << n) + dbb + 1

    L = da + db + 1
    n = (L - 1).bit_length()
    N, h = 1 << n, 1 << max(n - 1, 0)
    m = L - h
    if n >= 18 and da + 1 <= h and db + 1 <= h and N // 16 < m <= N // 4:
        ls = n - 3 if m <= N // 8 else n - 2
        S = 1 << ls
        block = cost(ls, S - 1) + 2 * S + max(0, da + 1 - S) + max(0, db + 1 - S)
        return cost(n - 1, db) + block + m * (h // S + 1), 1
    if n > 13 and da + 1 <= h and db + 1 <= h and (2 * m - 2).bit_length() <= n - 2:
        return cost(n - 1, db) + cost((2 * m - 2).bit_length(), m - 1), 1
    return cost(n, db), 0


@pytest.mark.parametrize("radix_log", [3, 4])
def test_plan_work_counts(N, ctx, radix_log):
    """ntt_plan_work reports the REDC of the products as planned (rules
    above), at the radix of the plan's shape."""
    rng = np.random.default_rng(5)
    shapes = SPLIT_SHAPES + TFT_SHAPES
    da = [s[0] for s in shapes]
    db = [s[1] for s in shapes]
    batch = wl.pack_products(PRIMES, rng.integers(0, len(PRIMES), len(da)), da, db, rng)
    old = N.tune_get()
    saved = [N.tune_get_length(n) for n in range(24)]
    try:
        N.tune_set(512, radix_log, 1)
        for n in range(24):
            N.tune_set_length(n, 0)
        plan = N.Plan.from_batch(ctx, batch)
        assert plan.shape() == (512, radix_log, 1)
        want, nsplit = 0, 0
        for a, b in zip(da, db):
            w, sp = planned_work(a, b, radix_log)
            want += w
            nsplit += sp
        assert plan.work() == (want, nsplit)
        assert nsplit > 0
        plan.close()
    finally:
        N.tune_set(*old)
        for n, sh in enumerate(saved):
            if sh[0]:
                N.tune_set_length(n, *sh)


def test_truncated_transform_shapes_vs_oracle(N, ctx):
    """Products the two-block truncated transform takes, at the edges of its
    ranges, with balanced and unbalanced operands: every coefficient against
    the oracle, in the persistent plan (two grids and a shuffled order) and
    through the one-call batch."""
    for sh in TFT_SHAPES:
        assert planned_work(*sh)[1] == 1 and N.task_count(*sh) < N.task_count(sh[0] + sh[1], 0)
    rng = np.random.default_rng(78)
    batch = wl.pack_products(PRIMES, rng.integers(0, len(PRIMES), len(TFT_SHAPES)),
                             [x[0] for x in TFT_SHAPES], [x[1] for x in TFT_SHAPES], rng)
    outs = []
    for grid, seed in [(0, 0), (5, 4242)]:
        st, got = run_plan(N, ctx, batch, grid=grid, order_seed=seed)
        assert st == 0
        outs.append(got)
    assert_batch_exact(batch, outs[0])
    assert outs[0].tobytes() == outs[1].tobytes()
    st, one = run_one_call(N, ctx, batch)
    assert st == 0 and one[:batch.out_len].tobytes() == outs[0].tobytes()


def test_truncated_transform_special_values(N, ctx):
    """All-(P-1) operands (the largest residues everywhere the folds add) at
    block lengths N/8 and N/4: c_k = min(k, 2d - k) + 1."""
    for d in (75535, 98303, 700000):
        P = PRIMES[d % len(PRIMES)]
        b = wl.pack_products(PRIMES, [PRIMES.index(P)], [d], [d], np.random.default_rng(0))
        b.coeffs[b.a_off[0]:b.a_off[0] + d + 1] = P - 1
        b.coeffs[b.b_off[0]:b.b_off[0] + d + 1] = P - 1
        st, got = run_plan(N, ctx, b)
        assert st == 0
        k = np.arange(2 * d + 1, dtype=np.int64)
        assert np.array_equal(got[:2 * d + 1].astype(np.int64), (np.minimum(k, 2 * d - k) + 1) % P)


# ---------------------------------------------------------------------------
# One-call batches planned on the device (ntt_polymul_batch)
# ---------------------------------------------------------------------------

def test_one_call_batch_vs_oracle(N, ctx):
    """Uneven batches, split shapes and a batch of single-task products
    through the one-call entry point: every coefficient against the oracle."""
    rng = np.random.default_rng(91)
    split = wl.pack_products(PRIMES, rng.integers(0, len(PRIMES), len(SPLIT_SHAPES)),
                             [x[0] for x in SPLIT_SHAPES], [x[1] for x in SPLIT_SHAPES], rng)
    for batch in (small_batch(96, 0, 17, 41), split, small_batch(300, 0, 13, 92), small_batch(1, 20, 21, 93)):
        st, got = run_one_call(N, ctx, batch)
        assert st == 0
        assert_batch_exact(batch, got)


def test_one_call_equals_plan_bytes(N, ctx):
    """The device planner and the host planner give the same bytes (the
    pipelined host order included) on a batch of many multi-pass products."""
    batch = small_batch(160, 13, 15, 43)
    st, plan_out = run_plan(N, ctx, batch)
    assert st == 0
    st, one = run_one_call(N, ctx, batch)
    assert st == 0
    assert one[:batch.out_len].tobytes() == plan_out[:batch.out_len].tobytes()


def test_one_call_scratch_bytes_match_the_planner(N, ctx):
    """ntt_scratch_bytes is exact: with one word less the planning kernel
    reports MONT_ENOMEM and computes nothing; with exactly that many bytes
    the batch is exact."""
    batch = small_batch(40, 4, 18, 94)
    descs = N.make_descs(batch.prime_id, batch.da, batch.db, batch.a_off, batch.b_off, batch.c_off)
    need = N.batch_scratch_bytes(ctx, descs)
    assert need % 4 == 0
    scr = torch.empty(need // 4, dtype=torch.int32, device="cuda")
    st, got = run_one_call(N, ctx, batch, scratch=scr)
    assert st == 0
    assert_batch_exact(batch, got)
    st, got = run_one_call(N, ctx, batch, scratch=scr[:need // 4 - 1])
    assert st == -4
    assert not np.any(got)


def test_one_call_errors(N, ctx):
    from paper_1609_00999_amd import mont
    batch = small_batch(5, 4, 12, 95)
    descs = N.make_descs(batch.prime_id, batch.da, batch.db, batch.a_off, batch.b_off, batch.c_off)
    scr = torch.empty((N.batch_scratch_bytes(ctx, descs) + 3) // 4, dtype=torch.int32, device="cuda")
    out = torch.zeros(batch.out_len, dtype=torch.int32, device="cuda")
    din = dev(batch.coeffs)
    for field, value, status in (("prime_id", 8, -1), ("reserved", 1, -1), ("da", 1 << 31, -2)):
        bad = descs.copy()
        bad[field][3] = value
        with pytest.raises(ValueError):
            N.batch_scratch_bytes(ctx, bad)
        N.polymul_batch(ctx, N.descs_to_device(bad), len(bad), din, out, scr)
        assert N.batch_status(scr) == status, field
        assert not torch.any(out)                     # nothing computed
    small_ctx = N.Context(PRIMES[:1], 12)
    try:
        long = descs.copy()
        long["prime_id"] = 0
        long["da"][0] = long["db"][0] = 3000              # length 6001 > 2^12
        N.polymul_batch(small_ctx, N.descs_to_device(long), len(long), din, out, scr)
        assert N.batch_status(scr) == -3
    finally:
        small_ctx.close()
    with pytest.raises(mont.MontError) as ei:
        N.polymul_batch(ctx, N.descs_to_device(descs), len(descs), din, out, scr[:16])
    assert ei.value.status == -4
    # an empty batch is planned (status OK) and computes nothing
    N.polymul_batch(ctx, N.descs_to_device(descs[:0]), 0, din, out, scr)
    assert N.batch_status(scr) == 0


def test_one_call_graph_replays_new_descriptors(N, ctx):
    """The one-call batch captured once in a graph: each replay plans the
    descriptors the device buffer holds at that moment, so a second batch of
    the same count runs through the same graph; every replay is exact, with
    eager work and synchronizations in between."""
    b1 = small_batch(24, 6, 18, 96)
    b2 = small_batch(24, 2, 19, 97)
    d1 = N.make_descs(b1.prime_id, b1.da, b1.db, b1.a_off, b1.b_off, b1.c_off)
    d2 = N.make_descs(b2.prime_id, b2.da, b2.db, b2.a_off, b2.b_off, b2.c_off)
    words = max(N.batch_scratch_bytes(ctx, d1), N.batch_scratch_bytes(ctx, d2)) // 4
    scr = torch.empty(words, dtype=torch.int32, device="cuda")
    nin = max(b1.coeffs.size, b2.coeffs.size)
    nout = max(b1.out_len, b2.out_len)
    din = torch.zeros(nin, dtype=torch.int32, device="cuda")
    out = torch.zeros(nout, dtype=torch.int32, device="cuda")
    ddesc = N.descs_to_device(d1)
    din[:b1.coeffs.size].copy_(dev(b1.coeffs))
    N.polymul_batch(ctx, ddesc, 24, din, out, scr)
    assert N.batch_status(scr) == 0
    eager1 = host(out)[:b1.out_len].copy()
    assert_batch_exact(b1, eager1)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        N.polymul_batch(ctx, ddesc, 24, din, out, scr)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        N.polymul_batch(ctx, ddesc, 24, din, out, scr)
    for rep, (b, d) in enumerate([(b2, d2), (b1, d1), (b2, d2)]):
        ddesc.copy_(N.descs_to_device(d))
        din.zero_()
        din[:b.coeffs.size].copy_(dev(b.coeffs))
        out.zero_()
        scr.fill_(-1)                          # eager work that dirties the header and counters
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert N.batch_status(scr) == 0, rep
        assert_batch_exact(b, host(out))
    del g
