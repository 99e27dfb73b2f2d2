"""Property tests (hypothesis) over random moduli, vectors and degrees: the
oracle against the definitions in Python integers, the library's host-side
validation and sizing (no GPU), and the serving scheduler's invariants.
Every run is derandomized, so a failure reproduces."""
import ctypes

import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
from paper_1609_00999_amd import serve  # noqa: E402

SETTINGS = settings(max_examples=150, deadline=None, derandomize=True)
R = 1 << 32

odd_moduli = st.integers(min_value=1, max_value=(1 << 30) - 1).map(lambda k: 2 * k + 1)   # odd P in [3, 2^31)
ntt_primes = st.sampled_from([2013265921, 1811939329, 2113929217, 1711276033, 1107296257, 2130706433,
                              1224736769, 2088763393, 998244353, 469762049, 65537, 257, 17])


@SETTINGS
@given(P=odd_moduli, data=st.data())
def test_oracle_montgomery_product_definition(P, data):
    """mul(a, b) R = a b (mod P) with the result canonical, for any odd P < 2^31."""
    n = data.draw(st.integers(1, 64))
    a = np.array(data.draw(st.lists(st.integers(0, P - 1), min_size=n, max_size=n)), dtype=np.uint32)
    b = np.array(data.draw(st.lists(st.integers(0, P - 1), min_size=n, max_size=n)), dtype=np.uint32)
    got = oracle.mont_mul(P, a, b)
    for x, y, z in zip(a.tolist(), b.tolist(), got.tolist()):
        assert 0 <= z < P and z * R % P == x * y % P
    back = oracle.from_mont(P, oracle.to_mont(P, a))
    assert np.array_equal(back, a)


@SETTINGS
@given(P=ntt_primes, data=st.data())
def test_oracle_power_definition(P, data):
    """pow returns the residue of a^e for the value a that the input residue represents."""
    n = data.draw(st.integers(1, 32))
    a = np.array(data.draw(st.lists(st.integers(0, P - 1), min_size=n, max_size=n)), dtype=np.uint32)
    e = np.array(data.draw(st.lists(st.integers(0, R - 1), min_size=n, max_size=n)), dtype=np.uint32)
    got = oracle.mont_pow(P, oracle.to_mont(P, a), e)
    want = [pow(x, y, P) * R % P for x, y in zip(a.tolist(), e.tolist())]
    assert got.tolist() == want


@SETTINGS
@given(P=ntt_primes, data=st.data())
def test_oracle_polymul_is_the_convolution(P, data):
    """Both oracle product paths equal the convolution in Python integers."""
    da = data.draw(st.integers(0, 40))
    db = data.draw(st.integers(0, 40))
    a = data.draw(st.lists(st.integers(0, P - 1), min_size=da + 1, max_size=da + 1))
    b = data.draw(st.lists(st.integers(0, P - 1), min_size=db + 1, max_size=db + 1))
    want = [0] * (da + db + 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            want[i + j] = (want[i + j] + x * y) % P
    A, B = np.array(a, dtype=np.uint32), np.array(b, dtype=np.uint32)
    assert oracle.polymul_schoolbook(P, A, B).tolist() == want
    if (P - 1) & -(P - 1) >= 1 << (da + db).bit_length():       # the transform path needs the root
        g = oracle.primitive_root(P)
        n = 1 << (da + db).bit_length()
        out = np.empty(da + db + 1, dtype=np.uint32)
        work = np.empty(2 * n, dtype=np.uint32)
        lib = oracle._load()
        assert lib.orc_polymul_ntt(P, g, oracle._p(A), da, oracle._p(B), db, oracle._p(out), oracle._p(work)) == 0
        assert out.tolist() == want


@pytest.fixture(scope="module")
def L():
    from paper_1609_00999_amd import mont
    try:
        return mont.lib()
    except Exception as e:            # the library is not built here
        pytest.skip(str(e))


@SETTINGS
@given(P=st.integers(0, (1 << 32) - 1))
def test_setup_validation_and_constants(L, P):
    """mont_setup (host only): odd 3 <= P < 2^31 gives P P' = -1 mod 2^32,
    R mod P and R^2 mod P; anything else is MONT_EINVAL."""
    from paper_1609_00999_amd import mont
    prm = mont.MontParams()
    st_ = L.mont_setup(P, ctypes.byref(prm))
    if P < 3 or P % 2 == 0 or P >= 1 << 31:
        assert st_ == -1
        return
    assert st_ == 0
    assert prm.P == P and (P * prm.Pprime) % R == R - 1
    assert prm.R1 == R % P and prm.R2 == R * R % P
    assert prm.k == ((P - 1) & -(P - 1)).bit_length() - 1


@SETTINGS
@given(da=st.integers(0, (1 << 22) - 1), db=st.integers(0, (1 << 22) - 1))
def test_scratch_and_task_sizing(L, da, db):
    """Host sizing of single products and plan tasks: scratch is 8N bytes for
    N > 2^13 (0 below), and a product adds at least one task and no more
    than the unsplit two-pass product (3 column tiles per row-block column
    group and one task per row block)."""
    n = (da + db).bit_length()
    assert L.ntt_polymul_scratch_bytes(da, db) == (0 if n <= 13 else 8 << n)
    t = L.ntt_plan_task_count(da, db)
    if n <= 13:
        assert t == 1
    else:
        lc = min(13, 14 - (n - 13))
        assert 1 <= t <= 3 * (1 << (13 - lc)) + (1 << (n - 13))


class _Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4
        return self.t


class _Exec:
    """Completes each batch after a fixed number of polls; fails chosen requests."""

    def __init__(self, fail):
        self.fail = set(fail)
        self.busy = set()

    def footprint(self, job):
        return 4 * (job.size if job.kind == "mul" else 2 * job.size + 1)

    def launch(self, slot, batch):
        assert slot not in self.busy
        self.busy.add(slot)
        return [slot, 3, batch]

    def poll(self, h):
        h[1] -= 1
        return h[1] <= 0

    def finish(self, h):
        self.busy.discard(h[0])
        return {j.rid: "injected" for j in h[2] if j.rid in self.fail}


jobs_st = st.lists(st.tuples(st.floats(0, 0.01), st.sampled_from(["mul", "polymul"]), st.integers(1, 5000)),
                   min_size=1, max_size=60)


@SETTINGS
@given(spec=jobs_st, slots=st.integers(1, 4), max_batch=st.integers(1, 16),
       budget=st.integers(1 << 12, 1 << 17), fail=st.sets(st.integers(0, 59), max_size=5))
def test_scheduler_invariants(spec, slots, max_batch, budget, fail):
    """Every request ends in exactly one terminal status (OK, FAILED for the
    injected failures, REJECTED only when larger than the budget), in-flight
    bytes never exceed the budget, batches respect max_batch, and requests
    are admitted in arrival order."""
    jobs = [serve.Job(i, t, k, 0, s) for i, (t, k, s) in enumerate(spec)]
    ex = _Exec(fail)
    stats = serve.Scheduler(ex, slots=slots, budget_bytes=budget, max_batch=max_batch, clock=_Clock(),
                            pause_gc=False).run(jobs)
    assert stats.max_inflight_bytes <= budget
    assert all(b <= max_batch for b in stats.batch_sizes)
    for j in stats.jobs:
        fp = ex.footprint(j)
        if fp > budget:
            assert j.status == serve.REJECTED
        elif j.rid in fail:
            assert j.status == serve.FAILED
        else:
            assert j.status == serve.OK
    admitted = sorted((j for j in stats.jobs if j.status in (serve.OK, serve.FAILED)),
                      key=lambda j: (j.t_admit, j.t_arrival, j.rid))
    order = [(j.t_arrival, j.rid) for j in admitted]
    assert order == sorted(order)
