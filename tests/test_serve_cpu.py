"""The serving scheduler without a GPU: a fake executor backed by the CPU
oracle checks admission by footprint, slot reuse, cancellation, time-outs,
error propagation and that results do not depend on batching."""
import numpy as np
import pytest

import oracle
from paper_1609_00999_amd import serve
from paper_1609_00999_amd import workloads as wl


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4          # every reading advances 0.1 ms
        return self.t


class FakeExecutor:
    """Completes a batch after a simulated duration; results from the oracle."""

    def __init__(self, clock, fail_rids=(), per_item=2e-3):
        self.clock = clock
        self.fail = set(fail_rids)
        self.per_item = per_item
        self.active = {}
        self.max_active = 0
        self.launched = []

    def footprint(self, job):
        return 4 * (job.size if job.kind == "mul" else 2 * job.size + 1)

    def launch(self, slot, batch):
        assert slot not in self.active, "slot reused while busy"
        self.active[slot] = batch
        self.max_active = max(self.max_active, len(self.active))
        self.launched.append([j.rid for j in batch])
        for j in batch:
            req = j.payload
            P, a, b = wl.request_operands(req)
            j.result = oracle.mont_mul(P, a, b) if j.kind == "mul" else oracle.polymul(P, a, b)
        return (slot, self.clock() + self.per_item * len(batch), batch)

    def poll(self, h):
        return self.clock() >= h[1]

    def finish(self, h):
        del self.active[h[0]]
        return {j.rid: "injected failure" for j in h[2] if j.rid in self.fail}


def make_jobs(count, rate, seed=5, mul_log2=(4, 10), poly_log2=(2, 8)):
    reqs = wl.request_stream(count, rate, seed=seed, mul_log2=mul_log2, poly_log2=poly_log2)
    jobs = serve.jobs_from_requests(reqs)
    for j, r in zip(jobs, reqs):
        j.payload = r
    return reqs, jobs


def test_all_complete_and_results_exact():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs, jobs = make_jobs(60, rate=2000.0)
    stats = serve.Scheduler(ex, slots=3, budget_bytes=1 << 30, max_batch=8, clock=clock).run(jobs)
    assert all(j.status == serve.OK for j in stats.jobs)
    assert ex.max_active <= 3
    assert max(stats.batch_sizes) <= 8 and stats.batches < len(jobs)   # requests were batched
    for j in stats.jobs:
        P, a, b = wl.request_operands(j.payload)
        ref = oracle.mont_mul(P, a, b) if j.kind == "mul" else oracle.polymul_schoolbook(P, a, b)
        assert np.array_equal(j.result, ref)
        assert j.t_done >= j.t_admit >= j.t_arrival
    s = stats.summary()
    assert s["completed"] == 60 and s["p99_ms"] >= s["p50_ms"] > 0


def test_fifo_admission_order():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs, jobs = make_jobs(40, rate=5000.0)
    serve.Scheduler(ex, slots=2, budget_bytes=1 << 30, max_batch=5, clock=clock).run(jobs)
    order = [rid for b in ex.launched for rid in b]
    assert order == sorted(order)


def test_footprint_budget_and_rejection():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs, jobs = make_jobs(50, rate=10000.0)
    budget = 3 * max(ex.footprint(j) for j in jobs)
    big = serve.Job(999, 0.0, "mul", 0, budget, payload=wl.Request(999, 0.0, "mul", 0, 16, 7))
    big.footprint = budget + 1
    stats = serve.Scheduler(ex, slots=4, budget_bytes=budget, max_batch=16, clock=clock).run(jobs + [big])
    assert stats.max_inflight_bytes <= budget
    byid = {j.rid: j for j in stats.jobs}
    assert byid[999].status == serve.REJECTED and "exceeds" in byid[999].error
    assert all(byid[j.rid].status == serve.OK for j in jobs)


def test_cancel_and_timeout():
    clock = FakeClock()
    ex = FakeExecutor(clock, per_item=5e-2)
    reqs, jobs = make_jobs(12, rate=1e6)
    jobs[5].cancelled = True
    for j in jobs[8:]:
        j.timeout = 0.0                 # expire as soon as they wait at all
    stats = serve.Scheduler(ex, slots=1, budget_bytes=1 << 30, max_batch=2, clock=clock).run(jobs)
    byid = {j.rid: j for j in stats.jobs}
    assert byid[jobs[5].rid].status == serve.CANCELLED
    assert all(byid[j.rid].status == serve.TIMED_OUT for j in jobs[8:])
    assert all(byid[j.rid].status == serve.OK for j in jobs[:5])


def test_executor_error_reaches_exactly_its_request():
    clock = FakeClock()
    reqs, jobs = make_jobs(30, rate=3000.0)
    bad = jobs[7].rid
    ex = FakeExecutor(clock, fail_rids=[bad])
    stats = serve.Scheduler(ex, slots=2, budget_bytes=1 << 30, max_batch=6, clock=clock).run(jobs)
    for j in stats.jobs:
        assert j.status == (serve.FAILED if j.rid == bad else serve.OK)
    assert stats.summary()["status_counts"] == {"ok": 29, "failed": 1}


def test_alone_equals_mix():
    clock = FakeClock()
    reqs, jobs = make_jobs(25, rate=1e5)
    mix = serve.Scheduler(FakeExecutor(clock), slots=2, budget_bytes=1 << 30, max_batch=10, clock=clock).run(jobs)
    res = {j.rid: j.result for j in mix.jobs}
    for r in reqs[:6]:
        _, alone = make_jobs(25, rate=1e5)
        one = [j for j in alone if j.rid == r.rid]
        one[0].t_arrival = 0.0
        st = serve.Scheduler(FakeExecutor(FakeClock()), slots=1, budget_bytes=1 << 30, clock=FakeClock()).run(one)
        assert np.array_equal(st.jobs[0].result, res[r.rid])


def test_scheduler_argument_checks():
    with pytest.raises(ValueError):
        serve.Scheduler(None, slots=0)
    with pytest.raises(ValueError):
        serve.Scheduler(None, budget_bytes=0)
