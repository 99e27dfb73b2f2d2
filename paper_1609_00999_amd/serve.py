"""Continuous-batching request loop for Montgomery products and polynomial
products on one GPU.

Requests (elementwise Montgomery products of n residues, or polynomial
products of degree d) arrive over time.  The scheduler keeps them in a FIFO,
and whenever an execution slot (a HIP stream with its own reusable batch
objects) is free it admits the longest prefix of the queue whose device
footprint (outputs + transform scratch) fits the HBM budget next to what is
already in flight, and launches it as ONE batch: one persistent launch for
all its elementwise requests and one for all its polynomial products.
Requests that arrive while other batches run are admitted as slots and
memory free up, and batches on different slots overlap on the device.
Per-prime constants and twiddle tables stay resident in one ntt.Context.

The executor interface (launch / poll / finish) lets the same scheduler
drive the GPU executor, a per-request plain-launch executor (the baseline)
and test doubles.
"""
from __future__ import annotations

import collections
import gc
import time
from dataclasses import dataclass, field

import numpy as np

OK = 0
REJECTED = 1        # larger than the whole HBM budget
CANCELLED = 2
TIMED_OUT = 3       # waited in the queue longer than the request's timeout
FAILED = 4          # the executor reported an error for this request

STATUS_NAMES = {OK: "ok", REJECTED: "rejected", CANCELLED: "cancelled", TIMED_OUT: "timed_out", FAILED: "failed"}


@dataclass
class Job:
    """One request as the scheduler sees it."""
    rid: int
    t_arrival: float             # seconds after the start of the run
    kind: str                    # "mul" or "polymul"
    prime_id: int
    size: int                    # n for "mul", degree d for "polymul"
    footprint: int = 0           # device bytes the request holds while in flight
    timeout: float = float("inf")
    payload: object = None       # executor-specific operand handles
    status: int = -1
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: object = None
    error: str = ""
    cancelled: bool = False

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclass
class RunStats:
    jobs: list
    wall: float
    batches: int
    max_inflight_bytes: int
    batch_sizes: list = field(default_factory=list)
    launch_s: list = field(default_factory=list)      # host time spent in each executor launch
    launch_first_rid: list = field(default_factory=list)   # first request id of each launched batch

    def latencies(self, kind=None, warmup: int = 0):
        return np.array([j.latency for j in self.jobs[warmup:] if j.status == OK and (kind is None or j.kind == kind)])

    def summary(self, warmup: int = 0) -> dict:
        lat = self.latencies(warmup=warmup)
        done = [j for j in self.jobs[warmup:] if j.status == OK]
        out = {"requests": len(self.jobs) - warmup, "completed": len(done), "batches": self.batches,
               "wall_s": round(self.wall, 4), "max_inflight_bytes": int(self.max_inflight_bytes)}
        if lat.size:
            span = max(j.t_done for j in done) - min(j.t_arrival for j in done)
            out.update({"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                        "mean_ms": round(float(lat.mean()) * 1e3, 3),
                        "throughput_req_per_s": round(len(done) / span, 1) if span > 0 else None})
            for kind in ("mul", "polymul"):
                lk = self.latencies(kind, warmup)
                if lk.size:
                    out["p50_ms_" + kind] = round(float(np.percentile(lk, 50)) * 1e3, 3)
                    out["p99_ms_" + kind] = round(float(np.percentile(lk, 99)) * 1e3, 3)
        if self.batch_sizes:
            out["mean_batch"] = round(float(np.mean(self.batch_sizes)), 2)
        if self.launch_s:
            ls = np.array([t for t, r in zip(self.launch_s, self.launch_first_rid) if r >= warmup]
                          if len(self.launch_first_rid) == len(self.launch_s) else self.launch_s)
            if ls.size == 0:
                ls = np.array(self.launch_s)
            out["launch_ms_p50"] = round(float(np.percentile(ls, 50)) * 1e3, 3)
            out["launch_ms_max"] = round(float(ls.max()) * 1e3, 3)
            out["launches_over_1ms"] = int((ls > 1e-3).sum())
        counts = collections.Counter(STATUS_NAMES.get(j.status, "?") for j in self.jobs[warmup:])
        out["status_counts"] = dict(counts)
        return out


class Scheduler:
    """FIFO admission by footprint into free slots; one batch per slot."""

    def __init__(self, executor, slots: int = 4, budget_bytes: int = 16 << 30, max_batch: int = 256,
                 clock=time.perf_counter, idle_sleep: float = 0.0, pause_gc: bool = True):
        if slots < 1 or budget_bytes <= 0 or max_batch < 1:
            raise ValueError("slots, budget and max_batch must be positive")
        self.ex = executor
        self.slots = slots
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.clock = clock
        self.idle_sleep = idle_sleep
        # Python's cyclic collector can stop the loop for milliseconds when a
        # full collection walks every live request; reference counting still
        # frees what the loop drops, and the collector resumes afterwards.
        self.pause_gc = pause_gc

    def run(self, jobs: list) -> RunStats:
        was_enabled = gc.isenabled()
        if self.pause_gc:
            gc.disable()
        try:
            return self._run(jobs)
        finally:
            if self.pause_gc and was_enabled:
                gc.enable()

    def _run(self, jobs: list) -> RunStats:
        jobs = sorted(jobs, key=lambda j: (j.t_arrival, j.rid))
        for j in jobs:
            if j.footprint <= 0:
                j.footprint = self.ex.footprint(j)
        pending: collections.deque = collections.deque()
        inflight = {}
        free = list(range(self.slots))[::-1]
        used = 0
        max_used = 0
        batches = 0
        sizes = []
        launch_s = []
        launch_rid = []
        nxt = 0
        t0 = self.clock()
        while nxt < len(jobs) or pending or inflight:
            now = self.clock() - t0
            progressed = False
            while nxt < len(jobs) and jobs[nxt].t_arrival <= now:
                pending.append(jobs[nxt])
                nxt += 1
                progressed = True
            # completions
            for slot in list(inflight):
                handle, batch, fp = inflight[slot]
                if self.ex.poll(handle):
                    t_done = self.clock() - t0
                    errors = self.ex.finish(handle)
                    for j in batch:
                        j.t_done = t_done
                        if j.rid in errors:
                            j.status, j.error = FAILED, errors[j.rid]
                        else:
                            j.status = OK
                    used -= fp
                    del inflight[slot]
                    free.append(slot)
                    progressed = True
            # drop cancelled and expired requests from the head of the queue
            now = self.clock() - t0
            if pending:
                keep = collections.deque()
                for j in pending:
                    if j.cancelled:
                        j.status, j.t_done = CANCELLED, now
                    elif now - j.t_arrival > j.timeout:
                        j.status, j.t_done = TIMED_OUT, now
                    else:
                        keep.append(j)
                pending = keep
            # admission: longest queue prefix that fits, one batch per free slot
            while free and pending:
                batch, fp = [], 0
                while pending and len(batch) < self.max_batch:
                    j = pending[0]
                    if j.footprint > self.budget:
                        pending.popleft()
                        j.status, j.t_done = REJECTED, self.clock() - t0
                        j.error = "footprint %d exceeds the budget %d" % (j.footprint, self.budget)
                        continue
                    if used + fp + j.footprint > self.budget:
                        break
                    batch.append(pending.popleft())
                    fp += j.footprint
                if not batch:
                    break
                slot = free.pop()
                t_admit = self.clock() - t0
                for j in batch:
                    j.t_admit = t_admit
                handle = self.ex.launch(slot, batch)
                launch_s.append(self.clock() - t0 - t_admit)
                launch_rid.append(min(j.rid for j in batch))
                inflight[slot] = (handle, batch, fp)
                used += fp
                max_used = max(max_used, used)
                batches += 1
                sizes.append(len(batch))
                progressed = True
            if not progressed and self.idle_sleep > 0:
                time.sleep(self.idle_sleep)
        return RunStats(jobs, self.clock() - t0, batches, max_used, sizes, launch_s, launch_rid)


# ---------------------------------------------------------------------------
# GPU executors
# ---------------------------------------------------------------------------

def _keeps(keep, rid) -> bool:
    """keep is True (keep every result), False, or a set of request ids."""
    return keep is True or (keep is not False and rid in keep)


class DeviceInputs:
    """Client-side operands: every request's inputs generated on the device
    from the request's own seed and packed into one arena (resident in HBM
    before the run starts, as a client would hand them over)."""

    def __init__(self, reqs, primes, device="cuda"):
        import torch
        self.torch = torch
        offs = {}
        pos = 0
        for r in reqs:
            n = r.size if r.kind == "mul" else r.size + 1
            # both operands start on a 16-byte boundary, so the kernels take
            # their 128-bit paths for every request
            offs[r.rid] = (pos, pos + _a4(n), n)
            pos += 2 * _a4(n)
        self.arena = torch.empty(max(4, pos), dtype=torch.int32, device=device)
        self.offs = offs
        self.kinds = {r.rid: r.kind for r in reqs}
        self.primes = primes
        gen = torch.Generator(device=device)
        for r in reqs:
            a0, b0, n = offs[r.rid]
            P = primes[r.prime_id]
            gen.manual_seed(int(r.seed) & ((1 << 63) - 1))
            vals = torch.randint(0, P, (2, n), generator=gen, device=device, dtype=torch.int64)
            self.arena[a0:a0 + n].copy_(vals[0].to(torch.int32))
            self.arena[b0:b0 + n].copy_(vals[1].to(torch.int32))
        torch.cuda.synchronize()

    def views(self, rid):
        a0, b0, n = self.offs[rid]
        return self.arena[a0:a0 + n], self.arena[b0:b0 + n]

    def host_operands(self, rid):
        a, b = self.views(rid)
        return a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32)


class GpuBatchExecutor:
    """Runs each admitted batch as one vector-batch launch for its elementwise
    requests and one persistent launch for its polynomial products, on the
    slot's stream."""

    def __init__(self, ctx, inputs: DeviceInputs, slots: int, max_batch: int, keep_results: bool = True,
                 max_tasks: int = 1 << 20, arena_bytes: int = 1 << 30, spin_limit: int = 0, warm: bool = True,
                 single_plain: bool = True):
        import torch
        from . import mont, ntt
        self.torch, self.mont, self.ntt = torch, mont, ntt
        self.ctx = ctx
        self.inputs = inputs
        self.keep = keep_results
        # bound on a transform task's dependency waits (0: the library default)
        self.spin_limit = int(spin_limit)
        # A batch holding one polynomial product runs it with ntt_polymul's
        # plain launches (one per pass, each sized to the product) instead of
        # a persistent launch: with nothing to overlap, the persistent grid
        # only adds its task queue and dependency waits to the latency.
        self.single_plain = bool(single_plain)
        # One pinned status word per slot: each batch's persistent launch
        # copies its status there on the slot's stream before the batch's
        # completion event, so finish() reads it without a synchronization.
        self.status_host = torch.zeros(slots, dtype=torch.int32, pin_memory=True)
        self._status_ptr = self.status_host.data_ptr()
        self.params = [mont.setup(P) for P in ctx.primes]
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.vecb = [mont.Batch(max_batch) for _ in range(slots)]
        self.plans = [ntt.Plan.reserve(ctx, max_batch, max_tasks) for _ in range(slots)]
        self.max_tasks = max_tasks
        self.max_batch = max_batch
        dev = inputs.arena.device
        # Per-slot device arenas: a batch carves its outputs and transform
        # scratch from its slot's arena (a slot runs one batch at a time), so
        # the request loop makes no allocator calls; a batch larger than the
        # arena falls back to torch allocations and is counted.
        self.arena_words = max(1024, arena_bytes // 4)
        self.arenas = [torch.empty(self.arena_words, dtype=torch.int32, device=dev) for _ in range(slots)]
        self.fallback_batches = 0
        # Results that are kept are copied out of the arena when their batch
        # finishes, into space reserved here for a known set of requests.
        self.kept = {}
        if isinstance(keep_results, (set, frozenset)):
            words = {rid: self._result_words(rid) for rid in keep_results}
            pool = torch.empty(max(1, sum(_a4(w) for w in words.values())), dtype=torch.int32, device=dev)
            pos = 0
            for rid, w in sorted(words.items()):
                self.kept[rid] = pool[pos:pos + w]
                pos += _a4(w)
        # Host-side breakdown of launches slower than 1 ms: (first request id,
        # seconds in plan update, vector batch, transform launch, the rest).
        self.slow_launches = []
        if warm:
            self.warm()

    def warm(self):
        """Run every kernel and library path a batch can take once on each
        slot (vector batches with descriptors in the launch and uploaded, a
        plan in the launch and an uploaded one with a split product and its
        fix-up), so that code objects load and first-use costs are paid
        before the first request instead of inside the request loop."""
        torch, mont, ntt = self.torch, self.mont, self.ntt
        dev = self.inputs.arena.device
        prm = self.params[0]
        x = torch.ones(1 << 20, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        # one product (lists in the launch), one that the plan splits (lists
        # uploaded, fix-up kernel), then the largest batch the slot takes of
        # two-pass products (a large upload: the runtime's copy path for
        # larger transfers is set up here too, not inside the request loop)
        nbig = max(2, min(self.max_batch, 64))
        shapes = ([(64, 64)], [(8200, 8200)],
                  [((1 << 20) - 1, (1 << 20) - 1)] * 2 + [(9000 + 7 * i, 9000) for i in range(nbig - 2)])
        for slot in range(len(self.streams)):
            s = self.streams[slot]
            for nv in sorted({1, 17, self.vecb[slot].cap} & set(range(1, self.vecb[slot].cap + 1))):
                descs = (mont.VecDesc * nv)()
                for i in range(nv):
                    descs[i] = mont.VecDesc(x.data_ptr() + 64 * i, x.data_ptr() + 64 * i, y.data_ptr() + 64 * i, 16,
                                            prm.P, prm.Pprime)
                self.vecb[slot].update_raw(descs, stream=s)
                self.vecb[slot].mul(stream=s)
            for shp in shapes:
                desc = np.zeros(len(shp), dtype=ntt.DESC_DTYPE)
                cpos = 0
                for i, (da, db) in enumerate(shp):
                    desc[i] = (0, da, db, 0, 0, 0, cpos)
                    cpos += da + db + 1
                plan = self.plans[slot]
                plan.update(desc, stream=s)
                out = torch.empty(max(cpos, 1), dtype=torch.int32, device=dev)
                scr = torch.empty((plan.scratch_bytes + 3) // 4, dtype=torch.int32, device=dev)
                plan.execute(x, out, scr, stream=s)
                plan.status_async(scr, self._status_ptr + 4 * slot, stream=s)
                s.synchronize()
                if int(self.status_host[slot]) != 0:
                    raise RuntimeError("warm-up batch of the serving executor timed out on the device")
        torch.cuda.synchronize()

    def _result_words(self, rid) -> int:
        _, _, n = self.inputs.offs[rid]       # n residues, or d + 1 coefficients
        return n if self.inputs.kinds[rid] == "mul" else 2 * n - 1

    def footprint(self, job: Job) -> int:
        if job.kind == "mul":
            return 4 * job.size
        d = job.size
        return 4 * (2 * d + 1) + self.ntt.scratch_bytes(d, d) + 8

    def launch(self, slot: int, batch):
        torch, mont, ntt = self.torch, self.mont, self.ntt
        clk = time.perf_counter
        t0 = clk()
        t_plan = t_vec = t_exec = 0.0
        s = self.streams[slot]
        muls = [j for j in batch if j.kind == "mul"]
        polys = [j for j in batch if j.kind == "polymul"]
        dev = self.inputs.arena.device
        # Every library call below names the slot's stream explicitly: looking
        # up torch's current stream costs more host time than the call itself.
        plan, desc, cpos = None, None, 0
        one = len(polys) == 1 and self.single_plain
        if one:
            cpos = 2 * polys[0].size + 1
        elif polys:
            desc = np.zeros(len(polys), dtype=ntt.DESC_DTYPE)
            for i, j in enumerate(polys):
                a0, b0, n = self.inputs.offs[j.rid]
                desc[i] = (j.prime_id, j.size, j.size, 0, a0, b0, cpos)
                cpos += 2 * j.size + 1
            plan = self.plans[slot]
            t1 = clk()
            plan.update(desc, stream=s)
            t_plan = clk() - t1
        if one:
            scr_words = (ntt.scratch_bytes(polys[0].size, polys[0].size) + 3) // 4
        else:
            scr_words = (plan.scratch_bytes + 3) // 4 if plan is not None else 0
        need = sum(_a4(j.size) for j in muls) + (_a4(cpos) + _a4(scr_words) if polys else 0)
        arena = self.arenas[slot] if need <= self.arena_words else None
        if arena is None:
            self.fallback_batches += 1
        pos = 0

        def take(nw):
            nonlocal pos
            if arena is None:
                with torch.cuda.stream(s):
                    return torch.empty(max(1, nw), dtype=torch.int32, device=dev)
            v = arena[pos:pos + max(1, nw)]
            pos += _a4(max(1, nw))
            return v

        keep = []
        if muls:
            descs = (mont.VecDesc * len(muls))()
            base = self.inputs.arena.data_ptr()
            for i, j in enumerate(muls):
                a0, b0, _ = self.inputs.offs[j.rid]
                out = take(j.size)
                prm = self.params[j.prime_id]
                descs[i] = mont.VecDesc(base + 4 * a0, base + 4 * b0, out.data_ptr(), j.size, prm.P, prm.Pprime)
                j.result = out
                keep.append(out)
            t1 = clk()
            self.vecb[slot].update_raw(descs, stream=s)
            self.vecb[slot].mul(stream=s)
            t_vec = clk() - t1
        if one:
            j = polys[0]
            out = take(cpos)
            scr = take(scr_words) if scr_words else None
            a0, b0, _ = self.inputs.offs[j.rid]
            base = self.inputs.arena.data_ptr()
            t1 = clk()
            mont.check(mont.lib().ntt_polymul(self.ctx.handle, j.prime_id, base + 4 * a0, j.size, base + 4 * b0, j.size,
                                              out.data_ptr(), scr.data_ptr() if scr is not None else None,
                                              4 * scr_words, s.cuda_stream), "ntt_polymul")
            t_exec = clk() - t1
            keep += [out] + ([scr] if scr is not None else [])
            j.result = out
        elif polys:
            out = take(cpos)
            scr = take(scr_words)
            t1 = clk()
            plan.execute(self.inputs.arena, out, scr, spin_limit=self.spin_limit, stream=s)
            plan.status_async(scr, self._status_ptr + 4 * slot, stream=s)
            t_exec = clk() - t1
            keep += [out, scr]
            for i, j in enumerate(polys):
                c0 = int(desc["c_off"][i])
                j.result = out[c0:c0 + 2 * j.size + 1]
        ev = torch.cuda.Event()
        ev.record(s)
        total = clk() - t0
        if total > 1e-3:
            rec = (min(j.rid for j in batch), round(t_plan, 6), round(t_vec, 6), round(t_exec, 6),
                   round(total - t_plan - t_vec - t_exec, 6))
            if plan is not None:
                rec += (plan.update_times_us(),)     # inside the library: plan, wait, upload, all (us)
            self.slow_launches.append(rec)
        return (ev, batch, keep, slot, arena is not None, bool(polys) and not one)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle) -> dict:
        """Keeps or drops each result; returns {rid: error} for the requests
        whose work failed on the device (a transform launch whose dependency
        wait gave up fails every polynomial product of its batch)."""
        ev, batch, keep, slot, in_arena, had_polys = handle
        torch = self.torch
        errors = {}
        if had_polys and int(self.status_host[slot]) != 0:
            msg = "MONT_ETIMEOUT: a dependency wait of the batch's transform launch gave up"
            for j in batch:
                if j.kind == "polymul":
                    errors[j.rid] = msg
        for j in batch:
            if j.rid in errors or not _keeps(self.keep, j.rid):
                j.result = None
            elif in_arena:
                # The slot's next batch reuses the arena: copy on the slot's
                # stream, so the copy is ordered before that batch.
                with torch.cuda.stream(self.streams[slot]):
                    dst = self.kept.get(j.rid)
                    j.result = dst.copy_(j.result) if dst is not None else j.result.clone()
        return errors

    def close(self):
        for b in self.vecb:
            b.close()
        for p in self.plans:
            p.close()
        self.arenas = []


def _a4(words: int) -> int:
    """Words rounded up to a multiple of 4 (16-byte alignment for vector access)."""
    return (int(words) + 3) & ~3


class GpuPlainExecutor:
    """Baseline: every request on its own with plain launches (mont_mul, or
    ntt_polymul's one-to-three launches), in arrival order on one stream."""

    def __init__(self, ctx, inputs: DeviceInputs, keep_results: bool = True):
        import torch
        from . import mont, ntt
        self.torch, self.mont, self.ntt = torch, mont, ntt
        self.ctx = ctx
        self.inputs = inputs
        self.keep = keep_results
        self.params = [mont.setup(P) for P in ctx.primes]
        self.stream = torch.cuda.Stream()

    def footprint(self, job: Job) -> int:
        if job.kind == "mul":
            return 4 * job.size
        return 4 * (2 * job.size + 1) + self.ntt.scratch_bytes(job.size, job.size)

    def launch(self, slot: int, batch):
        torch, mont, ntt = self.torch, self.mont, self.ntt
        with torch.cuda.stream(self.stream):
            for j in batch:
                a, b = self.inputs.views(j.rid)
                if j.kind == "mul":
                    j.result = mont.mul(self.params[j.prime_id], a, b)
                else:
                    j.result = ntt.polymul(self.ctx, j.prime_id, a, b)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return (ev, batch)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle) -> dict:
        for j in handle[1]:
            if not _keeps(self.keep, j.rid):
                j.result = None
        return {}

    def close(self):
        pass


def jobs_from_requests(reqs, timeout: float = float("inf")):
    """Scheduler jobs for workloads.Request objects (kind, prime, size, arrival)."""
    return [Job(r.rid, r.t_arrival, r.kind, r.prime_id, r.size, timeout=timeout) for r in reqs]
