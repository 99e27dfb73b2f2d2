"""Autotuner for libmont's launch shapes.

It times the candidate launch shapes of a kernel family on the device and
keeps the fastest, caching the choice as JSON keyed by GPU architecture,
kernel family and workload bucket.  The library applies the cache for the
running architecture when it is first loaded (``apply``), so later plans and
launches use the tuned shapes.  Launch shapes never change results (the GPU
tests check every shape against the oracle).

Tuned knobs:
  * elementwise (per op: to, from, mul, muladd, pow): threads per workgroup
    {64, 128, 256, 512} x 128-bit vectors per lane {1, 2, 4} x non-temporal {0, 1};
  * transforms: threads per workgroup {256, 512, 1024} x largest register
    round {3, 4} stages, and the persistent grid as a multiple of the
    resident workgroup count: one default for all lengths (timed on the
    2048-product batch) and one shape per length bucket (LEN_BUCKETS, timed
    on a single product's plain launches and on a batch of products of that
    length), which plain launches use by their length and plans by the
    length that carries most of their butterflies.  The transform kernels
    execute the same instructions for every prime below 2^31, so the buckets
    are keyed by length only.

Usage:  python -m paper_1609_00999_amd.tune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import time
import warnings

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(PKG, "tune_cache.json")

ELEM_SHAPES = [(b, v, nt) for b in (64, 128, 256, 512) for v in (1, 2, 4) for nt in (1, 0)]
NTT_SHAPES = [(t, r) for t in (256, 512, 1024) for r in (3, 4)]
GRID_MULTS = (1, 2)
# (first, last) log2 lengths of each bucket; the bucket is timed at its last length
LEN_BUCKETS = ((0, 13), (14, 16), (17, 19), (20, 21), (22, 23))
applied: dict = {}


def cache_path() -> str:
    return os.environ.get("MONT_TUNE_CACHE", DEFAULT_CACHE)


def load(path: str | None = None) -> dict:
    """The tuning cache ({} if there is none yet).  A cache that exists but
    cannot be read or parsed is reported with a RuntimeWarning and ignored."""
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError) as e:
        warnings.warn("libmont tuning cache %s not loaded (%s); built-in launch shapes stay in force"
                      % (path, e), RuntimeWarning)
        return {}
    if not isinstance(data, dict):
        warnings.warn("libmont tuning cache %s is not a JSON object; ignored" % path, RuntimeWarning)
        return {}
    return data


def save(cache: dict, path: str | None = None) -> str:
    path = path or cache_path()
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def merge(cache: dict, arch: str, family: str, bucket: str, entry: dict) -> dict:
    cache.setdefault(arch, {}).setdefault(family, {})[bucket] = entry
    return cache


def best_entry(results, tie: float = 0.0, cost=None):
    """results: list of (config, seconds); the fastest, with every measurement.
    With tie > 0, among the configs within that fraction of the fastest time
    the one of least cost(config) wins (ties keep the fastest)."""
    cfg, sec = min(results, key=lambda r: r[1])
    if tie > 0 and cost is not None:
        close = [r for r in results if r[1] <= sec * (1 + tie)]
        cfg, sec = min(close, key=lambda r: (cost(r[0]), r[1]))
    return {"config": list(cfg), "seconds": sec, "measured": [[list(c), s] for c, s in results]}


def choose(cache: dict, arch: str, family: str):
    """The tuned config of a family for an architecture: the entry of the
    largest numeric bucket (the bench sizes), or None."""
    fam = cache.get(arch, {}).get(family, {})
    if not fam:
        return None
    key = max(fam, key=lambda k: int(k) if k.lstrip("-").isdigit() else -1)
    return fam[key]["config"]


def apply(cache: dict, arch: str, lib) -> dict:
    """Set the tuned launch shapes of `arch` through the C ABI; returns what
    was applied."""
    applied = {}

    def rejected(family, cfg, why):
        warnings.warn("libmont tuning cache entry %s %r for %s not applied (%s)" % (family, cfg, arch, why),
                      RuntimeWarning)

    for op, idx in (("to", 0), ("from", 1), ("mul", 2), ("muladd", 3), ("pow", 4), ("modmul", 5)):
        fam = "elem_" + op
        cfg = choose(cache, arch, fam)
        if not cfg:
            continue
        try:
            st = lib.mont_elem_tune_set(idx, int(cfg[0]), int(cfg[1]), int(cfg[2]))
        except (TypeError, ValueError, IndexError) as e:
            rejected(fam, cfg, e)
            continue
        if st == 0:
            applied[fam] = cfg
        else:
            rejected(fam, cfg, "status %d" % st)
    for key, entry in sorted(cache.get(arch, {}).get("ntt_len", {}).items()):
        try:
            lo, hi = (int(x) for x in key.split("-"))
            cfg = [int(x) for x in entry["config"]]
            sts = [lib.ntt_tune_set_length(n, cfg[0], cfg[1], cfg[2]) for n in range(lo, hi + 1)]
        except (TypeError, ValueError, IndexError, KeyError, AttributeError) as e:
            rejected("ntt_len " + key, entry, e)
            continue
        if all(st == 0 for st in sts):
            applied["ntt_len_" + key] = cfg
        else:
            rejected("ntt_len " + key, cfg, "status %r" % sts)
    cfg = choose(cache, arch, "ntt")
    if cfg:
        try:
            st = lib.ntt_tune_set(int(cfg[0]), int(cfg[1]), int(cfg[2]))
        except (TypeError, ValueError, IndexError) as e:
            st = None
            rejected("ntt", cfg, e)
        if st == 0:
            applied["ntt"] = cfg
        elif st is not None:
            rejected("ntt", cfg, "status %d" % st)
    return applied


# ---------------------------------------------------------------------------
# measurement (needs the GPU)
# ---------------------------------------------------------------------------

def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def tune_elementwise(n_log2: int = 28, reps: int = 5, ops=("to", "from", "mul", "muladd", "pow", "modmul")):
    import torch
    from . import mont
    n = 1 << n_log2
    P = 2013265921
    prm = mont.setup(P)
    g = torch.Generator(device="cuda").manual_seed(7)
    a = torch.randint(0, P, (n,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
    b = torch.randint(0, P, (n,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
    c = torch.empty_like(a)
    o = torch.empty_like(a)
    calls = {"to": lambda: mont.to_mont(prm, a, out=o), "from": lambda: mont.from_mont(prm, a, out=o),
             "mul": lambda: mont.mul(prm, a, b, out=o), "muladd": lambda: mont.muladd(prm, a, b, c, out=o),
             "pow": lambda: mont.pow(prm, a, b, out=o),
             "modmul": lambda: mont.modmul(prm, a, b, out=o)}
    out = {}
    for op in ops:
        old = mont.elem_tune_get(op)
        res = []
        for shape in ELEM_SHAPES:
            mont.elem_tune_set(op, *shape)
            res.append((shape, _time(torch, calls[op], reps)))
        best = best_entry(res) if res else None
        if best:
            mont.elem_tune_set(op, *best["config"])
            out[op] = best
        else:
            mont.elem_tune_set(op, *old)
    return out


def tune_ntt(batch=None, reps: int = 3):
    import torch
    from . import mont, ntt
    from . import workloads as wl
    batch = batch or wl.polymul_batch()
    ctx = ntt.Context(wl.PRIMES_NTT, 23)
    din = torch.from_numpy(batch.coeffs.view(np.int32)).cuda()
    dout = torch.empty(batch.out_len, dtype=torch.int32, device="cuda")
    L = mont.lib()
    res = []
    # per-length entries could override the default for the plan: time the
    # default alone (a plan takes its launch shape when it is created); the
    # per-length tuning runs afterwards
    for n in range(24):
        ntt.tune_set_length(n, 0)
    scr = None
    for threads, radix in NTT_SHAPES:
        for gm in GRID_MULTS:
            mont.check(L.ntt_tune_set(threads, radix, gm), "ntt_tune_set")
            plan = ntt.Plan.from_batch(ctx, batch)
            if scr is None:
                scr = plan.alloc_scratch()
            t = _time(torch, lambda: plan.execute(din, dout, scr), reps)
            res.append(((threads, radix, gm), t))
            plan.close()
    # A larger grid multiplier only adds workgroups that find the queue empty;
    # within 1 % of the fastest batch the smaller grid wins, since it costs
    # less launch latency when a batch is small (a serving loop).
    best = best_entry(res, tie=0.01, cost=lambda c: c[2])
    mont.check(L.ntt_tune_set(*best["config"]), "ntt_tune_set")
    ctx.close()
    return best


def tune_ntt_lengths(reps: int = 3, buckets=LEN_BUCKETS):
    """One launch shape per length bucket: each shape is timed on one product
    of the bucket's longest length (plain launches) and on a batch of
    products of that length (one persistent launch); the shape with the
    least sum of the two times, each relative to its fastest, wins."""
    import torch
    from . import ntt
    from . import workloads as wl
    ctx = ntt.Context(wl.PRIMES_NTT, 23)
    rng = np.random.default_rng(11)
    out = {}
    try:
        for lo, hi in buckets:
            n = hi
            d = (1 << (n - 1)) - 1                       # one product of length 2^n - 1
            a = torch.randint(0, wl.PRIMES_NTT[0], (d + 1,), dtype=torch.int64, device="cuda").to(torch.int32)
            pout = torch.empty(2 * d + 1, dtype=torch.int32, device="cuda")
            pscr = torch.empty(max(1, ntt.scratch_bytes(d, d) // 4), dtype=torch.int32, device="cuda")
            # products whose length lies in (0.9 N, N]: each is one whole
            # product of length N = 2^n (no split, no truncated transform),
            # so the plan takes this length's shape
            count = max(8, min(512, 1 << max(0, 24 - n)))
            degs = rng.integers(int(0.45 * (1 << n)), 1 << (n - 1), count)
            batch = wl.pack_products(wl.PRIMES_NTT, rng.integers(0, 8, count), degs, degs, rng)
            din = torch.from_numpy(batch.coeffs.view(np.int32)).cuda()
            dout = torch.empty(batch.out_len, dtype=torch.int32, device="cuda")
            plain, batched = {}, {}
            for threads, radix in NTT_SHAPES:
                for m in range(lo, hi + 1):
                    ntt.tune_set_length(m, threads, radix, 1)
                plain[(threads, radix)] = _time(torch, lambda: ntt.polymul(ctx, 0, a, a, out=pout, scratch=pscr), reps)
                for gm in GRID_MULTS:
                    for m in range(lo, hi + 1):
                        ntt.tune_set_length(m, threads, radix, gm)
                    plan = ntt.Plan.from_batch(ctx, batch)
                    scr = plan.alloc_scratch()
                    batched[(threads, radix, gm)] = _time(torch, lambda: plan.execute(din, dout, scr), reps)
                    plan.close()
                    del scr
            p0, b0 = min(plain.values()), min(batched.values())
            res = [(cfg, plain[cfg[:2]] / p0 + t / b0) for cfg, t in batched.items()]
            best = best_entry(res, tie=0.01, cost=lambda c: c[2])
            best["plain_seconds"] = {"%d_%d" % k: v for k, v in plain.items()}
            best["batch_seconds"] = {"%d_%d_%d" % k: v for k, v in batched.items()}
            cfg = best["config"]
            for m in range(lo, hi + 1):
                ntt.tune_set_length(m, cfg[0], cfg[1], cfg[2])
            out["%d-%d" % (lo, hi)] = best
    finally:
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=cache_path())
    ap.add_argument("--quick", action="store_true", help="smaller elementwise size (2^24)")
    args = ap.parse_args()
    arch = device_arch()
    cache = load(args.out)
    t0 = time.time()
    n_log2 = 24 if args.quick else 28
    for op, entry in tune_elementwise(n_log2).items():
        merge(cache, arch, "elem_" + op, str(n_log2), entry)
        print("elem_%s 2^%d -> %s (%.1f us)" % (op, n_log2, entry["config"], entry["seconds"] * 1e6), flush=True)
    entry = tune_ntt()
    merge(cache, arch, "ntt", "batch2048", entry)
    print("ntt batch2048 -> %s (%.3f ms)" % (entry["config"], entry["seconds"] * 1e3), flush=True)
    for key, e in tune_ntt_lengths().items():
        merge(cache, arch, "ntt_len", key, e)
        print("ntt lengths 2^%s -> %s (relative score %.3f)" % (key, e["config"], e["seconds"]), flush=True)
    print("saved %s in %.1f s" % (save(cache, args.out), time.time() - t0))


if __name__ == "__main__":
    main()
