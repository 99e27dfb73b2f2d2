"""Python binding of libmont's transforms and polynomial products
(argument marshalling only; every step runs in libmont's HIP kernels).

Coefficients are ordinary residues in [0, P) held in torch.uint32 / torch.int32
ROCm tensors.  All calls go to torch's current HIP stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import mont

c_u32 = ctypes.c_uint32
c_u64 = ctypes.c_uint64
c_int = ctypes.c_int
c_size = ctypes.c_size_t
c_vp = ctypes.c_void_p


class PolymulDesc(ctypes.Structure):
    """Mirror of ``polymul_desc`` (include/mont_ntt.h)."""
    _fields_ = [("prime_id", c_u32), ("da", c_u32), ("db", c_u32), ("reserved", c_u32),
                ("a_off", c_u64), ("b_off", c_u64), ("c_off", c_u64)]


DESC_DTYPE = np.dtype([("prime_id", "<u4"), ("da", "<u4"), ("db", "<u4"), ("reserved", "<u4"),
                       ("a_off", "<u8"), ("b_off", "<u8"), ("c_off", "<u8")])
assert DESC_DTYPE.itemsize == ctypes.sizeof(PolymulDesc)


def register(L) -> None:
    """Declare ctypes argument types for the transform entry points."""
    pp = ctypes.POINTER(mont.MontParams)
    vpp = ctypes.POINTER(c_vp)
    L.ntt_ctx_create.argtypes = [ctypes.POINTER(c_u32), c_int, c_int, vpp]
    L.ntt_ctx_destroy.argtypes = [c_vp]
    L.ntt_ctx_prime.argtypes = [c_vp, c_int, pp, ctypes.POINTER(c_u32), ctypes.POINTER(c_u32), vpp, vpp]
    L.ntt_ctx_read_twiddles.argtypes = [c_vp, c_int, c_vp, c_vp]
    L.ntt_tune_set.argtypes = [c_int, c_int, c_int]
    L.ntt_tune_get.argtypes = [ctypes.POINTER(c_int)] * 3
    L.ntt_tune_set_length.argtypes = [c_int, c_int, c_int, c_int]
    L.ntt_tune_get_length.argtypes = [c_int] + [ctypes.POINTER(c_int)] * 3
    L.ntt_forward.argtypes = [c_vp, c_int, c_vp, c_u32, c_vp]
    L.ntt_inverse.argtypes = [c_vp, c_int, c_vp, c_u32, c_vp]
    L.ntt_polymul_scratch_bytes.argtypes = [c_u32, c_u32]
    L.ntt_polymul_scratch_bytes.restype = c_size
    L.ntt_polymul.argtypes = [c_vp, c_int, c_vp, c_u32, c_vp, c_u32, c_vp, c_vp, c_size, c_vp]
    L.ntt_plan_create.argtypes = [c_vp, c_vp, c_int, c_u32, vpp]
    L.ntt_plan_reserve.argtypes = [c_vp, c_int, c_u32, vpp]
    L.ntt_plan_work.argtypes = [c_vp, ctypes.POINTER(c_u64), ctypes.POINTER(c_u32)]
    L.ntt_plan_shape.argtypes = [c_vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    L.ntt_plan_task_count.argtypes = [c_u32, c_u32]
    L.ntt_plan_task_count.restype = c_u32
    L.ntt_plan_update.argtypes = [c_vp, c_vp, c_int, c_u32, c_vp]
    L.ntt_plan_info.argtypes = [c_vp, ctypes.POINTER(c_size), ctypes.POINTER(c_u32), ctypes.POINTER(c_u64),
                                ctypes.POINTER(c_u64), ctypes.POINTER(c_int)]
    L.ntt_plan_execute.argtypes = [c_vp, c_vp, c_vp, c_vp, c_size, c_int, c_u32, c_vp]
    L.ntt_plan_status.argtypes = [c_vp, c_vp, c_vp]
    L.ntt_plan_status_async.argtypes = [c_vp, c_vp, c_vp, c_vp]
    L.ntt_polymul_noalloc.argtypes = [c_vp, c_int, c_vp, c_u32, c_vp, c_u32, c_vp, c_vp]
    L.ntt_plan_update_times.argtypes = [c_vp, ctypes.POINTER(c_u32)]
    L.ntt_scratch_bytes.argtypes = [c_vp, c_vp, c_int]
    L.ntt_scratch_bytes.restype = c_size
    L.ntt_polymul_batch.argtypes = [c_vp, c_vp, c_int, c_vp, c_vp, c_vp, c_size, c_vp]
    L.ntt_batch_status.argtypes = [c_vp, c_vp]
    L.ntt_plan_destroy.argtypes = [c_vp]


def _torch():
    import torch
    return torch


def ceil_log2(x: int) -> int:
    return max(0, (int(x) - 1).bit_length())


class Context:
    """Per-prime constants and resident twiddle tables (ntt_ctx)."""

    def __init__(self, primes, log2_nmax: int = 23):
        L = mont.lib()
        self.primes = tuple(int(p) for p in primes)
        arr = (c_u32 * len(self.primes))(*self.primes)
        h = c_vp()
        mont.check(L.ntt_ctx_create(arr, len(self.primes), log2_nmax, ctypes.byref(h)), "ntt_ctx_create")
        self.handle = h
        self.log2_nmax = log2_nmax

    def close(self):
        if self.handle:
            mont.check(mont.lib().ntt_ctx_destroy(self.handle), "ntt_ctx_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prime(self, prime_id: int):
        """(params, root, log2_max, twf_ptr, twi_ptr) for one prime."""
        prm = mont.MontParams()
        root, lmax = c_u32(), c_u32()
        f, i = c_vp(), c_vp()
        mont.check(mont.lib().ntt_ctx_prime(self.handle, prime_id, ctypes.byref(prm), ctypes.byref(root),
                                            ctypes.byref(lmax), ctypes.byref(f), ctypes.byref(i)),
                   "ntt_ctx_prime")
        return prm, root.value, lmax.value, f.value, i.value

    def twiddles(self, prime_id: int):
        """Host copies of the forward and inverse tables (numpy uint32)."""
        _, _, lmax, _, _ = self.prime(prime_id)
        f = np.empty(1 << lmax, dtype=np.uint32)
        i = np.empty(1 << lmax, dtype=np.uint32)
        mont.check(mont.lib().ntt_ctx_read_twiddles(self.handle, prime_id, f.ctypes.data, i.ctypes.data),
                   "ntt_ctx_read_twiddles")
        return f, i


def forward(ctx: Context, prime_id: int, x):
    """In-place forward transform (bit-reversed output) of a power-of-two length tensor."""
    n = x.numel()
    logn = ceil_log2(n)
    if n == 0 or (1 << logn) != n:
        raise ValueError("length must be a power of two")
    mont.check(mont.lib().ntt_forward(ctx.handle, prime_id, mont.dev_ptr(x, "x"), logn, mont.stream_handle()),
               "ntt_forward")
    return x


def inverse(ctx: Context, prime_id: int, x):
    """In-place inverse transform (bit-reversed input, includes N^-1)."""
    n = x.numel()
    logn = ceil_log2(n)
    if n == 0 or (1 << logn) != n:
        raise ValueError("length must be a power of two")
    mont.check(mont.lib().ntt_inverse(ctx.handle, prime_id, mont.dev_ptr(x, "x"), logn, mont.stream_handle()),
               "ntt_inverse")
    return x


def tune_set(threads: int, radix_log: int, grid_mult: int = 1) -> None:
    mont.check(mont.lib().ntt_tune_set(threads, radix_log, grid_mult), "ntt_tune_set")


def tune_get():
    t, r, g = c_int(), c_int(), c_int()
    mont.check(mont.lib().ntt_tune_get(ctypes.byref(t), ctypes.byref(r), ctypes.byref(g)), "ntt_tune_get")
    return t.value, r.value, g.value


def tune_set_length(log2n: int, threads: int, radix_log: int = 4, grid_mult: int = 1) -> None:
    """Launch shape for transforms of length 2^log2n (threads 0 removes the entry)."""
    mont.check(mont.lib().ntt_tune_set_length(log2n, threads, radix_log, grid_mult), "ntt_tune_set_length")


def tune_get_length(log2n: int):
    t, r, g = c_int(), c_int(), c_int()
    mont.check(mont.lib().ntt_tune_get_length(log2n, ctypes.byref(t), ctypes.byref(r), ctypes.byref(g)),
               "ntt_tune_get_length")
    return t.value, r.value, g.value


def scratch_bytes(da: int, db: int) -> int:
    return int(mont.lib().ntt_polymul_scratch_bytes(da, db))


def polymul(ctx: Context, prime_id: int, a, b, out=None, scratch=None):
    """Product of polynomials a (len da+1) and b (len db+1) modulo the prime, plain launches."""
    torch = _torch()
    if a.numel() == 0 or b.numel() == 0:
        raise ValueError("empty polynomial")
    da, db = a.numel() - 1, b.numel() - 1
    if out is None:
        out = torch.empty(da + db + 1, dtype=a.dtype, device=a.device)
    if out.numel() != da + db + 1:
        raise ValueError("out must hold da+db+1 coefficients")
    if mont._checked_depth:
        P = ctx.prime(prime_id)[0].P
        mont._maybe_check(P, a, b)
    need = scratch_bytes(da, db)
    if need and scratch is None:
        scratch = torch.empty((need + 3) // 4, dtype=torch.int32, device=a.device)
    sp = mont.dev_ptr(scratch, "scratch") if need else None
    sb = scratch.numel() * scratch.element_size() if need else 0
    mont.check(mont.lib().ntt_polymul(ctx.handle, prime_id, mont.dev_ptr(a, "a"), da, mont.dev_ptr(b, "b"), db,
                                      mont.dev_ptr(out, "out"), sp, sb, mont.stream_handle()), "ntt_polymul")
    return out


def polymul_noalloc(ctx: Context, prime_id: int, a, b, out, stream=None):
    """ntt_polymul_noalloc: the product into the caller's `out` (da+db+1
    words) with the library's static scratch (transform length <= 2^21)."""
    if a.numel() == 0 or b.numel() == 0:
        raise ValueError("empty polynomial")
    da, db = a.numel() - 1, b.numel() - 1
    if out.numel() != da + db + 1:
        raise ValueError("out must hold da+db+1 coefficients")
    mont.check(mont.lib().ntt_polymul_noalloc(ctx.handle, prime_id, mont.dev_ptr(a, "a"), da, mont.dev_ptr(b, "b"),
                                              db, mont.dev_ptr(out, "out"), mont.stream_handle(stream)),
               "ntt_polymul_noalloc")
    return out


def task_count(da: int, db: int) -> int:
    """Tasks one product adds to a plan."""
    return int(mont.lib().ntt_plan_task_count(da, db))


def make_descs(prime_id, da, db, a_off, b_off, c_off) -> np.ndarray:
    count = len(da)
    descs = np.zeros(count, dtype=DESC_DTYPE)
    descs["prime_id"] = prime_id
    descs["da"] = da
    descs["db"] = db
    descs["a_off"] = a_off
    descs["b_off"] = b_off
    descs["c_off"] = c_off
    return descs


class Plan:
    """A planned batch of polynomial products for one persistent launch (ntt_plan)."""

    def __init__(self, ctx: Context, prime_id, da, db, a_off, b_off, c_off, order_seed: int = 0, _reserve=None):
        L = mont.lib()
        h = c_vp()
        self.ctx = ctx
        if _reserve is not None:
            max_products, max_tasks = _reserve
            mont.check(L.ntt_plan_reserve(ctx.handle, max_products, max_tasks, ctypes.byref(h)), "ntt_plan_reserve")
            self.handle = h
            self._info()
            return
        descs = make_descs(prime_id, da, db, a_off, b_off, c_off)
        count = len(descs)
        self._descs = descs
        mont.check(L.ntt_plan_create(ctx.handle, descs.ctypes.data if count else None, count, order_seed,
                                     ctypes.byref(h)), "ntt_plan_create")
        self.handle = h
        self._info()

    @classmethod
    def reserve(cls, ctx: Context, max_products: int, max_tasks: int):
        """A reusable plan (ntt_plan_reserve); fill it with update()."""
        return cls(ctx, None, None, None, None, None, None, _reserve=(max_products, max_tasks))

    def update(self, descs: np.ndarray, order_seed: int = 0, stream=None):
        """Replan for a new batch (structured array of DESC_DTYPE), uploaded on
        `stream` (a torch stream; the current stream if None)."""
        descs = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
        self._descs = descs
        mont.check(mont.lib().ntt_plan_update(self.handle, descs.ctypes.data if len(descs) else None, len(descs),
                                              order_seed, mont.stream_handle(stream)), "ntt_plan_update")
        self._info()

    def update_times_us(self):
        """Host microseconds of the last update: (planning, wait for the
        previous upload, upload call, whole call)."""
        us = (c_u32 * 4)()
        mont.check(mont.lib().ntt_plan_update_times(self.handle, us), "ntt_plan_update_times")
        return tuple(us)

    def work(self):
        """(REDC per execution as planned, number of split products)."""
        r, sp = c_u64(), c_u32()
        mont.check(mont.lib().ntt_plan_work(self.handle, ctypes.byref(r), ctypes.byref(sp)), "ntt_plan_work")
        return r.value, sp.value

    def shape(self):
        """(threads, log2 radix, grid multiplier) of the plan's persistent launch."""
        t, r, g = c_int(), c_int(), c_int()
        mont.check(mont.lib().ntt_plan_shape(self.handle, ctypes.byref(t), ctypes.byref(r), ctypes.byref(g)),
                   "ntt_plan_shape")
        return t.value, r.value, g.value

    def _info(self):
        sb, nt, iw, ow, g = c_size(), c_u32(), c_u64(), c_u64(), c_int()
        mont.check(mont.lib().ntt_plan_info(self.handle, ctypes.byref(sb), ctypes.byref(nt), ctypes.byref(iw),
                                            ctypes.byref(ow), ctypes.byref(g)), "ntt_plan_info")
        self.scratch_bytes, self.ntasks = sb.value, nt.value
        self.in_words, self.out_words, self.default_grid = iw.value, ow.value, g.value

    @classmethod
    def from_batch(cls, ctx: Context, batch, order_seed: int = 0):
        """Plan for a workloads.PolymulBatch (its primes must match the context's)."""
        if tuple(batch.primes) != ctx.primes:
            raise ValueError("batch primes differ from the context's")
        return cls(ctx, batch.prime_id, batch.da, batch.db, batch.a_off, batch.b_off, batch.c_off, order_seed)

    def close(self):
        if self.handle:
            mont.check(mont.lib().ntt_plan_destroy(self.handle), "ntt_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_scratch(self, device="cuda"):
        torch = _torch()
        return torch.empty(max(1, (self.scratch_bytes + 3) // 4), dtype=torch.int32, device=device)

    def execute(self, coeffs_in, out, scratch, grid: int = 0, spin_limit: int = 0, stream=None):
        """One launch of the whole batch on `stream` (the current stream if None)."""
        if coeffs_in.numel() < self.in_words or out.numel() < self.out_words:
            raise ValueError("input or output buffer shorter than the plan needs")
        if scratch.numel() * scratch.element_size() < self.scratch_bytes:
            raise ValueError("scratch smaller than the plan needs")
        mont.check(mont.lib().ntt_plan_execute(self.handle, mont.dev_ptr(coeffs_in, "coeffs_in"),
                                               mont.dev_ptr(out, "out"), mont.dev_ptr(scratch, "scratch"),
                                               scratch.numel() * scratch.element_size(), grid, spin_limit,
                                               mont.stream_handle(stream)), "ntt_plan_execute")
        return out

    def status(self, scratch, stream=None) -> int:
        """0 if the last execution on this scratch completed, else MONT_ETIMEOUT (-6). Synchronizes."""
        return int(mont.lib().ntt_plan_status(self.handle, mont.dev_ptr(scratch, "scratch"),
                                              mont.stream_handle(stream)))

    def status_async(self, scratch, host_word_ptr: int, stream=None) -> None:
        """Enqueue a copy of the last execution's status word into the pinned
        host word at host_word_ptr (0: completed, nonzero: a wait gave up)."""
        mont.check(mont.lib().ntt_plan_status_async(self.handle, mont.dev_ptr(scratch, "scratch"), host_word_ptr,
                                                    mont.stream_handle(stream)), "ntt_plan_status_async")


# ---------------------------------------------------------------------------
# One-call batches planned on the device (ntt_polymul_batch)
# ---------------------------------------------------------------------------

def batch_scratch_bytes(ctx: Context, descs: np.ndarray) -> int:
    """Scratch bytes ntt_polymul_batch needs for these (host) descriptors;
    raises ValueError if a descriptor is invalid for the context."""
    descs = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
    n = int(mont.lib().ntt_scratch_bytes(ctx.handle, descs.ctypes.data if len(descs) else None, len(descs)))
    if n == 0:
        raise ValueError("invalid descriptor for this context")
    return n


def descs_to_device(descs: np.ndarray, device="cuda"):
    """The descriptors as a device tensor (int32 words) for polymul_batch."""
    torch = _torch()
    descs = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
    words = descs.view(np.int32) if len(descs) else np.zeros(0, dtype=np.int32)
    return torch.from_numpy(words.copy()).to(device)


def polymul_batch(ctx: Context, d_descs, count: int, coeffs_in, out, scratch, stream=None):
    """Every product of a batch in one call: the descriptors (device words,
    count records) are planned on the device inside `scratch`, then one
    persistent launch and the split-product fix-up run, all on `stream`."""
    if d_descs.numel() * d_descs.element_size() < count * DESC_DTYPE.itemsize:
        raise ValueError("descriptor buffer shorter than count records")
    mont.check(mont.lib().ntt_polymul_batch(ctx.handle, mont.dev_ptr(d_descs, "descs") if count else None, count,
                                            mont.dev_ptr(coeffs_in, "coeffs_in") if count else None,
                                            mont.dev_ptr(out, "out") if count else None,
                                            mont.dev_ptr(scratch, "scratch"),
                                            scratch.numel() * scratch.element_size(), mont.stream_handle(stream)),
               "ntt_polymul_batch")
    return out


def batch_status(scratch, stream=None) -> int:
    """Status of the last ntt_polymul_batch on this scratch (synchronizes):
    0, MONT_ETIMEOUT, or the planning error (MONT_EINVAL, MONT_ERANGE,
    MONT_ENOROOT, MONT_ENOMEM)."""
    return int(mont.lib().ntt_batch_status(mont.dev_ptr(scratch, "scratch"), mont.stream_handle(stream)))
