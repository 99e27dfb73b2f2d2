"""Python binding of the exact integer polynomial products (include/mont_crt.h).

Argument marshalling only: residue reduction, the modular products and the
Chinese-remainder reconstruction all run in libmont's HIP kernels.
Coefficients are uint32 (torch uint32 or int32 bit patterns); results are
three little-endian uint32 limbs per coefficient, shape (n, 3).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import mont, ntt

c_u32 = ctypes.c_uint32
c_vp = ctypes.c_void_p
c_size = ctypes.c_size_t


class CrtParams(ctypes.Structure):
    """Mirror of ``crt_params``."""
    _fields_ = [("P", c_u32 * 3), ("m", mont.MontParams * 3), ("inv12", c_u32), ("p1_mod3", c_u32),
                ("inv123", c_u32), ("reserved", c_u32)]

    @property
    def primes(self):
        return tuple(int(p) for p in self.P)


_registered = False


def lib():
    global _registered
    L = mont.lib()
    if not _registered:
        pp = ctypes.POINTER(CrtParams)
        L.crt_setup.argtypes = [ctypes.POINTER(c_u32), pp]
        L.crt_reduce.argtypes = [pp, c_vp, c_size, c_vp, c_vp, c_vp, c_vp]
        L.crt_combine.argtypes = [pp, c_vp, c_vp, c_vp, c_size, c_vp, c_vp]
        L.crt_polymul_scratch_bytes.argtypes = [c_u32, c_u32]
        L.crt_polymul_scratch_bytes.restype = c_size
        L.crt_polymul.argtypes = [c_vp, ctypes.POINTER(ctypes.c_int), pp, c_vp, c_u32, c_vp, c_u32, c_vp, c_vp, c_size,
                                  c_vp]
        _registered = True
    return L


def setup(primes) -> CrtParams:
    """Garner constants for three distinct primes in (2^30, 2^31)."""
    arr = (c_u32 * 3)(*[int(p) for p in primes])
    out = CrtParams()
    mont.check(lib().crt_setup(arr, ctypes.byref(out)), "crt_setup")
    return out


def reduce(prm: CrtParams, x, out=None):
    """Residues of uint32 x modulo the three primes, shape (3, n)."""
    torch = mont._torch()
    n = x.numel()
    if out is None:
        out = torch.empty((3, n), dtype=x.dtype, device=x.device)
    if out.shape != (3, n):
        raise ValueError("out must have shape (3, n)")
    mont.check(lib().crt_reduce(ctypes.byref(prm), mont.dev_ptr(x, "x"), n, mont.dev_ptr(out[0], "r0"),
                                mont.dev_ptr(out[1], "r1"), mont.dev_ptr(out[2], "r2"), mont.stream_handle()),
               "crt_reduce")
    return out


def combine(prm: CrtParams, r0, r1, r2, out=None):
    """Integers with the given residues, shape (n, 3) of uint32 limbs."""
    torch = mont._torch()
    n = r0.numel()
    if r1.numel() != n or r2.numel() != n:
        raise ValueError("residue arrays differ in size")
    if out is None:
        out = torch.empty((n, 3), dtype=r0.dtype, device=r0.device)
    if out.numel() != 3 * n:
        raise ValueError("out must hold 3n words")
    mont.check(lib().crt_combine(ctypes.byref(prm), mont.dev_ptr(r0, "r0"), mont.dev_ptr(r1, "r1"),
                                 mont.dev_ptr(r2, "r2"), n, mont.dev_ptr(out, "out"), mont.stream_handle()),
               "crt_combine")
    return out


def _prime_ids(ctx: ntt.Context, prm: CrtParams):
    ids = []
    for P in prm.primes:
        if P not in ctx.primes:
            raise ValueError("prime %d is not in the context" % P)
        ids.append(ctx.primes.index(P))
    return ids


def scratch_bytes(da: int, db: int) -> int:
    return int(lib().crt_polymul_scratch_bytes(da, db))


def polymul(ctx: ntt.Context, prm: CrtParams, a, b, out=None, scratch=None):
    """Exact integer product of uint32-coefficient polynomials a and b:
    (len(a)+len(b)-1, 3) uint32 limbs, plain launches (crt_polymul)."""
    torch = mont._torch()
    if a.numel() == 0 or b.numel() == 0:
        raise ValueError("empty polynomial")
    da, db = a.numel() - 1, b.numel() - 1
    if out is None:
        out = torch.empty((da + db + 1, 3), dtype=a.dtype, device=a.device)
    if out.numel() != 3 * (da + db + 1):
        raise ValueError("out must hold 3 (da+db+1) words")
    need = scratch_bytes(da, db)
    if scratch is None:
        scratch = torch.empty((need + 3) // 4, dtype=torch.int32, device=a.device)
    ids = (ctypes.c_int * 3)(*_prime_ids(ctx, prm))
    mont.check(lib().crt_polymul(ctx.handle, ids, ctypes.byref(prm), mont.dev_ptr(a, "a"), da, mont.dev_ptr(b, "b"),
                                 db, mont.dev_ptr(out, "out"), mont.dev_ptr(scratch, "scratch"),
                                 scratch.numel() * scratch.element_size(), mont.stream_handle()), "crt_polymul")
    return out


class Batch:
    """Exact integer products of a packed batch in one persistent launch.

    The operands of product i are coeffs[a_off[i] : +da[i]+1] and
    coeffs[b_off[i] : +db[i]+1] (uint32, offsets multiples of 4 words) and its
    da+db+1 coefficients go to rows c_off[i] : ... of an (out_words, 3) limb
    array.  A run is: crt_reduce over the whole input (one launch, three
    residue copies), one ntt_plan_execute over the 3 x count modular products
    (product i modulo prime j reads copy j), and crt_combine over the whole
    output (one launch)."""

    def __init__(self, ctx: ntt.Context, prm: CrtParams, da, db, a_off, b_off, c_off, in_words: int, out_words: int):
        da, db = np.asarray(da, dtype=np.int64), np.asarray(db, dtype=np.int64)
        a_off, b_off, c_off = (np.asarray(x, dtype=np.int64) for x in (a_off, b_off, c_off))
        if np.any(np.minimum(da, db) + 1 > (1 << 26)):
            raise ValueError("min(da, db) + 1 above 2^26: three 31-bit primes cannot hold the product")
        self.in_words = int(in_words + (-in_words) % 4)   # keeps each residue copy 16-byte aligned
        self.out_words = int(out_words)
        self.prm = prm
        count = da.size
        ids = np.repeat(np.asarray(_prime_ids(ctx, prm), dtype=np.int64), count)
        shift_in = np.repeat(np.arange(3, dtype=np.int64) * self.in_words, count)
        shift_out = np.repeat(np.arange(3, dtype=np.int64) * self.out_words, count)
        self.plan = ntt.Plan(ctx, ids, np.tile(da, 3), np.tile(db, 3), np.tile(a_off, 3) + shift_in,
                             np.tile(b_off, 3) + shift_in, np.tile(c_off, 3) + shift_out)

    @classmethod
    def from_batch(cls, ctx: ntt.Context, prm: CrtParams, batch):
        """For a workloads.PolymulBatch whose coefficients are plain uint32 integers."""
        return cls(ctx, prm, batch.da, batch.db, batch.a_off, batch.b_off, batch.c_off, batch.coeffs.size,
                   batch.out_len)

    def buffers(self, device="cuda"):
        """Device work buffers: residues of the input, modular products, plan scratch."""
        torch = mont._torch()
        return (torch.empty(3 * self.in_words, dtype=torch.int32, device=device),
                torch.empty(max(1, 3 * self.out_words), dtype=torch.int32, device=device),
                self.plan.alloc_scratch(device))

    def run(self, coeffs, out, work, grid: int = 0, check: bool = True, spin_limit: int = 0):
        """coeffs: device uint32 input (at least in_words before padding);
        out: (out_words, 3) limbs; work: from buffers().  With check (the
        default) the call synchronizes and raises MontError(MONT_ETIMEOUT)
        when a dependency wait of the modular products' launch gave up;
        without it the run stays asynchronous and status(work) tells."""
        red, prod, scratch = work
        n = coeffs.numel()
        if n > self.in_words:
            raise ValueError("input longer than planned")
        iw, ow = self.in_words, self.out_words
        reduce(self.prm, coeffs, out=red[:3 * iw].view(3, iw)[:, :n])
        self.plan.execute(red, prod, scratch, grid=grid, spin_limit=spin_limit)
        combine(self.prm, prod[:ow], prod[ow:2 * ow], prod[2 * ow:3 * ow], out=out)
        if check:
            st = self.status(work)
            if st != 0:
                raise mont.MontError(st, "crt Batch.run: modular products")
        return out

    def status(self, work) -> int:
        """0 if the last run on these work buffers completed, else
        MONT_ETIMEOUT (-6).  Synchronizes the current stream."""
        return self.plan.status(work[2])

    def close(self):
        self.plan.close()


def limbs_to_int(limbs) -> list:
    """Host conversion of (n, 3) uint32 limbs to Python integers."""
    w = np.asarray(limbs, dtype=np.uint64).reshape(-1, 3)
    return [int(x) | (int(y) << 32) | (int(z) << 64) for x, y, z in w]
