"""CPU oracle for Montgomery modular arithmetic and modular polynomial products.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the bench's
CPU-baseline leg may import this package.  It shares no code with the GPU
library and never imports it.  Every routine computes the plain definition of
its result with 64-bit products and remainders (``oracle.c``), following
Meng, arXiv:1609.00999, section 3.1:

* precomputation ``R*R^-1 - P*P' = 1`` with ``0 < R^-1 < P``, ``0 < P' < R``;
* residue of ``i``: ``i*R mod P``;
* Montgomery product (Algorithm 2's result): ``a_bar*b_bar*R^-1 mod P``.

Large arrays are split over host threads; ctypes releases the GIL for each
C call, so the threads run in parallel.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle64.c")]
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
# ORACLE_LIB names another build of the same sources to load instead (the
# sanitizer test loads an address- and undefined-behaviour-sanitized one).
_LIB = os.environ.get("ORACLE_LIB") or _DEFAULT_LIB

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_lib = None


def build(force: bool = False, out: str | None = None, extra_flags=()) -> str:
    """Compile oracle.c and oracle64.c with gcc into liboracle.so next to them
    (or into `out`, with extra compiler flags such as sanitizers)."""
    out = out or _DEFAULT_LIB
    stale = not os.path.exists(out) or any(os.path.getmtime(out) < os.path.getmtime(f) for f in _SRCS)
    if force or stale:
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", *extra_flags, "-shared", "-fPIC",
                               "-o", tmp, *_SRCS])
        os.replace(tmp, out)
    return out


def loaded_path() -> str:
    """Path of the oracle library this process loaded."""
    return _load()._name


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        if _LIB != _DEFAULT_LIB:
            raise FileNotFoundError("ORACLE_LIB=%s does not exist" % _LIB)
        build()
    lib = ctypes.CDLL(_LIB)
    sz = ctypes.c_size_t
    u32 = ctypes.c_uint32
    lib.orc_setup.argtypes = [u32, ctypes.c_int, _u32p]
    lib.orc_setup.restype = ctypes.c_int
    lib.orc_to.argtypes = [u32, ctypes.c_int, _u32p, _u32p, sz]
    lib.orc_from.argtypes = [u32, u32, _u32p, _u32p, sz]
    lib.orc_mul.argtypes = [u32, u32, _u32p, _u32p, _u32p, sz]
    lib.orc_muladd.argtypes = [u32, u32, _u32p, _u32p, _u32p, _u32p, sz]
    lib.orc_pow.argtypes = [u32, ctypes.c_int, u32, _u32p, _u32p, _u32p, sz]
    lib.orc_modmul.argtypes = [u32, _u32p, _u32p, _u32p, sz]
    lib.orc_modpow.argtypes = [u32, _u32p, _u32p, _u32p, sz]
    lib.orc_polymul_schoolbook.argtypes = [u32, _u32p, u32, _u32p, u32, _u32p]
    lib.orc_horner.argtypes = [u32, _u32p, u32, u32]
    lib.orc_horner.restype = u32
    lib.orc_primitive_root.argtypes = [u32]
    lib.orc_primitive_root.restype = u32
    lib.orc_ntt.argtypes = [u32, _u32p, u32, u32]
    lib.orc_polymul_ntt.argtypes = [u32, u32, _u32p, u32, _u32p, u32, _u32p, _u32p]
    lib.orc_polymul_ntt.restype = ctypes.c_int
    u64 = ctypes.c_uint64
    lib.orc64_setup.argtypes = [u64, ctypes.c_int, _u64p]
    lib.orc64_setup.restype = ctypes.c_int
    lib.orc64_to.argtypes = [u64, ctypes.c_int, _u64p, _u64p, sz]
    lib.orc64_from.argtypes = [u64, u64, _u64p, _u64p, sz]
    lib.orc64_mul.argtypes = [u64, u64, _u64p, _u64p, _u64p, sz]
    lib.orc64_muladd.argtypes = [u64, u64, _u64p, _u64p, _u64p, _u64p, sz]
    lib.orc64_pow.argtypes = [u64, ctypes.c_int, u64, _u64p, _u64p, _u64p, sz]
    lib.orc_crt.argtypes = [_u32p, ctypes.c_int, _u32p, sz, _u32p, ctypes.c_int]
    lib.orc_crt.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(x: np.ndarray):
    return x.ctypes.data_as(_u32p)


def _u32(x) -> np.ndarray:
    x = np.ascontiguousarray(x)
    if x.dtype != np.uint32:
        raise TypeError("oracle arrays must be uint32, got %s" % x.dtype)
    return x


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


class Params:
    """Precomputed constants for odd modulus P and R = 2^r (section 3.1)."""

    def __init__(self, P: int, r: int = 32):
        out = (ctypes.c_uint32 * 5)()
        if _load().orc_setup(P, r, out) != 0:
            raise ValueError("invalid modulus %d for R = 2^%d" % (P, r))
        self.P, self.r = P, r
        self.Pprime, self.R1, self.R2, self.Rinv, self.k = (int(v) for v in out)

    def __repr__(self):
        return "Params(P=%d, r=%d, Pprime=%d, R1=%d, R2=%d, Rinv=%d, k=%d)" % (
            self.P, self.r, self.Pprime, self.R1, self.R2, self.Rinv, self.k)


def setup(P: int, r: int = 32) -> Params:
    return Params(P, r)


def _split(n: int, threads: int, grain: int = 1 << 16):
    threads = max(1, min(threads, (n + grain - 1) // grain))
    step = (n + threads - 1) // threads
    return [(s, min(n, s + step)) for s in range(0, n, step)] if n else []


def _run_chunked(fn, n: int, threads: int | None):
    threads = threads or default_threads()
    parts = _split(n, threads)
    if len(parts) <= 1:
        for s, e in parts:
            fn(s, e)
        return
    with ThreadPoolExecutor(len(parts)) as ex:
        list(ex.map(lambda se: fn(*se), parts))


def to_mont(P: int, a, r: int = 32, threads: int | None = None) -> np.ndarray:
    """a*R mod P for every uint32 a."""
    a = _u32(a)
    out = np.empty_like(a)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc_to(P, r, _p(a[s:e]), _p(out[s:e]), e - s), a.size, threads)
    return out


def from_mont(P: int, x, r: int = 32, threads: int | None = None) -> np.ndarray:
    """x*R^-1 mod P for every uint32 x."""
    x = _u32(x)
    prm = Params(P, r)
    out = np.empty_like(x)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc_from(P, prm.Rinv, _p(x[s:e]), _p(out[s:e]), e - s), x.size, threads)
    return out


def mont_mul(P: int, a, b, r: int = 32, threads: int | None = None) -> np.ndarray:
    """a_bar*b_bar*R^-1 mod P (Algorithm 2's result)."""
    a, b = _u32(a), _u32(b)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    prm = Params(P, r)
    out = np.empty_like(a)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc_mul(P, prm.Rinv, _p(a[s:e]), _p(b[s:e]), _p(out[s:e]), e - s),
                 a.size, threads)
    return out


def mont_muladd(P: int, a, b, c, r: int = 32, threads: int | None = None) -> np.ndarray:
    """(a_bar*b_bar*R^-1 + c_bar) mod P."""
    a, b, c = _u32(a), _u32(b), _u32(c)
    if not (a.shape == b.shape == c.shape):
        raise ValueError("shape mismatch")
    prm = Params(P, r)
    out = np.empty_like(a)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc_muladd(P, prm.Rinv, _p(a[s:e]), _p(b[s:e]), _p(c[s:e]),
                                             _p(out[s:e]), e - s), a.size, threads)
    return out


def mont_pow(P: int, base, exp, r: int = 32, threads: int | None = None) -> np.ndarray:
    """Residue of a^e, where a is the value the residue base_bar represents."""
    base, exp = _u32(base), _u32(exp)
    if base.shape != exp.shape:
        raise ValueError("shape mismatch")
    prm = Params(P, r)
    out = np.empty_like(base)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc_pow(P, r, prm.Rinv, _p(base[s:e]), _p(exp[s:e]), _p(out[s:e]),
                                          e - s), base.size, threads)
    return out


def modmul(P: int, a, b, threads: int | None = None) -> np.ndarray:
    """Ordinary a*b mod P."""
    a, b = _u32(a), _u32(b)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    out = np.empty_like(a)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc_modmul(P, _p(a[s:e]), _p(b[s:e]), _p(out[s:e]), e - s), a.size, threads)
    return out


def modpow(P: int, base, exp, threads: int | None = None) -> np.ndarray:
    """Ordinary a^e mod P (0^0 = 1)."""
    base, exp = _u32(base), _u32(exp)
    if base.shape != exp.shape:
        raise ValueError("shape mismatch")
    out = np.empty_like(base)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc_modpow(P, _p(base[s:e]), _p(exp[s:e]), _p(out[s:e]), e - s), base.size,
                 threads)
    return out


def primitive_root(P: int) -> int:
    g = int(_load().orc_primitive_root(P))
    if g == 0:
        raise ValueError("%d has no primitive root below it" % P)
    return g


def horner(P: int, a, x: int) -> int:
    """a(x) mod P for coefficient array a (a[i] multiplies x^i)."""
    a = _u32(a)
    if a.size == 0:
        return 0
    return int(_load().orc_horner(P, _p(a), a.size - 1, x % P))


def ntt(P: int, a, w: int) -> np.ndarray:
    """Plain forward transform A_k = sum_j a_j w^(jk) mod P, len(a) a power of two."""
    a = _u32(a).copy()
    n = a.size
    logn = n.bit_length() - 1
    if n == 0 or (1 << logn) != n:
        raise ValueError("length must be a power of two")
    _load().orc_ntt(P, _p(a), logn, w % P)
    return a


def polymul_schoolbook(P: int, a, b) -> np.ndarray:
    a, b = _u32(a), _u32(b)
    if a.size == 0 or b.size == 0:
        raise ValueError("empty polynomial")
    c = np.empty(a.size + b.size - 1, dtype=np.uint32)
    _load().orc_polymul_schoolbook(P, _p(a), a.size - 1, _p(b), b.size - 1, _p(c))
    return c


_roots: dict[int, int] = {}


def polymul(P: int, a, b) -> np.ndarray:
    """Product of two polynomials modulo P (coefficient arrays, low degree
    first).  Schoolbook when both degrees are small, the plain transform
    otherwise."""
    a, b = _u32(a), _u32(b)
    if a.size == 0 or b.size == 0:
        raise ValueError("empty polynomial")
    if a.size * b.size <= (1 << 22):
        return polymul_schoolbook(P, a, b)
    g = _roots.get(P)
    if g is None:
        g = _roots[P] = primitive_root(P)
    need = a.size + b.size - 1
    n = 1 << (need - 1).bit_length()
    c = np.empty(need, dtype=np.uint32)
    work = np.empty(2 * n, dtype=np.uint32)
    if _load().orc_polymul_ntt(P, g, _p(a), a.size - 1, _p(b), b.size - 1, _p(c), _p(work)) != 0:
        raise ValueError("P - 1 is not divisible by %d" % n)
    return c


def polymul_many(jobs, threads: int | None = None):
    """polymul over a list of (P, a, b) in parallel host threads."""
    threads = threads or default_threads()
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda j: polymul(*j), jobs))


# --------------------------------------------------------------------------
# 64-bit residues (R = 2^64 by default) and Chinese remaindering
# --------------------------------------------------------------------------

def _p64(x: np.ndarray):
    return x.ctypes.data_as(_u64p)


def _u64(x) -> np.ndarray:
    x = np.ascontiguousarray(x)
    if x.dtype != np.uint64:
        raise TypeError("oracle arrays must be uint64, got %s" % x.dtype)
    return x


class Params64:
    """Section 3.1 constants for odd modulus P < 2^63 and R = 2^r (r <= 64)."""

    def __init__(self, P: int, r: int = 64):
        out = (ctypes.c_uint64 * 5)()
        if _load().orc64_setup(P, r, out) != 0:
            raise ValueError("invalid modulus %d for R = 2^%d" % (P, r))
        self.P, self.r = P, r
        self.Pprime, self.R1, self.R2, self.Rinv, self.k = (int(v) for v in out)


def setup64(P: int, r: int = 64) -> Params64:
    return Params64(P, r)


def to_mont64(P: int, a, r: int = 64, threads: int | None = None) -> np.ndarray:
    a = _u64(a)
    out = np.empty_like(a)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc64_to(P, r, _p64(a[s:e]), _p64(out[s:e]), e - s), a.size, threads)
    return out


def from_mont64(P: int, x, r: int = 64, threads: int | None = None) -> np.ndarray:
    x = _u64(x)
    prm = Params64(P, r)
    out = np.empty_like(x)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc64_from(P, prm.Rinv, _p64(x[s:e]), _p64(out[s:e]), e - s), x.size, threads)
    return out


def mont_mul64(P: int, a, b, r: int = 64, threads: int | None = None) -> np.ndarray:
    a, b = _u64(a), _u64(b)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    prm = Params64(P, r)
    out = np.empty_like(a)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc64_mul(P, prm.Rinv, _p64(a[s:e]), _p64(b[s:e]), _p64(out[s:e]), e - s),
                 a.size, threads)
    return out


def mont_muladd64(P: int, a, b, c, r: int = 64, threads: int | None = None) -> np.ndarray:
    a, b, c = _u64(a), _u64(b), _u64(c)
    if not (a.shape == b.shape == c.shape):
        raise ValueError("shape mismatch")
    prm = Params64(P, r)
    out = np.empty_like(a)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc64_muladd(P, prm.Rinv, _p64(a[s:e]), _p64(b[s:e]), _p64(c[s:e]),
                                               _p64(out[s:e]), e - s), a.size, threads)
    return out


def mont_pow64(P: int, base, exp, r: int = 64, threads: int | None = None) -> np.ndarray:
    base, exp = _u64(base), _u64(exp)
    if base.shape != exp.shape:
        raise ValueError("shape mismatch")
    prm = Params64(P, r)
    out = np.empty_like(base)
    lib = _load()
    _run_chunked(lambda s, e: lib.orc64_pow(P, r, prm.Rinv, _p64(base[s:e]), _p64(exp[s:e]), _p64(out[s:e]),
                                            e - s), base.size, threads)
    return out


def crt(primes, residues, limbs: int) -> np.ndarray:
    """Integers X in [0, prod(primes)) with X = residues[j] mod primes[j], as
    ``limbs`` little-endian uint32 words per element (shape (n, limbs))."""
    pr = np.ascontiguousarray(np.asarray(primes, dtype=np.uint32))
    res = _u32(np.ascontiguousarray(np.asarray(residues, dtype=np.uint32)))
    if res.ndim != 2 or res.shape[0] != pr.size:
        raise ValueError("residues must have shape (len(primes), n)")
    n = res.shape[1]
    out = np.empty((n, limbs), dtype=np.uint32)
    if _load().orc_crt(_p(pr), pr.size, _p(res), n, _p(out), limbs) != 0:
        raise ValueError("bad moduli or too few limbs")
    return out
