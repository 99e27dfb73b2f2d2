"""Seeded synthetic workloads for the Montgomery / NTT library.

This module only draws random inputs; it holds none of the method's
arithmetic, so both the GPU path and the CPU oracle can be fed from it.
Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and
``integers(lo, hi, dtype=uint32)``; log-uniform sizes are ``floor(2**U)``
with ``U`` uniform on ``[lo, hi)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# 29- and 30-bit and 31-bit Fourier primes used by the elementwise workloads.
PRIMES_BW = (469762049, 998244353, 2013265921, 2113929217)
P_PLAIN = 2013265921            # 15 * 2^27 + 1
P_POW = 998244353               # 119 * 2^23 + 1
# Eight 31-bit primes c*2^k + 1 with the largest 2-adic valuation of P-1
# (k >= 23, so every one supports transforms up to length 2^23).
PRIMES_NTT = (2013265921, 1811939329, 2113929217, 1711276033,
              1107296257, 2130706433, 1224736769, 2088763393)

# 62- and 63-bit primes for the 64-bit residues: 29*2^57+1, 87*2^56+1,
# 505*2^54+1 and 2^63-25 (the largest prime below 2^63).
PRIMES64 = (4179340454199820289, 6269010681299730433, 9097271247288401921, 9223372036854775783)

SEED_PLAIN = 1
SEED_BW_BASE = 200
SEED_POW = 3
SEED_BATCH = 4
SEED_SERVE = 5
SEED_BW64_BASE = 600
SEED_POW64 = 7
SEED_CRT = 8
SEED_VEC = 9


def uniform(rng: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    """n uint32 values uniform on [lo, hi)."""
    return rng.integers(lo, hi, size=n, dtype=np.uint32)


def log_uniform(rng: np.random.Generator, lo_log2: float, hi_log2: float, n: int) -> np.ndarray:
    """floor(2**U), U uniform on [lo_log2, hi_log2)."""
    return np.floor(np.exp2(rng.uniform(lo_log2, hi_log2, size=n))).astype(np.int64)


def plain_pairs(n: int = 1 << 20, P: int = P_PLAIN, seed: int = SEED_PLAIN):
    """Pairs of ordinary residues in [0, P) for the to -> mul -> from pipeline."""
    rng = np.random.default_rng(seed)
    return uniform(rng, 0, P, n), uniform(rng, 0, P, n)


def bandwidth_triple(prime_index: int, n: int = 1 << 28):
    """(P, a, b, c): three arrays uniform on [0, P), taken as Montgomery residues."""
    P = PRIMES_BW[prime_index]
    rng = np.random.default_rng(SEED_BW_BASE + prime_index)
    return P, uniform(rng, 0, P, n), uniform(rng, 0, P, n), uniform(rng, 0, P, n)


def pow_inputs(n: int = 1 << 24, P: int = P_POW, seed: int = SEED_POW):
    """Bases uniform on [1, P) (taken as residues) and exponents uniform on [0, 2^31)."""
    rng = np.random.default_rng(seed)
    return uniform(rng, 1, P, n), uniform(rng, 0, 1 << 31, n)


@dataclass
class PolymulBatch:
    """Uneven batch of polynomial products, packed back to back.

    prime_id[i], da[i], db[i] describe product i; its operands are
    coeffs[a_off[i] : a_off[i]+da[i]+1] and coeffs[b_off[i] : b_off[i]+db[i]+1],
    and its da+db+1 result coefficients go to out[c_off[i] : ...].
    """
    primes: tuple
    prime_id: np.ndarray
    da: np.ndarray
    db: np.ndarray
    a_off: np.ndarray
    b_off: np.ndarray
    c_off: np.ndarray
    coeffs: np.ndarray
    out_len: int

    @property
    def count(self) -> int:
        return int(self.da.size)

    def operands(self, i: int):
        P = self.primes[int(self.prime_id[i])]
        a = self.coeffs[self.a_off[i]: self.a_off[i] + self.da[i] + 1]
        b = self.coeffs[self.b_off[i]: self.b_off[i] + self.db[i] + 1]
        return P, a, b


def pack_products(primes, prime_id, da, db, rng: np.random.Generator) -> PolymulBatch:
    """Draw coefficients uniform on [0, P) for the given shapes and pack them."""
    prime_id = np.asarray(prime_id, dtype=np.int64)
    da = np.asarray(da, dtype=np.int64)
    db = np.asarray(db, dtype=np.int64)
    count = da.size
    la, lb = da + 1, db + 1
    a_off = np.zeros(count, dtype=np.int64)
    b_off = np.zeros(count, dtype=np.int64)
    c_off = np.zeros(count, dtype=np.int64)
    pos = 0
    cpos = 0
    for i in range(count):
        a_off[i] = pos                       # every operand starts on a 16-byte boundary
        pos += (int(la[i]) + 3) & ~3
        b_off[i] = pos
        pos += (int(lb[i]) + 3) & ~3
        c_off[i] = cpos
        cpos += int(la[i] + lb[i] - 1)
    coeffs = np.zeros(pos, dtype=np.uint32)
    for i in range(count):
        P = primes[int(prime_id[i])]
        vals = uniform(rng, 0, P, int(la[i] + lb[i]))
        coeffs[a_off[i]: a_off[i] + la[i]] = vals[:la[i]]
        coeffs[b_off[i]: b_off[i] + lb[i]] = vals[la[i]:]
    return PolymulBatch(tuple(primes), prime_id, da, db, a_off, b_off, c_off, coeffs, cpos)


def polymul_batch(count: int = 2048, lo_log2: float = 8, hi_log2: float = 20, seed: int = SEED_BATCH,
                  primes=PRIMES_NTT) -> PolymulBatch:
    """count products of two degree-d polynomials, d = floor(2^U), U ~ U[lo, hi),
    each with a prime drawn uniformly from ``primes``."""
    rng = np.random.default_rng(seed)
    d = log_uniform(rng, lo_log2, hi_log2, count)
    prime_id = rng.integers(0, len(primes), size=count)
    return pack_products(primes, prime_id, d, d, rng)


@dataclass
class Request:
    rid: int
    t_arrival: float        # seconds from the start of the stream
    kind: str               # "mul" or "polymul"
    prime_id: int
    size: int               # n for "mul", degree d for "polymul"
    seed: int               # seed of the request's own operands


def request_stream(count: int, rate_per_s: float, seed: int = SEED_SERVE, mul_log2=(10, 24),
                   poly_log2=(10, 22), primes=PRIMES_NTT):
    """Poisson arrivals at ``rate_per_s``; a 50/50 mix of elementwise Montgomery
    products (n log-uniform) and polynomial products (degree log-uniform)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    kinds = rng.integers(0, 2, size=count)
    pids = rng.integers(0, len(primes), size=count)
    mul_sizes = log_uniform(rng, mul_log2[0], mul_log2[1], count)
    poly_sizes = log_uniform(rng, poly_log2[0], poly_log2[1], count)
    seeds = rng.integers(0, 2**62, size=count)
    out = []
    for i in range(count):
        if kinds[i] == 0:
            out.append(Request(i, float(t[i]), "mul", int(pids[i]), int(mul_sizes[i]), int(seeds[i])))
        else:
            out.append(Request(i, float(t[i]), "polymul", int(pids[i]), int(poly_sizes[i]), int(seeds[i])))
    return out


def request_operands(req: Request, primes=PRIMES_NTT):
    """The operands of one request, drawn from its own seed."""
    P = primes[req.prime_id]
    rng = np.random.default_rng(req.seed)
    if req.kind == "mul":
        return P, uniform(rng, 0, P, req.size), uniform(rng, 0, P, req.size)
    return P, uniform(rng, 0, P, req.size + 1), uniform(rng, 0, P, req.size + 1)


def uniform64(rng: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    return rng.integers(lo, hi, size=n, dtype=np.uint64)


def bandwidth_triple64(prime_index: int, n: int = 1 << 27):
    """a, b, c uniform in [0, P) for the 64-bit residue workload (2^27 words
    of 8 bytes = 1 GiB per array, the same bytes as 2^28 32-bit residues)."""
    P = PRIMES64[prime_index]
    rng = np.random.default_rng(SEED_BW64_BASE + prime_index)
    return P, uniform64(rng, 0, P, n), uniform64(rng, 0, P, n), uniform64(rng, 0, P, n)


def pow64_inputs(n: int = 1 << 22, P: int = PRIMES64[3], seed: int = SEED_POW64):
    """Bases uniform in [1, P), exponents uniform over all 64-bit words."""
    rng = np.random.default_rng(seed)
    base = uniform64(rng, 1, P, n)
    e = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    return base, e


def int_products(count: int = 256, lo_log2: float = 8, hi_log2: float = 18, seed: int = SEED_CRT) -> PolymulBatch:
    """count products of two degree-d integer polynomials, d = floor(2^U),
    U ~ U[lo, hi), coefficients uniform over all uint32 words (the packing
    of pack_products with the single bound 2^32 in place of a prime)."""
    rng = np.random.default_rng(seed)
    d = log_uniform(rng, lo_log2, hi_log2, count)
    return pack_products((1 << 32,), np.zeros(count, dtype=np.int64), d, d, rng)


def vector_batch(count: int = 4096, lo_log2: float = 10, hi_log2: float = 20, seed: int = SEED_VEC,
                 primes=PRIMES_NTT):
    """Sizes and primes of a batch of uneven elementwise products: n =
    floor(2^U), U ~ U[lo, hi), each vector with a prime drawn uniformly.
    (Operand values are drawn on the device by the caller.)"""
    rng = np.random.default_rng(seed)
    n = log_uniform(rng, lo_log2, hi_log2, count)
    prime_id = rng.integers(0, len(primes), size=count)
    return n, prime_id
