"""The two-block truncated transform that the batch planner uses for products
of length L = N/2 + m (N/16 < m <= N/4, both operands shorter than N/2,
block length s = N/4 or N/8 with m <= s), checked in Python
integers on the CPU: the cyclic part r = c mod (x^(N/2) - 1), the block
residue u = c mod (x^s - w^s) from a cyclic product of folded and twisted
operands, and the join c = r + (x^(N/2) - 1) q with q = (r mod (x^s - w^s) -
u) / 2, against the plain product (schoolbook convolution)."""
import numpy as np
import pytest

P = 998244353                       # 119 * 2^23 + 1, generator 3


def root(n):
    return pow(3, (P - 1) // n, P)


def cyclic(a, b, n):
    c = [0] * n
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            c[(i + j) % n] = (c[(i + j) % n] + x * y) % P
    return c


def conv(a, b):
    c = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            c[i + j] = (c[i + j] + x * y) % P
    return c


def two_block(a, b, N, s):
    """The product through the cyclic part of length N/2 and one block of length s."""
    h = N // 2
    w = root(N)
    r = cyclic(a, b, h)                                       # c mod (x^h - 1)

    def fold_twist(x):
        out = [0] * s
        for i, v in enumerate(x):                             # x(w y) mod (y^s - 1)
            out[i % s] = (out[i % s] + v * pow(w, i, P)) % P
        return out

    t = cyclic(fold_twist(a), fold_twist(b), s)               # the block's cyclic product
    winv = pow(w, P - 2, P)
    u = [t[k] * pow(winv, k, P) % P for k in range(s)]        # c mod (x^s - w^s)
    inv2 = (P + 1) // 2
    m = len(a) + len(b) - 1 - h
    c = r[:] + [0] * m
    for k in range(m):
        f = sum(r[k + i * s] * pow(w, i * s, P) for i in range(h // s)) % P    # r mod (x^s - w^s)
        q = (f - u[k]) * inv2 % P
        c[k] = (r[k] - q) % P
        c[h + k] = q
    return c


@pytest.mark.parametrize("N,s,da,db", [(64, 16, 23, 24), (64, 16, 31, 16), (64, 8, 20, 19), (128, 32, 60, 35),
                                       (128, 16, 40, 39), (256, 64, 127, 64), (256, 32, 80, 79), (256, 64, 100, 91)])
def test_two_block_product_equals_the_convolution(N, s, da, db):
    h = N // 2
    m = da + db + 1 - h
    assert 0 < m <= s and da < h and db < h
    rng = np.random.default_rng(N + s + da)
    a = [int(x) for x in rng.integers(0, P, da + 1)]
    b = [int(x) for x in rng.integers(0, P, db + 1)]
    assert two_block(a, b, N, s) == conv(a, b)


def test_the_join_needs_the_block_residue():
    """With the block output disturbed in one coefficient, the join is wrong
    exactly where the disturbed coefficient lands (the pin is sensitive)."""
    N, s, da, db = 64, 16, 23, 24
    rng = np.random.default_rng(3)
    a = [int(x) for x in rng.integers(0, P, da + 1)]
    b = [int(x) for x in rng.integers(0, P, db + 1)]
    good = conv(a, b)
    bad_b = b[:]
    bad_b[-1] = (bad_b[-1] + 1) % P
    assert two_block(a, bad_b, N, s) != good
