"""Butterflies by a unit twiddle (CPU).  In a radix-2 transform, the pair
(i, i + 2^t) of stage t inside a block of 2^(t+1) residues is multiplied by
w^(i mod 2^t) scaled to the block, so the first pair of every block takes
w^0 = 1.  The kernels run those pairs as a plain add and subtract in the
register round that holds stage 0 (the only round where they sit at fixed
positions of every group).  This pins the count the plans report and the
identity that makes the shortcut exact."""
import numpy as np
import pytest

from paper_1609_00999_amd import workloads as wl

R = 1 << 32


def unit_twiddle_butterflies(n, rm):
    """Butterflies of one product's three length-2^n transforms whose twiddle
    is w^0 = 1 and which the kernels run as a plain add and subtract: in the
    register round (at most rm stages) that holds stages 0 .. r-1, stage t
    has 2^n / 2^(t+1) of them.  The row pass of a multi-pass transform has 13
    stages in ceil(13 / rm) rounds as even as possible, the stage-0 round
    being the smallest for the forward transforms and the inverse alike; a
    one-task transform of n stages has its smallest round at stage 0 going
    forward and its largest going back."""
    if n == 0:
        return 0
    N = 1 << n
    lr = min(n, 13)
    rounds = -(-lr // rm)
    sizes = [lr // rounds + (1 if i < lr % rounds else 0) for i in range(rounds)]
    unit = lambda r: sum(N >> (t + 1) for t in range(r))
    if n > 13:
        return 3 * unit(min(sizes))
    return 2 * unit(min(sizes)) + unit(max(sizes))


def test_unit_twiddle_counts_small_cases():
    """The unit-twiddle count against a direct enumeration of every
    butterfly's twiddle exponent (stage t pairs i and i + 2^t inside blocks
    of 2^(t+1); the exponent is i mod 2^t, scaled to the block) for
    transforms up to 2^13 in one task: the count is that of the zero
    exponents in the stages of the stage-0 round."""
    for rm in (3, 4):
        for n in range(1, 14):
            rounds = -(-n // rm)
            sizes = [n // rounds + (1 if i < n % rounds else 0) for i in range(rounds)]
            def zeros(r):
                return sum(1 for t in range(r) for i in range(1 << n)
                           if (i >> t) & 1 == 0 and i % (1 << t) == 0)
            assert unit_twiddle_butterflies(n, rm) == 2 * zeros(min(sizes)) + zeros(max(sizes))


def redc(T, P):
    """Algorithm 2 from its definition: (T + m P) / R with m = -T P^-1 mod R,
    reduced once."""
    m = (-T * pow(P, -1, R)) % R
    t = (T + m * P) // R
    return t - P if t >= P else t


@pytest.mark.parametrize("P", wl.PRIMES_NTT)
def test_unit_twiddle_product_is_identity(P):
    """The twiddle 1 in Montgomery form is R mod P, and REDC(y (R mod P)) = y
    for every residue y: the butterfly's product by it can be left out
    without changing a result, in both directions of the transform."""
    rng = np.random.default_rng(P % 1000)
    ys = [0, 1, P - 1, P // 2] + rng.integers(0, P, 2000).tolist()
    one = R % P
    assert all(redc(int(y) * one, P) == int(y) for y in ys)
    # the forward butterfly's form x w + y (P - w) with w = R mod P
    xs = rng.integers(0, P, len(ys)).tolist()
    assert all(redc(int(x) * one + int(y) * (P - one), P) == (int(x) - int(y)) % P for x, y in zip(xs, ys))
