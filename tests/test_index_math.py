"""The division by a fixed divisor that the paper-order LSC kernels use for
their (voxel, direction) and (channel, tap) indices (FastDiv in
csrc/kernels.hip): mul = ceil(2^(32+s) / d) with s = ceil(log2 d), and
n / d = (n * mul) >> (32 + s) for 0 <= n < 2^31.  The formula is restated
here and checked against exact integer division: every divisor the layers
use (directions per shell or sampled set, taps per kernel, channels) and
all divisors up to 4096 at the edges and at random dividends, plus every
dividend below 2^16 for small divisors.  The round-up reciprocal is exact
because mul * d - 2^(32+s) < d <= 2^s, so the error of n * mul / 2^(32+s)
against n / d stays below 1/d for n < 2^32."""
import numpy as np
import pytest


def make(d):
    s = 0
    while (1 << s) < d:
        s += 1
    shift = 32 + s
    mul = ((1 << shift) + d - 1) // d
    assert mul < (1 << 34) and mul * ((1 << 31) - 1) < (1 << 64)  # the 64-bit product cannot wrap
    return mul, shift


def div(n, mul, shift):
    return (n * mul) >> shift


LAYER_DIVISORS = [1, 2, 3, 5, 8, 9, 15, 16, 17, 25, 30, 32, 33, 45, 60, 64, 90, 96, 1530, 4096 + 37, (1 << 20)]


@pytest.mark.parametrize("d", LAYER_DIVISORS)
def test_fastdiv_layer_divisors(d):
    mul, shift = make(d)
    rng = np.random.default_rng(d)
    ns = [int(x) for x in rng.integers(0, 1 << 31, 20000)]
    edges = [0, 1, d - 1, d, d + 1, (1 << 31) - 1, (1 << 31) - d, (1 << 31) - 1 - ((1 << 31) - 1) % d]
    for q in (1, 2, 7, 1000, ((1 << 31) - 1) // d):
        edges += [q * d - 1, q * d, q * d + 1]
    for n in ns + [e for e in edges if 0 <= e < (1 << 31)]:
        assert div(n, mul, shift) == n // d, (d, n)


def test_fastdiv_all_divisors_edges():
    for d in range(1, 4097):
        mul, shift = make(d)
        top = (1 << 31) - 1
        for n in (0, d - 1, d, 2 * d - 1, top, top - top % d, top - top % d - 1):
            if n >= 0:
                assert div(n, mul, shift) == n // d, (d, n)


def test_fastdiv_small_divisors_exhaustive():
    n = np.arange(1 << 16, dtype=np.uint64)
    for d in range(1, 130):
        mul, shift = make(d)
        got = (n * np.uint64(mul)) >> np.uint64(shift)
        assert np.array_equal(got, n // np.uint64(d)), d
