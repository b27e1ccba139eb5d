"""Pins of the oracle's canonical pairwise sum R.

R(a_0..a_{L-1}) = a_0 for L = 1, else R(first P) + R(rest) with P the largest
power of two below L.  The trees below are written out by hand; a left fold,
a split at P <= L, or a right-anchored tree gives different bits on the
cancellation inputs used here.
"""
import math

import numpy as np
import pytest


def _hand_tree(a):
    L = len(a)
    if L == 1:
        return a[0]
    if L == 2:
        return a[0] + a[1]
    if L == 3:
        return (a[0] + a[1]) + a[2]
    if L == 4:
        return (a[0] + a[1]) + (a[2] + a[3])
    if L == 5:
        return ((a[0] + a[1]) + (a[2] + a[3])) + a[4]
    if L == 6:
        return ((a[0] + a[1]) + (a[2] + a[3])) + (a[4] + a[5])
    if L == 7:
        return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + a[6])
    if L == 8:
        return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))
    if L == 9:
        return (((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))) + a[8]
    raise ValueError


@pytest.mark.parametrize("L", range(1, 10))
def test_matches_hand_written_trees(oracle, L):
    rng = np.random.default_rng(100 + L)
    for _ in range(200):
        # wildly different magnitudes make every association visible
        a = rng.standard_normal(L) * 10.0 ** rng.integers(-8, 17, size=L)
        got = oracle.pairwise_sum(a)
        want = _hand_tree([float(v) for v in a])
        assert np.float64(got).view(np.uint64) == np.float64(want).view(np.uint64)


def test_association_is_visible(oracle):
    # 1e16 + 1 rounds back to 1e16 (ulp 2): (a+b)+c differs from a+(b+c)
    assert oracle.pairwise_sum([1e16, 1.0, 1.0]) == 1e16
    assert oracle.pairwise_sum([1.0, 1.0, 1e16]) == 1e16 + 2.0
    # L = 4 pairs (0,1) and (2,3): (1+1e100)+(-1e100+1) = 0, a left fold gives 1
    assert oracle.pairwise_sum([1.0, 1e100, -1e100, 1.0]) == 0.0
    # L = 5 splits 4 + 1: ((1e100+1)+(-1e100+1))+1 = 1; a 2 + 3 split gives
    # (1e100+1)+((-1e100+1)+1) = 0 and a left fold gives 2
    assert oracle.pairwise_sum([1e100, 1.0, -1e100, 1.0, 1.0]) == 1.0


def test_exact_on_dyadic_data(oracle):
    rng = np.random.default_rng(7)
    for L in (1, 2, 3, 17, 1000, 4097):
        a = np.round(rng.uniform(-1000, 1000, size=L) * 256) / 256
        assert oracle.pairwise_sum(a) == math.fsum(a)


def test_error_bound_against_exact_sum(oracle):
    # |R - sum| <= ceil(log2 L) * u * sum|a|  (u = 2^-53)
    rng = np.random.default_rng(8)
    for L in (3, 100, 1023, 1024, 1025, 65537):
        a = rng.standard_normal(L) * 10.0 ** rng.integers(-3, 4, size=L)
        exact = math.fsum(a)
        bound = math.ceil(math.log2(L)) * 2.0 ** -53 * math.fsum(np.abs(a))
        assert abs(oracle.pairwise_sum(a) - exact) <= bound


def test_single_and_signed_zero(oracle):
    assert oracle.pairwise_sum([3.5]) == 3.5
    z = oracle.pairwise_sum([-0.0, -0.0, -0.0])
    assert z == 0.0 and math.copysign(1.0, z) == -1.0
