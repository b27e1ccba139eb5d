"""Whole-fit invariants of the oracle, from the paper and the mathematics.

I1  counts sum to n after every round (Eq. 4: merges add counts).
I2  the number of active cells never grows (Section 2.1: m is non-increasing).
I4  a converged exit has no two adjacent final cells (Theorem 2).
I5  points of one initial cell share a label (supplement, Definition: all
    points of a cell share one local minimum).
I7  permuting the points permutes the labels: bitwise on dyadic data, where
    every point-to-cell sum is exact and so order-free.
I8  translating by an integer multiple of h (h a power of two, dyadic data)
    shifts every key by that integer and leaves the partition unchanged.
I9  well separated Gaussian blobs (spacing 8h, sigma h/4, cut at 3 sigma)
    are recovered exactly.
Plus the degenerate cases: no points, one point, identical points, cells
that are already isolated, max_iter = 0, and the error codes.
"""
import numpy as np
import pytest

from paper_2206_02200_amd import synth


def _blobs(seed, n=1500, d=3, k=8, scale=5.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 12 * scale, size=(k, d))
    lab = rng.integers(0, k, size=n)
    return c[lab] + scale * 0.8 * rng.standard_normal(size=(n, d))


def _same_partition(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    pairs = set(zip(a.tolist(), b.tolist()))
    return len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


@pytest.mark.parametrize("seed", [201, 202, 203, 204])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_counts_conserved_and_cells_non_increasing(oracle, seed, d):
    x = _blobs(seed, d=d)
    r = oracle.fit(x, 4.0, max_iter=100)
    assert r.counts.sum() == len(x)
    assert np.all(np.diff(r.m_hist) <= 0)
    assert r.m_hist[-1] == r.K
    for t in range(min(r.n_iter, 6) + 1):
        rt = oracle.fit(x, 4.0, max_iter=t)
        assert rt.counts.sum() == len(x)
        assert rt.K == r.m_hist[t]
        assert np.bincount(rt.labels, minlength=rt.K).tolist() == rt.counts.tolist()


@pytest.mark.parametrize("seed", [211, 212, 213])
def test_converged_exit_has_no_adjacent_cells(oracle, seed):
    x = _blobs(seed, d=2)
    r = oracle.fit(x, 3.0, max_iter=1000)
    assert r.flags & oracle.CONVERGED
    for a in range(r.K):
        cheb = np.abs(r.keys - r.keys[a]).max(axis=1)
        cheb[a] = 99
        assert cheb.min() > 1


@pytest.mark.parametrize("seed", [221, 222])
def test_labels_constant_on_initial_cells(oracle, seed):
    x = _blobs(seed, d=3)
    h = 2.5
    r = oracle.fit(x, h)
    q = np.floor(x / h).astype(np.int64)
    _, inv = np.unique(q, axis=0, return_inverse=True)
    inv = inv.ravel()
    for c in np.unique(inv):
        assert len(np.unique(r.labels[inv == c])) == 1


@pytest.mark.parametrize("seed", [231, 232, 233])
def test_permutation_invariance_bitwise_on_dyadic(oracle, seed):
    x = synth.dyadic(_blobs(seed, d=3), bits=8)
    perm = np.random.default_rng(seed).permutation(len(x))
    a = oracle.fit(x, 4.0)
    b = oracle.fit(x[perm], 4.0)
    assert b.labels.tolist() == a.labels[perm].tolist()
    assert a.n_iter == b.n_iter and a.flags == b.flags
    np.testing.assert_array_equal(a.modes.view(np.uint64), b.modes.view(np.uint64))
    np.testing.assert_array_equal(a.counts, b.counts)


@pytest.mark.parametrize("seed", [241, 242])
def test_permutation_invariance_partition_on_generic_data(oracle, seed):
    x = _blobs(seed, d=2)
    perm = np.random.default_rng(seed).permutation(len(x))
    a = oracle.fit(x, 3.0)
    b = oracle.fit(x[perm], 3.0)
    assert _same_partition(a.labels[perm], b.labels)
    np.testing.assert_allclose(a.modes, b.modes, rtol=1e-12)


@pytest.mark.parametrize("shift_cells", [1, -3, 17])
def test_translation_by_multiple_of_h(oracle, shift_cells):
    h = 4.0
    x = synth.dyadic(_blobs(250, d=3), bits=6)
    a = oracle.fit(x, h)
    b = oracle.fit(x + shift_cells * h, h)
    assert _same_partition(a.labels, b.labels)
    np.testing.assert_array_equal(b.keys, a.keys + shift_cells)
    np.testing.assert_allclose(b.modes, a.modes + shift_cells * h, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [261, 262, 263, 264])
@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_separated_blobs_recovered(oracle, seed, d):
    k = 7
    h = 2.0
    x, truth = synth.separated_blobs(k, d, per=120, h=h, seed=seed)
    r = oracle.fit(x, h)
    assert r.flags & oracle.CONVERGED
    assert r.K == k
    assert _same_partition(r.labels, truth)


def test_no_points(oracle):
    r = oracle.fit(np.zeros((0, 3)), 1.0)
    assert r.K == 0 and r.n_iter == 0 and r.flags == oracle.CONVERGED


def test_single_point(oracle):
    r = oracle.fit(np.array([[1.25, -7.5]]), 0.5)
    assert r.K == 1 and r.n_iter == 0 and r.flags == oracle.CONVERGED
    assert r.modes.tolist() == [[1.25, -7.5]] and r.labels.tolist() == [0]


def test_identical_points(oracle):
    x = np.full((1000, 4), 3.14159)
    r = oracle.fit(x, 1.0)
    assert r.K == 1 and r.counts.tolist() == [1000] and r.n_iter == 0
    assert np.all(r.labels == 0)


def test_already_isolated_cells_take_zero_rounds(oracle):
    x = np.array([[0.5, 0.5], [0.6, 0.4], [2.5, 0.5], [0.5, 2.5], [2.5, 2.5]])
    r = oracle.fit(x, 1.0)
    assert r.n_iter == 0 and r.K == 4 and r.flags == oracle.CONVERGED
    assert r.labels.tolist() == [0, 0, 2, 1, 3]


def test_max_iter_zero_caps_when_neighbours_exist(oracle):
    x = np.array([[0.5], [1.5]])
    r = oracle.fit(x, 1.0, max_iter=0)
    assert r.flags == oracle.CAPPED and r.n_iter == 0 and r.K == 2


def test_errors(oracle):
    with pytest.raises(oracle.OracleError) as e:
        oracle.fit(np.array([[np.nan]]), 1.0)
    assert e.value.code == 2
    with pytest.raises(oracle.OracleError) as e:
        oracle.fit(np.array([[1.0]]), 0.0)
    assert e.value.code == 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.fit(np.array([[1e300]]), 1e-300)
    assert e.value.code == 3


def test_key_range_edge(oracle):
    # The oracle keeps keys as int64 and accepts |floor(x/h)| < 2^62: the last
    # binary64 value below 2^62 is accepted, 2^62 itself (either sign) is not.
    below = 2.0**62 - 1024.0  # spacing of binary64 just below 2^62 is 1024
    for v in (below, -below):
        r = oracle.fit(np.array([[v], [0.5]]), 1.0)
        assert r.K == 2 and r.flags == oracle.CONVERGED
        assert sorted(r.keys.ravel().tolist()) == sorted([int(v), 0])
    for v in (2.0**62, -(2.0**62)):
        with pytest.raises(oracle.OracleError) as e:
            oracle.fit(np.array([[v], [0.5]]), 1.0)
        assert e.value.code == 3


def test_far_apart_cells_are_not_neighbours(oracle):
    # Cells 2^32 apart (a distance that wraps to 0 in 32 bits) are not
    # neighbours (Section 2.1 (v)): two clusters, no round.
    r = oracle.fit(np.array([[0.5], [2.0**32 + 0.5]]), 1.0)
    assert (r.K, r.n_iter, r.flags) == (2, 0, oracle.CONVERGED)
    x = np.array([[0.5, 0.5], [0.5, 2.0**32 + 0.5], [1.5, 2.0**32 + 1.5]])
    r = oracle.fit(x, 1.0)
    assert (r.K, r.n_iter) == (2, 1) and r.labels.tolist() == [0, 1, 1]


def test_independent_calls_on_several_threads_match_sequential(oracle):
    # the benchmark runs the oracle one instance per host thread: calls must
    # not share state (bitwise the same results as one after another)
    from concurrent.futures import ThreadPoolExecutor

    rng = np.random.default_rng(11)
    xs = [rng.uniform(0, 200, size=(int(rng.integers(500, 20000)), 3)) for _ in range(16)]
    seq = [oracle.fit(x, 12.0, 100) for x in xs]
    oracle.ensure_loaded()
    with ThreadPoolExecutor(8) as pool:
        par = list(pool.map(lambda x: oracle.fit(x, 12.0, 100), xs))
    for a, b in zip(seq, par):
        assert (a.K, a.n_iter, a.flags) == (b.K, b.n_iter, b.flags)
        np.testing.assert_array_equal(a.labels, b.labels)
        np.testing.assert_array_equal(a.sums.view(np.uint64), b.sums.view(np.uint64))
