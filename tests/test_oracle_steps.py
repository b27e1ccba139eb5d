"""Pins of the oracle's individual steps against what the mathematics fixes.

* binning (Section 2.1 (i)): keys, counts and membership equal numpy's
  floor + unique; sums within R's error bound of the exact sum, and equal to
  it on dyadic data;
* shift (Eq. 1-2, parallel form Eq. 6): p_j is the exact weighted mean of the
  3^d neighbourhood up to the rounding bound, with the neighbourhood found
  here by brute force over all pairs with Chebyshev key distance <= 1 (the
  supplement's M <= 1); the weighted mean minimises the weighted squared
  distance (supplement, Corollary 1 proof); an isolated cell is a fixed point;
* merge (Eq. 3-4): counts conserved, landing keys are floor(p/h), merged sums
  within the bound of the exact weighted sum, merged centroid inside the
  members' bounding box.
"""
import math

import numpy as np
import pytest

from paper_2206_02200_amd import synth

U = 2.0 ** -53


def _blobs(seed, n=600, d=3, k=6, scale=6.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 10 * scale, size=(k, d))
    lab = rng.integers(0, k, size=n)
    return c[lab] + scale * 0.7 * rng.standard_normal(size=(n, d))


@pytest.mark.parametrize("seed", [101, 102, 103])
@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_binning_matches_numpy(oracle, seed, d):
    x = _blobs(seed, d=d)
    h = 3.7
    table, cell0 = oracle.bin_points(x, h)
    q = np.floor(x / h).astype(np.int64)
    uk, inv, cnt = np.unique(q, axis=0, return_inverse=True, return_counts=True)
    np.testing.assert_array_equal(table.keys, uk)
    np.testing.assert_array_equal(table.counts, cnt)
    np.testing.assert_array_equal(cell0, inv.ravel())
    for c in range(len(uk)):
        mem = x[inv.ravel() == c]
        for k in range(d):
            exact = math.fsum(mem[:, k])
            L = len(mem)
            bound = max(1, math.ceil(math.log2(L))) * U * math.fsum(np.abs(mem[:, k]))
            assert abs(table.sums[c, k] - exact) <= bound


def test_binning_sums_exact_on_dyadic(oracle):
    x = synth.dyadic(_blobs(104, d=2), bits=8)
    table, cell0 = oracle.bin_points(x, 2.0)
    for c in range(len(table.counts)):
        mem = x[cell0 == c]
        assert table.sums[c].tolist() == [math.fsum(mem[:, k]) for k in range(2)]


def test_floor_of_negatives_and_boundaries(oracle):
    x = np.array([[-0.5], [-1.0], [-1e-300], [0.0], [3.0], [2.9999999999999996]])
    table, cell0 = oracle.bin_points(x, 1.5)
    # -0.5/1.5 -> -1 ; -1/1.5 -> -1 ; tiny negative -> -1 ; 0 -> 0 ;
    # 3/1.5 = 2 exactly -> 2 ; just below 3 -> 1
    assert table.keys.ravel().tolist() == [-1, 0, 1, 2]
    assert cell0.tolist() == [0, 0, 0, 1, 3, 2]


def test_float32_denormal_is_widened_exactly(oracle):
    tiny = np.float32(1e-45)  # smallest f32 denormal, 2^-149
    x = np.array([[tiny], [tiny]], dtype=np.float32)
    table, _ = oracle.bin_points(x.astype(np.float64), 1.0)
    assert table.sums[0, 0] == 2.0 ** -148


def _neighbours_brute(keys):
    m = len(keys)
    out = []
    for j in range(m):
        cheb = np.abs(keys - keys[j]).max(axis=1)
        out.append(np.nonzero(cheb <= 1)[0])  # ascending index = ascending key
    return out


@pytest.mark.parametrize("seed", [111, 112, 113])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_shift_is_weighted_mean_of_neighbourhood(oracle, seed, d):
    x = _blobs(seed, n=400, d=d)
    table, _ = oracle.bin_points(x, 4.0)
    p, W = oracle.shift(table)
    nbs = _neighbours_brute(table.keys)
    for j, nb in enumerate(nbs):
        assert W[j] == table.counts[nb].sum()
        for k in range(d):
            terms = table.sums[nb, k]
            exact = math.fsum(terms) / W[j]
            # left fold of len(nb) terms then one division
            bound = (len(nb) + 1) * U * math.fsum(np.abs(terms)) / W[j] + U * abs(exact)
            assert abs(p[j, k] - exact) <= bound * 1.0000001


@pytest.mark.parametrize("seed", [121, 122])
def test_shift_minimises_weighted_squared_distance(oracle, seed):
    # Corollary 1 (supplement): the weighted mean minimises
    # f(z) = sum_k C_k ||z - c_k||^2 over the neighbourhood, so f(p_j) <= f(c_j)
    x = _blobs(seed, n=500, d=3)
    table, _ = oracle.bin_points(x, 5.0)
    p, _ = oracle.shift(table)
    cent = table.sums / table.counts[:, None]
    for j, nb in enumerate(_neighbours_brute(table.keys)):
        def f(z):
            return float((table.counts[nb] * ((cent[nb] - z) ** 2).sum(axis=1)).sum())
        fp, fc = f(p[j]), f(cent[j])
        assert fp <= fc * (1 + 1e-12) + 1e-9
        # and no small move in any coordinate direction improves on p_j
        for k in range(3):
            for s in (-1e-3, 1e-3):
                z = p[j].copy()
                z[k] += s
                assert fp <= f(z) * (1 + 1e-12)


def test_isolated_cell_is_a_fixed_point(oracle):
    x = np.array([[0.2, 0.3], [0.7, 0.9], [10.5, 10.5]])
    table, _ = oracle.bin_points(x, 1.0)
    p, W = oracle.shift(table)
    assert W.tolist() == [2, 1]
    assert p[0].tolist() == [(0.2 + 0.7) / 2, (0.3 + 0.9) / 2]
    assert p[1].tolist() == [10.5, 10.5]
    assert not oracle.has_neighbours(table)


@pytest.mark.parametrize("seed", [131, 132, 133])
def test_merge_conserves_and_averages(oracle, seed):
    x = _blobs(seed, n=800, d=2, k=4)
    h = 3.0
    table, _ = oracle.bin_points(x, h)
    p, _ = oracle.shift(table)
    new, g = oracle.merge(table.counts, p, h)
    kap = np.floor(p / h).astype(np.int64)
    assert new.counts.sum() == table.counts.sum()
    for c in range(len(new.counts)):
        mem = np.nonzero(g == c)[0]
        assert len(mem) >= 1
        assert np.all(kap[mem] == new.keys[c])
        assert new.counts[c] == table.counts[mem].sum()
        for k in range(2):
            terms = table.counts[mem] * p[mem, k]
            exact = math.fsum(terms)
            bound = (max(1, math.ceil(math.log2(len(mem)))) + 1) * U * math.fsum(np.abs(terms))
            assert abs(new.sums[c, k] - exact) <= bound
            mean = new.sums[c, k] / new.counts[c]
            lo, hi = p[mem, k].min(), p[mem, k].max()
            assert lo - 4 * U * abs(lo) <= mean <= hi + 4 * U * abs(hi)
    # keys strictly ascending (lexicographic), distinct
    for a, b in zip(new.keys[:-1], new.keys[1:]):
        assert tuple(a) < tuple(b)


def test_has_neighbours_diagonal_only(oracle):
    # cells (0,0) and (1,1) touch at a corner: neighbours per Section 2.1 (ii)
    t, _ = oracle.bin_points(np.array([[0.5, 0.5], [1.5, 1.5]]), 1.0)
    assert oracle.has_neighbours(t)
    t, _ = oracle.bin_points(np.array([[0.5, 0.5], [2.5, 1.5]]), 1.0)
    assert not oracle.has_neighbours(t)
