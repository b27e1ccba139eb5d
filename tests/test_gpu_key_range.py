"""GPU parity across the key space: wide key boxes, the range edges, and the
stop on an unchanged state.

Every case runs the HIP path (through the C ABI) and the FP64 oracle on the
same bytes and compares labels, keys, counts, sums, modes, round counts and
flags bit for bit.  The inputs are built to reach the code paths that only
large key boxes take:

* packed keys wider than 32 bits (64-bit sort passes, the 64-bit merge
  keys, neighbour lookups through the open-addressing hash because the
  range is too large for a dense table);
* an instance key range above 2^53, where the one-workgroup tail ranks the
  landing keys linearly instead of packing (key, index) into one word;
* a key-box extent of 2^31 or more in some dimension, where the tail keeps
  64-bit cell coordinates (cells 2^32 apart must not look adjacent);
* more than 4096 columns along dimension 0, where the tail finds candidate
  neighbours by binary search instead of its column table;
* the edges of the packed key space: |floor(x/h)| < 2^52 and key boxes below
  2^62 cells.  The oracle keeps plain int64 keys (|floor(x/h)| < 2^62), so
  inputs between the two limits are an expected difference: the device
  returns GS_ERR_KEY_RANGE while the oracle computes a result.
* the stop on a bitwise unchanged state (Section 2.1 (v) with the reading
  that an unchanged state ends the loop), in the one-workgroup tail and in
  the device-wide rounds, for both update rules.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import gs_oracle  # noqa: E402
from paper_2206_02200_amd import gridshift  # noqa: E402

DEV = torch.device("cuda:0")
KEY_RANGE = 3


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bits(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).view(np.uint64)


_CTX = {}


def _ctx(rule="parallel", **cfg):
    key = (rule, tuple(sorted(cfg.items())))
    if key not in _CTX:
        c = gridshift.Context(0)
        c.set_update(rule)
        if cfg:
            c.set_config(**cfg)
        _CTX[key] = c
    return _CTX[key]


def parity(x_np, h, max_iter=100, what="", rule="parallel", **cfg):
    _say(f"key-range case {what}: n={x_np.shape[0]} d={x_np.shape[1]} h={h} rule={rule} cfg={cfg}")
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    g = gridshift.fit(x, h, max_iter, with_sums=True, with_keys=True, ctx=_ctx(rule, **cfg))
    torch.cuda.synchronize()
    o = gs_oracle.fit(np.asarray(x_np, dtype=np.float64), h, max_iter, rule=rule)
    assert (g.info["n_clusters"], g.info["n_iter"], g.info["flags"]) == (o.K, o.n_iter, o.flags), what
    assert g.info["n_cells0"] == o.m_hist[0], what
    np.testing.assert_array_equal(g.labels.cpu().numpy(), o.labels, err_msg=what)
    np.testing.assert_array_equal(g.counts.cpu().numpy(), o.counts, err_msg=what)
    np.testing.assert_array_equal(g.keys.cpu().numpy(), o.keys, err_msg=what)
    np.testing.assert_array_equal(_bits(g.sums.cpu().numpy()), _bits(o.sums), err_msg=what)
    np.testing.assert_array_equal(_bits(g.modes.cpu().numpy()), _bits(o.modes), err_msg=what)
    return g, o


def device_error(x_np, h):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    with pytest.raises(gridshift.GridShiftError) as e:
        gridshift.fit(x, h, 100, ctx=_ctx())
    return e.value.code


def _blobs(seed, n, d, k=8, scale=5.0, spread=12.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, spread * scale, size=(k, d))
    lab = rng.integers(0, k, size=n)
    return c[lab] + scale * 0.8 * rng.standard_normal(size=(n, d))


def _corner(origin):
    """Five points in four mutually adjacent cells and one cell two away:
    one merging round, then a converged pair."""
    o = np.asarray(origin, dtype=np.float64)
    d = o.size
    e = np.eye(d)
    pts = [o + 0.5, o + 0.5 + e[0], o + 0.5 + e[-1], o + 0.25 + e[0] + e[-1], o + 0.5 + 3 * e[0]]
    return np.array(pts)


# ---------------------------------------------------------------------------
# cells 2^32 apart: 64-bit tail coordinates (a 32-bit difference wraps to 0)
# ---------------------------------------------------------------------------
def test_two_cells_2_32_apart_1d():
    g, o = parity(np.array([[0.5], [2.0**32 + 0.5]]), 1.0, what="1-D, 2^32 apart")
    assert (o.K, o.n_iter, o.flags) == (2, 0, gs_oracle.CONVERGED)


def test_long_axis_is_dimension_1():
    x = np.concatenate([_corner([0.0, 0.0]), _corner([0.0, 2.0**32]), _corner([6.0, 2.0**33])])
    g, o = parity(x, 1.0, what="2-D, extent 2^33 along dimension 1")
    assert o.n_iter >= 1 and o.K == 6


@pytest.mark.parametrize("rule", ["parallel", "sequential"])
def test_wide_coordinates_sequential_and_parallel(rule):
    # extents about 2^33.3 x 12 x 2^20 (below 2^62 cells in all)
    x = np.concatenate([_corner([0.0, 0.0, 0.0]), _corner([2.0**33, 5.0, 2.0**20]),
                        _corner([-(2.0**31), 3.0, 7.0])])
    parity(x, 1.0, what=f"3-D, extents above 2^31 ({rule})", rule=rule)


# ---------------------------------------------------------------------------
# 64-bit keys, hash lookups, linear rank
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("far,what", [(2.0**12, "span about 2^36: 64-bit keys, packed rank"),
                                      (2.0**20, "span about 2^60: 64-bit keys, linear rank")])
@pytest.mark.parametrize("merge_small", [1, 0])
def test_wide_key_space_with_device_wide_rounds(far, what, merge_small):
    # about 20K points in 3-D at h = 1: several thousand initial cells (device-
    # wide rounds with 64-bit keys through the hash), then the tail; two far
    # corners stretch the key box beyond 32 bits
    x = np.concatenate([_blobs(7100, 20000, 3, k=10, scale=3.0, spread=12.0),
                        _corner([far, far, far]), _corner([-far, 3.0, far])])
    g, o = parity(x, 1.0, what=what, merge_small=merge_small)
    assert o.m_hist[0] > 1024


def test_wide_key_space_f32_4d():
    x = np.concatenate([_blobs(7101, 30000, 4, k=12, scale=2.0, spread=10.0),
                        _corner([-3000.0, 0.0, 4000.0, 0.0])]).astype(np.float32)
    g, o = parity(x, 1.0, what="4-D f32, span above 2^32")
    assert o.m_hist[0] > 1024


# ---------------------------------------------------------------------------
# more than 4096 columns along dimension 0: the tail's binary-search window
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [1, 2, 3])
def test_many_columns_along_dimension_0(d):
    rng = np.random.default_rng(7200 + d)
    centres = np.zeros((60, d))
    centres[:, 0] = np.sort(rng.uniform(0.0, 20000.0, size=60))
    if d > 1:
        centres[:, 1:] = rng.uniform(0.0, 6.0, size=(60, d - 1))
    lab = rng.integers(0, 60, size=6000)
    x = centres[lab] + 0.9 * rng.standard_normal(size=(6000, d))
    g, o = parity(x, 1.0, what=f"d={d}, about 20000 columns along dimension 0")
    assert o.n_iter >= 1


# ---------------------------------------------------------------------------
# the edges of the packed key space
# ---------------------------------------------------------------------------
def test_key_magnitude_edge_2_52():
    below = 2.0**52 - 0.5  # floor = 2^52 - 1
    x = np.concatenate([_corner([0.0]), np.array([[below], [below - 1.0], [-(2.0**52) + 1.0]])])
    parity(x, 1.0, what="|floor(x/h)| = 2^52 - 1")
    # |floor(x/h)| = 2^52: outside the packed key space of the device, inside
    # the oracle's int64 keys (the recorded difference)
    for v in (2.0**52, -(2.0**52)):
        edge = np.array([[0.5], [v]])
        assert device_error(edge, 1.0) == KEY_RANGE
        o = gs_oracle.fit(edge, 1.0, 100)
        assert o.K == 2 and o.flags == gs_oracle.CONVERGED


def test_key_box_edge_2_62():
    # per-dimension extent E_k = max_k - min_k + 3 (one spare cell per side)
    hi = 2.0**31 - 3.0  # E = 2^31
    ok = np.concatenate([_corner([0.0, 0.0]), _corner([hi - 3.0, hi - 2.0])])  # 2^31 x (2^31 - 1) cells
    assert np.floor(ok.max(axis=0)).tolist() == [hi, hi - 1.0]
    parity(ok, 1.0, what="key box 2^62 - 2^31 cells")
    full = np.concatenate([_corner([0.0, 0.0]), _corner([hi - 3.0, hi - 1.0])])  # 2^31 x 2^31 = 2^62
    assert np.floor(full.max(axis=0)).tolist() == [hi, hi]
    assert device_error(full, 1.0) == KEY_RANGE
    o = gs_oracle.fit(full, 1.0, 100)
    assert o.K == 4


# ---------------------------------------------------------------------------
# stop on an unchanged state
# ---------------------------------------------------------------------------
_K = 2.0**51
_S1 = np.array([[_K + 0.5], [_K + 0.5], [_K + 1.5], [_K + 2.0], [_K + 2.0], [_K + 2.0]])


@pytest.mark.parametrize("rule", ["parallel", "sequential"])
def test_stationary_in_the_tail(rule):
    g, o = parity(_S1, 1.0, what=f"stationary, one workgroup ({rule})", rule=rule)
    assert (o.n_iter, o.flags) == (1, gs_oracle.STATIONARY)


@pytest.mark.parametrize("rule,merge_small,dense", [("parallel", 1, 1), ("parallel", 0, 1), ("parallel", 1, 0),
                                                    ("sequential", 1, 1), ("sequential", 0, 0)])
def test_stationary_in_device_wide_rounds(rule, merge_small, dense):
    # 400 spaced copies: 1200 cells, so the round that stops runs device-wide
    x = np.concatenate([_S1 + 4.0 * j for j in range(400)])
    g, o = parity(x, 1.0, what=f"stationary, device-wide ({rule})", rule=rule, merge_small=merge_small,
                  dense_table=dense)
    assert (o.n_iter, o.flags, o.K) == (1, gs_oracle.STATIONARY, 1200)


def test_stationary_instances_in_a_batch():
    # a stationary instance next to converging ones, in one batched pass
    xs = [_S1, _blobs(7300, 3000, 1, k=4, scale=2.0, spread=8.0), np.concatenate([_S1 + 4.0 * j for j in range(400)])]
    off = np.concatenate([[0], np.cumsum([len(v) for v in xs])]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs)).to(DEV)
    br = gridshift.fit_batched(X, off, [1.0, 1.0, 1.0], 100, with_sums=True)
    labels = br.labels.cpu().numpy()
    sums = br.sums.cpu().numpy()
    for b, x in enumerate(xs):
        o = gs_oracle.fit(x, 1.0, 100)
        ko = slice(br.k_offsets[b], br.k_offsets[b + 1])
        assert (br.infos[b]["n_clusters"], br.infos[b]["n_iter"], br.infos[b]["flags"]) == (o.K, o.n_iter, o.flags)
        np.testing.assert_array_equal(labels[off[b]:off[b + 1]], o.labels)
        np.testing.assert_array_equal(_bits(sums[ko]), _bits(o.sums))
