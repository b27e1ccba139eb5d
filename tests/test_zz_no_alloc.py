"""gs_fit_noalloc (the plain fit whose device scratch is the library's fixed
array) through the C ABI: bitwise the labels, summary, modes and counts of
gs_fit on the same input, call after call on the one shared array, at the
largest size it takes, and its errors."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2206_02200_amd import gridshift, synth  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bits(t):
    return np.ascontiguousarray(t.detach().cpu().numpy().astype(np.float64)).view(np.uint64)


def _blobs(seed, n, d, k=8, scale=5.0, spread=12.0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, spread * scale, size=(k, d))
    return (c[rng.integers(0, k, size=n)] + scale * 0.8 * rng.standard_normal(size=(n, d))).astype(dtype)


def _check_equal(x, h, max_iter=100):
    """gs_fit_noalloc against gs_fit (hipMalloc'd result) on the same points."""
    a = gridshift.fit_noalloc(x, h, max_iter)
    r = gridshift.fit_result(x, h, max_iter, allocator=None)
    info = r.info(0)
    assert a.info == info
    modes, counts = r.copy()
    np.testing.assert_array_equal(a.labels.cpu().numpy(), r.labels.cpu().numpy())
    np.testing.assert_array_equal(_bits(a.modes), _bits(modes))
    np.testing.assert_array_equal(a.counts.cpu().numpy(), counts.cpu().numpy())
    r.close()
    return info


def test_two_calls_in_a_row_equal_gs_fit():
    # the 160x120 RGB float64 image, then a smaller float32 set with d = 5:
    # the second call overwrites what the first left in the array
    w = synth.image_rgb_f64()
    _say(f"noalloc call 1: {w.name} n={len(w.x)}")
    info1 = _check_equal(torch.from_numpy(w.x).to(DEV), w.h, w.max_iter)
    assert info1["n_clusters"] > 1
    x2 = torch.from_numpy(_blobs(71, 5003, 5, k=5, scale=3.0, dtype=np.float32)).to(DEV)
    _say("noalloc call 2: blobs n=5003 d=5 f32")
    info2 = _check_equal(x2, 2.0)
    assert info2["n_points"] == 5003 and info2["n_clusters"] >= 1
    # and the first input again, after the smaller one
    _say("noalloc call 3: the image again")
    assert _check_equal(torch.from_numpy(w.x).to(DEV), w.h, w.max_iter) == info1


def test_largest_input_every_point_its_own_cell():
    # 2^17 points on a 8x8x8x8x8x4 lattice of cell centres (d = 6, float64,
    # h = 1): every point is its own cell and every cell has neighbours, so
    # the first rounds run device-wide on all 131072 cells (the worst case the
    # fixed array is sized for)
    n = gridshift.NOALLOC_MAX_POINTS
    idx = np.arange(n)
    dims = [8, 8, 8, 8, 8, 4]
    coords = []
    for e in reversed(dims):
        coords.append(idx % e)
        idx = idx // e
    x = np.stack(coords[::-1], axis=1).astype(np.float64) + 0.5
    _say(f"noalloc lattice n={n} d=6")
    info = _check_equal(torch.from_numpy(x).to(DEV), 1.0, 100)
    assert info["n_cells0"] == n and info["n_iter"] >= 1


def test_largest_input_with_64_bit_keys():
    # 2^17 points spread over a key box of about 2^36 cells (d = 6): 64-bit
    # keys in the binning sort
    rng = np.random.default_rng(72)
    x = rng.uniform(0.0, 64.0, size=(gridshift.NOALLOC_MAX_POINTS, 6))
    _say("noalloc wide keys n=131072 d=6")
    info = _check_equal(torch.from_numpy(x).to(DEV), 1.0, 100)
    assert info["n_cells0"] > 100000


def test_empty_and_single_point():
    _say("noalloc empty / single")
    x0 = torch.empty((0, 3), dtype=torch.float32, device=DEV)
    a = gridshift.fit_noalloc(x0, 1.0)
    assert a.info["n_clusters"] == 0 and a.info["n_iter"] == 0
    x1 = torch.tensor([[1.5, -2.5]], dtype=torch.float64, device=DEV)
    a = gridshift.fit_noalloc(x1, 1.0)
    assert a.info["n_clusters"] == 1 and a.labels.tolist() == [0]
    assert a.modes.cpu().tolist() == [[1.5, -2.5]] and a.counts.tolist() == [1]


def test_errors():
    _say("noalloc errors")
    big = torch.zeros((gridshift.NOALLOC_MAX_POINTS + 1, 2), dtype=torch.float32, device=DEV)
    with pytest.raises(RuntimeError, match="GS_ERR_INVALID_ARG.*at most 131072 points"):
        gridshift.fit_noalloc(big, 1.0)
    x = torch.from_numpy(_blobs(73, 3000, 3)).to(DEV)
    ref = gridshift.fit_noalloc(x, 2.0)
    K = ref.info["n_clusters"]
    assert K > 1
    labels = torch.full((3000,), -1, dtype=torch.int32, device=DEV)
    modes = torch.full((K - 1, 3), 7.0, dtype=torch.float64, device=DEV)
    counts = torch.full((K - 1,), 7, dtype=torch.int64, device=DEV)
    with pytest.raises(RuntimeError, match="GS_ERR_INVALID_ARG.*clusters"):
        gridshift.fit_noalloc(x, 2.0, labels=labels, modes=modes, counts=counts)
    # labels written, modes and counts untouched
    np.testing.assert_array_equal(labels.cpu().numpy(), ref.labels.cpu().numpy())
    assert bool((modes == 7.0).all()) and bool((counts == 7).all())
    p = gridshift.Problem(x.data_ptr(), gridshift.GS_F64, 3000, 3, 3, 2.0, 100, 1)
    info = gridshift.Info()
    lib = gridshift.load_library()
    rc = lib.gs_fit_noalloc(p, None, labels.data_ptr(), None, None, 0, info)
    assert gridshift.STATUS[rc] == "GS_ERR_UNSUPPORTED"
