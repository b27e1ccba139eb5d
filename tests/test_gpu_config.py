"""Launch configurations and the autotuner.

Every configuration runs the same binary64 operations in the same order, so
labels, counts, keys, sums and modes must be bitwise identical under all of
them (and equal to the oracle).  The inputs are chosen so that fits pass
through both merge paths: rounds with more than 8192 cells (device-wide
merge), rounds with 1025..8192 cells (one-workgroup merge when enabled) and
the tail.
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
CONFIGS = [dict(merge_small=ms, tile_chunks=tc, dense_table=dt, sort_digit10=sd, sort_tile=st)
           for ms in (1, 0) for dt in (1, 0) for tc in (1, 8) for sd in (1, 0) for st in (8192, 4096)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _bits(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).view(np.uint64)


def _blobs(seed, n, d, k=8, scale=5.0, spread=12.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, spread * scale, size=(k, d))
    lab = rng.integers(0, k, size=n)
    return c[lab] + scale * 0.8 * rng.standard_normal(size=(n, d))


CASES = [
    ("d3_f64_h3", _blobs(800, 60000, 3, k=30, scale=8.0, spread=20.0), 3.0, np.float64),
    ("d2_f32_h1.5", _blobs(801, 100000, 2, k=20, scale=8.0, spread=20.0), 1.5, np.float32),
    ("d4_f64_h4", _blobs(802, 80000, 4, k=20, scale=6.0, spread=20.0), 4.0, np.float64),
]


@pytest.mark.parametrize("name,x,h,dtype", CASES, ids=[c[0] for c in CASES])
def test_every_configuration_gives_the_same_fit(name, x, h, dtype):
    x = x.astype(dtype)
    o = gs_oracle.fit(x.astype(np.float64), h, 100)
    _say(f"{name}: cells per round {o.m_hist[:8].tolist()} rounds={o.n_iter}")
    assert o.m_hist[0] > 8192 or any(1024 < m <= 8192 for m in o.m_hist)
    xt = torch.from_numpy(x).to(DEV)
    ctx = gridshift.Context(0)
    for cfg in CONFIGS:
        ctx.set_config(**cfg)
        assert ctx.config() == cfg
        r = gridshift.fit(xt, h, 100, ctx=ctx, with_sums=True, with_keys=True)
        what = f"{name} {cfg}"
        assert (r.info["n_clusters"], r.info["n_iter"], r.info["flags"]) == (o.K, o.n_iter, o.flags), what
        np.testing.assert_array_equal(r.labels.cpu().numpy(), o.labels, err_msg=what)
        np.testing.assert_array_equal(r.counts.cpu().numpy(), o.counts, err_msg=what)
        np.testing.assert_array_equal(r.keys.cpu().numpy(), o.keys, err_msg=what)
        np.testing.assert_array_equal(_bits(r.sums.cpu().numpy()), _bits(o.sums), err_msg=what)
    ctx.close()


def test_batched_under_both_merge_paths():
    xs = [CASES[0][1], _blobs(810, 3000, 3), _blobs(811, 0, 3), _blobs(812, 40000, 3, k=20, scale=8.0, spread=20.0)]
    hs = [3.0, 2.0, 1.0, 2.5]
    off = np.concatenate([[0], np.cumsum([len(v) for v in xs])]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs, axis=0)).to(DEV)
    ref = [gs_oracle.fit(v, h, 100) for v, h in zip(xs, hs)]
    ctx = gridshift.Context(0)
    for ms, dt, sd, st in ((1, 1, 1, 8192), (0, 0, 1, 4096), (1, 0, 0, 4096), (0, 1, 0, 8192)):
        ctx.set_config(merge_small=ms, dense_table=dt, sort_digit10=sd, sort_tile=st)
        br = gridshift.fit_batched(X, off, hs, 100, ctx=ctx, with_sums=True)
        sums = br.sums.cpu().numpy()
        for b, o in enumerate(ref):
            ko = slice(br.k_offsets[b], br.k_offsets[b + 1])
            assert br.infos[b]["n_iter"] == o.n_iter and br.infos[b]["n_clusters"] == o.K
            np.testing.assert_array_equal(br.labels[off[b]:off[b + 1]].cpu().numpy(), o.labels)
            np.testing.assert_array_equal(_bits(sums[ko]), _bits(o.sums))
    ctx.close()


def test_backward_under_both_merge_paths():
    x = CASES[0][1]
    xt = torch.from_numpy(x).to(DEV)
    res, tape = gs_oracle.fit_tape(x, 3.0)
    mubar = np.random.default_rng(9).standard_normal(size=(res.K, 3))
    want = tape.point_adjoint(mubar)
    for ms in (1, 0):
        ctx = gridshift.Context(0)
        ctx.set_config(merge_small=ms)
        ctx.set_tape(True)
        gridshift.fit(xt, 3.0, 100, ctx=ctx)
        g = gridshift.backward_modes(ctx, torch.from_numpy(mubar).to(DEV), x.shape[0], 3).cpu().numpy()
        np.testing.assert_array_equal(_bits(g), _bits(want))
        ctx.close()


def test_autotune_keeps_a_candidate_and_results():
    x, h = CASES[0][1], CASES[0][2]
    xt = torch.from_numpy(x).to(DEV)
    ctx = gridshift.Context(0)
    cfg = ctx.autotune(xt, h, 100, reps=2)
    _say(f"autotuned configuration: {cfg}")
    assert cfg["merge_small"] in (0, 1) and cfg["dense_table"] in (0, 1) and cfg["tile_chunks"] in (1, 2, 4, 8)
    assert cfg["sort_digit10"] in (0, 1) and cfg["sort_tile"] in (8192, 4096)
    o = gs_oracle.fit(x, h, 100)
    r = gridshift.fit(xt, h, 100, ctx=ctx)
    np.testing.assert_array_equal(r.labels.cpu().numpy(), o.labels)
    ctx.close()


def test_autotune_choice_is_kept_per_shape(tmp_path, monkeypatch):
    # a shape tuned once is not tuned again: a second context takes the same
    # configuration from the process's cache at once, and the choice is
    # appended to the file GRIDSHIFT_TUNE_CACHE names
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GRIDSHIFT_TUNE_CACHE", str(path))
    x = _blobs(820, 30000, 5, k=12, scale=6.0, spread=20.0)
    xt = torch.from_numpy(x).to(DEV)
    import time

    c1 = gridshift.Context(0)
    t0 = time.perf_counter()
    cfg1 = c1.autotune(xt, 3.0, 100, reps=1)
    t1 = time.perf_counter()
    c2 = gridshift.Context(0)
    cfg2 = c2.autotune(xt, 3.0, 100, reps=1)
    t2 = time.perf_counter()
    _say(f"tuned in {t1 - t0:.3f} s, cached in {t2 - t1:.4f} s: {cfg1}")
    assert cfg2 == cfg1
    assert (t2 - t1) < 0.2 * (t1 - t0)
    lines = [ln.split() for ln in path.read_text().splitlines()]
    # device d dtype logB logN merge_small dense_table tile_chunks sort_digit10 sort_tile ms
    mine = [ln for ln in lines if ln[1] == "5" and ln[2] == "1" and ln[3] == "0" and ln[4] == str(30000 .bit_length() - 1)]
    assert mine and [int(v) for v in mine[-1][5:10]] == [cfg1[k] for k in ("merge_small", "dense_table", "tile_chunks",
                                                                            "sort_digit10", "sort_tile")]
    c1.close()
    c2.close()


def test_configuration_errors():
    ctx = gridshift.Context(0)
    for kv in (dict(merge_small=2), dict(tile_chunks=0), dict(tile_chunks=65), dict(dense_table=-1),
               dict(sort_digit10=2), dict(sort_tile=2048)):
        with pytest.raises(gridshift.GridShiftError) as e:
            ctx.set_config(**kv)
        assert e.value.code == 1
    assert gridshift._lib.gs_context_set_config(ctx.handle, 7, 1) == 1  # unknown key
    assert ctx.config() == {"merge_small": 1, "tile_chunks": 4, "dense_table": 1, "sort_digit10": 0,
                            "sort_tile": 8192}
    ctx.close()


def test_context_reuse_across_inputs():
    # One context fits several different inputs in a row; state a fit leaves
    # behind (dense-table epochs, histogram buffers, tile counters) must never
    # leak into the next one.
    seq = [CASES[0], CASES[2], CASES[1], CASES[0]]
    ctx = gridshift.Context(0)
    for name, x, h, dtype in seq:
        x = x.astype(dtype)
        o = gs_oracle.fit(x.astype(np.float64), h, 100)
        r = gridshift.fit(torch.from_numpy(x).to(DEV), h, 100, ctx=ctx, with_sums=True)
        assert (r.info["n_clusters"], r.info["n_iter"], r.info["flags"]) == (o.K, o.n_iter, o.flags), name
        np.testing.assert_array_equal(r.labels.cpu().numpy(), o.labels, err_msg=name)
        np.testing.assert_array_equal(_bits(r.sums.cpu().numpy()), _bits(o.sums), err_msg=name)
    ctx.close()
