"""GPU bandwidth sweep (gs_fit_hsweep): one batched pass over many h values
against the FP64 oracle run once per h, bit-exact (labels, counts, rounds,
flags, sums), on a clustering set scaled into [0,1]^d with h over (0,1]."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import gs_oracle  # noqa: E402
from paper_2206_02200_amd import gridshift, synth  # noqa: E402

DEV = torch.device("cuda:0")


def _bits(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).view(np.uint64)


def _check_sweep(x_np, hs, max_iter=100, ld_pad=0, what=""):
    print(f"hsweep case {what}: n={x_np.shape[0]} d={x_np.shape[1]} H={len(hs)} pad={ld_pad}", flush=True)
    sys.stdout.flush()
    n, d = x_np.shape
    if ld_pad:
        buf = torch.zeros((n, d + ld_pad), dtype=torch.from_numpy(x_np).dtype, device=DEV)
        buf[:, :d] = torch.from_numpy(x_np).to(DEV)
        x = buf[:, :d]
    else:
        x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    r = gridshift.fit_hsweep(x, hs, max_iter, with_sums=True)
    labels = r.labels.cpu().numpy()
    sums = r.sums.cpu().numpy()
    counts = r.counts.cpu().numpy()
    assert labels.shape == (len(hs), n)
    for j, h in enumerate(hs):
        o = gs_oracle.fit(x_np.astype(np.float64), float(h), max_iter)
        ko = slice(r.k_offsets[j], r.k_offsets[j + 1])
        assert r.infos[j]["n_clusters"] == o.K, (what, h)
        assert r.infos[j]["n_iter"] == o.n_iter and r.infos[j]["flags"] == o.flags, (what, h)
        np.testing.assert_array_equal(labels[j], o.labels, err_msg=f"{what} h={h}")
        np.testing.assert_array_equal(counts[ko], o.counts, err_msg=f"{what} h={h}")
        np.testing.assert_array_equal(_bits(sums[ko]), _bits(o.sums), err_msg=f"{what} h={h}")
    return r


def test_sweep_grid_f32():
    x = synth.unit_gmm_f32(20000, 3, seed=90)
    _check_sweep(x, synth.hsweep_grid(20), what="unit gmm d=3 f32")


def test_sweep_fine_grid_with_wide_rounds_f32():
    # h = 0.01 gives well over a tail workgroup's 1024 cells
    x = synth.unit_gmm_f32(60000, 3, seed=91)
    r = _check_sweep(x, [0.01, 0.015, 0.5], what="fine h")
    assert r.infos[0]["n_cells0"] > 4096


def test_sweep_strided_f64_rows():
    x = synth.unit_gmm_f32(5000, 4, seed=92).astype(np.float64)
    _check_sweep(x, [0.05, 0.1, 0.2, 0.4, 0.8], ld_pad=3, what="strided f64 d=4")


def test_sweep_equals_plain_fits():
    x_np = synth.unit_gmm_f32(10000, 2, seed=93)
    x = torch.from_numpy(x_np).to(DEV)
    hs = [0.03, 0.07, 0.3]
    r = gridshift.fit_hsweep(x, hs, 100, with_sums=True)
    for j, h in enumerate(hs):
        p = gridshift.fit(x, h, 100, with_sums=True)
        np.testing.assert_array_equal(r.labels[j].cpu().numpy(), p.labels.cpu().numpy())
        ko = slice(r.k_offsets[j], r.k_offsets[j + 1])
        np.testing.assert_array_equal(_bits(r.sums[ko].cpu().numpy()), _bits(p.sums.cpu().numpy()))


def test_sweep_of_many_positions_equals_plain_fits():
    # 200,000 points x 42 bandwidths = 8.4M positions: the sweep looks every
    # position's initial cell up from its key (2^23 positions or more), the
    # plain fits of 200,000 points scatter it from the heads scan
    x_np = synth.unit_gmm_f32(200_000, 3, seed=94)
    x = torch.from_numpy(x_np).to(DEV)
    hs = synth.hsweep_grid(42)
    assert x_np.shape[0] * len(hs) >= 1 << 23
    print("hsweep case: 200000 points x 42 bandwidths against plain fits", flush=True)
    r = gridshift.fit_hsweep(x, hs, 100, with_sums=True)
    for j, h in enumerate(hs):
        p = gridshift.fit(x, float(h), 100, with_sums=True)
        np.testing.assert_array_equal(r.labels[j].cpu().numpy(), p.labels.cpu().numpy(), err_msg=f"h={h}")
        ko = slice(r.k_offsets[j], r.k_offsets[j + 1])
        np.testing.assert_array_equal(_bits(r.sums[ko].cpu().numpy()), _bits(p.sums.cpu().numpy()), err_msg=f"h={h}")
    o = gs_oracle.fit(x_np.astype(np.float64), float(hs[0]), 100)  # the finest bandwidth against the oracle
    np.testing.assert_array_equal(r.labels[0].cpu().numpy(), o.labels)


def test_sweep_single_h_and_empty():
    x = synth.unit_gmm_f32(3000, 3, seed=94)
    _check_sweep(x, [0.25], what="one h")
    e = torch.empty((0, 3), dtype=torch.float32, device=DEV)
    r = gridshift.fit_hsweep(e, [0.1, 0.2], 100)
    assert r.labels.shape == (2, 0) and all(i["n_clusters"] == 0 for i in r.infos)
    with pytest.raises(RuntimeError):
        gridshift.fit_hsweep(torch.from_numpy(x).to(DEV), [0.1, -1.0], 100)


def test_sweep_64_bit_keys():
    # d = 6 and h = 0.01 over the unit cube: about 103^6 keys per bandwidth,
    # so the sweep's keys are 64-bit
    x = synth.unit_gmm_f32(3000, 6, seed=95)
    _check_sweep(x, [0.01, 0.02, 0.6], what="d=6 64-bit keys")


def test_sweep_refuses_a_recording_context():
    x = torch.from_numpy(synth.unit_gmm_f32(2000, 3, seed=96)).to(DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(True)
    with pytest.raises(gridshift.GridShiftError) as e:
        gridshift.fit_hsweep(x, [0.1, 0.2], 100, ctx=ctx)
    assert e.value.code == 6  # GS_ERR_UNSUPPORTED
    ctx.close()
