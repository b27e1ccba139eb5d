"""The per-fit result API (gs_fit / gs_fit_batched -> gs_result) through the C
ABI, with the device memory taken from torch's caching allocator: bitwise
the same labels, modes, counts, summaries, adjoint and loss as the context
calls, every allocation returned on gs_result_free, and the errors."""
import ctypes
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


def _bits(t):
    return np.ascontiguousarray(t.detach().cpu().numpy().astype(np.float64)).view(np.uint64)


def _blobs(seed, n, d, k=8, scale=5.0, spread=12.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, spread * scale, size=(k, d))
    return c[rng.integers(0, k, size=n)] + scale * 0.8 * rng.standard_normal(size=(n, d))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("allocator", ["torch", None])
def test_plain_result_equals_context_fit(allocator):
    _say(f"result api plain, allocator={allocator}")
    w = synth.image_rgb_f64()
    x = torch.from_numpy(w.x).to(DEV)
    before = dict(gridshift.ALLOC_STATS)
    r = gridshift.fit_result(x, w.h, w.max_iter, allocator=allocator)
    c = gridshift.fit(x, w.h, w.max_iter)
    info = r.info(0)
    assert info == c.info
    assert r.offsets().tolist() == [0, c.info["n_clusters"]]
    modes, counts = r.copy()
    np.testing.assert_array_equal(r.labels.cpu().numpy(), c.labels.cpu().numpy())
    np.testing.assert_array_equal(_bits(modes), _bits(c.modes))
    np.testing.assert_array_equal(counts.cpu().numpy(), c.counts.cpu().numpy())
    used = gridshift.ALLOC_STATS["allocs"] - before["allocs"]
    r.close()
    torch.cuda.synchronize()
    if allocator == "torch":
        assert used > 0
        assert gridshift.ALLOC_STATS["frees"] - before["frees"] == used
    else:
        assert used == 0


def test_batched_result_equals_context_fit():
    _say("result api batched")
    sizes = [0, 300, 12000, 5, 40000]
    xs = [_blobs(6000 + i, s, 3) for i, s in enumerate(sizes)]
    hs = [2.0, 3.0, 1.5, 2.0, 2.5]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs, axis=0)).to(DEV)
    r = gridshift.fit_batched_result(X, off, hs, 100)
    c = gridshift.fit_batched(X, off, hs, 100)
    assert [r.info(b) for b in range(len(sizes))] == c.infos
    assert r.offsets().tolist() == c.k_offsets.tolist()
    modes, counts = r.copy()
    np.testing.assert_array_equal(r.labels.cpu().numpy(), c.labels.cpu().numpy())
    np.testing.assert_array_equal(_bits(modes), _bits(c.modes))
    with pytest.raises(RuntimeError, match="GS_ERR_INVALID_ARG"):
        r.info(len(sizes))
    r.close()


@pytest.mark.parametrize("ckpt", [1, 8])
def test_result_adjoint_and_loss_equal_context(ckpt):
    _say(f"result api adjoint, ckpt_every={ckpt}")
    x_np = _blobs(6100, 30000, 5, k=6, scale=4.0)
    x = torch.from_numpy(x_np).to(DEV)
    r = gridshift.fit_result(x, 3.0, 100, ckpt_every=ckpt)
    ctx = gridshift.Context(0)
    ctx.set_tape(ckpt)
    c = gridshift.fit(x, 3.0, 100, ctx=ctx)
    rng = np.random.default_rng(1)
    gm = torch.from_numpy(rng.standard_normal(size=(c.info["n_clusters"], 5))).to(DEV)
    np.testing.assert_array_equal(_bits(r.backward(gm)), _bits(gridshift.backward_modes(ctx, gm, 30000, 5)))
    loss_r = r.loss(x)
    loss_c = gridshift.point_mode_loss_values(ctx, x, c.labels, 1)
    np.testing.assert_array_equal(_bits(loss_r), _bits(loss_c))
    gl = torch.tensor([0.75], dtype=torch.float64, device=DEV)
    np.testing.assert_array_equal(_bits(r.loss_backward(x, gl)),
                                  _bits(gridshift.point_mode_loss_grad(ctx, x, c.labels, gl)))
    r.close()


def test_unrecorded_result_has_no_adjoint():
    x = torch.from_numpy(_blobs(6200, 2000, 2)).to(DEV)
    r = gridshift.fit_result(x, 2.0, 100)
    with pytest.raises(RuntimeError, match="GS_ERR_STATE"):
        r.backward(torch.zeros((r.info()["n_clusters"], 2), dtype=torch.float64, device=DEV))
    r.close()


def test_result_loss_with_column_sliced_points():
    # points as a column slice of a wider tensor (row stride 5, d = 3): the
    # loss and its gradient read the rows with the fit's stride, bitwise as a
    # fit of the dense copy
    _say("result api loss, column-sliced points")
    wide = torch.from_numpy(_blobs(6300, 20000, 5, k=6, scale=4.0)).to(DEV)
    view = wide[:, :3]
    dense = view.contiguous()
    r = gridshift.fit_result(view, 3.0, 100, ckpt_every=1)
    q = gridshift.fit_result(dense, 3.0, 100, ckpt_every=1)
    assert r.info() == q.info()
    np.testing.assert_array_equal(_bits(r.loss(view)), _bits(q.loss(dense)))
    gl = torch.tensor([1.25], dtype=torch.float64, device=DEV)
    np.testing.assert_array_equal(_bits(r.loss_backward(view, gl)), _bits(q.loss_backward(dense, gl)))
    with pytest.raises(ValueError, match="layout"):
        r.loss(dense)  # same values, another row stride
    with pytest.raises(ValueError, match="layout"):
        q.loss(view.to(torch.float32))
    r.close()
    q.close()


@pytest.mark.parametrize("ckpt", [0, 8])
def test_allocation_failure_returns_every_allocation(ckpt):
    # the caller's allocator fails at its k-th call, for every k a clean fit
    # reaches: gs_fit returns GS_ERR_ALLOC, no result, and every allocation
    # it made has been given back
    _say(f"result api allocation failure, ckpt_every={ckpt}")
    x = torch.from_numpy(_blobs(6400, 30000, 3, k=6, scale=4.0)).to(DEV)
    lib = gridshift.load_library()
    st = {"calls": 0, "fail_at": None, "live": set()}

    def alloc(ctx, nbytes, stream):
        st["calls"] += 1
        if st["fail_at"] is not None and st["calls"] == st["fail_at"]:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        st["live"].add(p)
        return p

    def free(ctx, p, stream):
        st["live"].remove(int(p))
        torch.cuda.caching_allocator_delete(int(p))

    al = gridshift.Allocator(gridshift._ALLOC_FN(alloc), gridshift._FREE_FN(free), None)
    labels = torch.empty(x.shape[0], dtype=torch.int32, device=DEV)
    p = gridshift.Problem(x.data_ptr(), gridshift.GS_F64, x.shape[0], 3, 3, 3.0, 100, ckpt)
    sp = gridshift._stream_ptr(None)
    out = ctypes.c_void_p()
    assert lib.gs_fit(ctypes.byref(p), ctypes.byref(al), sp, labels.data_ptr(), ctypes.byref(out)) == 0
    n_calls = st["calls"]
    assert n_calls >= 1 and st["live"]
    lib.gs_result_free(out)
    assert not st["live"]
    for k in range(1, n_calls + 1):
        st.update(calls=0, fail_at=k)
        out = ctypes.c_void_p()
        rc = lib.gs_fit(ctypes.byref(p), ctypes.byref(al), sp, labels.data_ptr(), ctypes.byref(out))
        assert gridshift.STATUS[rc] == "GS_ERR_ALLOC", (k, rc)
        assert not out.value
        assert not st["live"], k
    torch.cuda.synchronize()


def test_result_calls_on_another_stream():
    # copies, loss and adjoint queued on a second stream, then the result
    # released without waiting: the same bits as on the fit's stream
    _say("result api, calls on a second stream")
    x = torch.from_numpy(_blobs(6500, 30000, 5, k=6, scale=4.0)).to(DEV)
    r = gridshift.fit_result(x, 3.0, 100, ckpt_every=8)
    modes_a, counts_a = r.copy()
    gm = torch.from_numpy(np.random.default_rng(2).standard_normal(size=(r.info()["n_clusters"], 5))).to(DEV)
    grad_a = r.backward(gm)
    loss_a = r.loss(x)
    s2 = torch.cuda.Stream()
    sp2 = ctypes.c_void_p(s2.cuda_stream)
    lib = gridshift.load_library()
    with torch.cuda.stream(s2):
        tot = int(r.offsets()[-1])
        modes_b = torch.empty((tot, 5), dtype=torch.float64, device=DEV)
        counts_b = torch.empty(tot, dtype=torch.int64, device=DEV)
        grad_b = torch.empty((x.shape[0], 5), dtype=torch.float64, device=DEV)
        loss_b = torch.empty(1, dtype=torch.float64, device=DEV)
        g2 = gm.clone()
        assert lib.gs_result_copy(r.handle, modes_b.data_ptr(), counts_b.data_ptr(), sp2) == 0
        assert lib.gs_backward(r.handle, g2.data_ptr(), grad_b.data_ptr(), sp2) == 0
        assert lib.gs_point_mode_loss(r.handle, x.data_ptr(), loss_b.data_ptr(), sp2) == 0
    r.close()
    s2.synchronize()
    np.testing.assert_array_equal(_bits(modes_b), _bits(modes_a))
    np.testing.assert_array_equal(counts_b.cpu().numpy(), counts_a.cpu().numpy())
    np.testing.assert_array_equal(_bits(grad_b), _bits(grad_a))
    np.testing.assert_array_equal(_bits(loss_b), _bits(loss_a))


def test_current_stream_handle():
    # the binding reads the current stream's raw handle (no Stream object per
    # call): it must be torch's current stream, on the default stream and
    # inside a `torch.cuda.stream` block
    _say("binding: current stream handle")
    assert (gridshift._stream_ptr(None).value or 0) == torch.cuda.current_stream().cuda_stream
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        assert (gridshift._stream_ptr(None).value or 0) == s2.cuda_stream
        x = torch.from_numpy(_blobs(6600, 5000, 3)).to(DEV)
        r = gridshift.fit(x, 3.0, 100)  # queued on s2
    s2.synchronize()
    o = gs_oracle.fit(x.cpu().numpy(), 3.0, 100)
    np.testing.assert_array_equal(r.labels.cpu().numpy(), o.labels)
