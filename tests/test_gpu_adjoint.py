"""GPU parity of the differentiable form (adjoint along a fixed trajectory).

The HIP backward runs the same binary64 recursion in the same order as the
oracle's gso_tape_adjoint (q_j = (C_j * Sbar_g(j)) / W_j, then a left fold in
ascending neighbour key), so gradients are compared bitwise; the point-to-mode
loss and its gradient likewise.  The gradient is also checked against central
finite differences of the loss, evaluated in binary128 along the same
trajectory, at perturbations whose FP64 fits follow the identical discrete path
(bar: 1e-6 relative).
"""
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


def _gpu_backward(x_np, h, mubar_fn, max_iter=100):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(True)
    r = gridshift.fit(x, h, max_iter, ctx=ctx)
    mubar = mubar_fn(r.modes.shape)
    g = gridshift.backward_modes(ctx, torch.from_numpy(mubar).to(DEV), x.shape[0], x.shape[1])
    torch.cuda.synchronize()
    return r, mubar, g.cpu().numpy(), ctx


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_backward_bitwise_vs_oracle(d):
    _say(f"adjoint d={d}")
    x = _blobs(700 + d, 6000, d)
    rng = np.random.default_rng(d)
    r, mubar, g, _ = _gpu_backward(x, 3.0, lambda s: rng.standard_normal(size=s))
    res, tape = gs_oracle.fit_tape(x, 3.0)
    assert res.K == r.info["n_clusters"] and res.n_iter == r.info["n_iter"]
    np.testing.assert_array_equal(_bits(g), _bits(tape.point_adjoint(mubar)))


def test_backward_with_wide_rounds_f32():
    _say("adjoint wide rounds f32")
    x = _blobs(710, 150000, 3, k=30, scale=8.0, spread=20.0).astype(np.float32)
    rng = np.random.default_rng(3)
    r, mubar, g, _ = _gpu_backward(x, 1.0, lambda s: rng.standard_normal(size=s))
    res, tape = gs_oracle.fit_tape(x.astype(np.float64), 1.0)
    assert res.m_hist[0] > 1024
    want = tape.point_adjoint(mubar)
    bad = np.nonzero(_bits(g) != _bits(want))
    if len(bad[0]):
        _say(f"rounds={res.n_iter} m_hist={res.m_hist.tolist()[:8]} gpu_info={r.info}")
        for i, k in zip(*bad):
            c0 = tape.cell0[i]
            _say(f"point {i} dim {k} cell0 {c0} count0 {tape.rounds[0]['counts'][c0]} gpu {g[i, k]!r} oracle {want[i, k]!r}")
    np.testing.assert_array_equal(_bits(g), _bits(want))


def test_backward_capped_and_zero_rounds():
    rng = np.random.default_rng(4)
    for x, h, mi in [(_blobs(711, 3000, 2), 2.0, 3), (np.array([[0.5, 0.5], [5.5, 5.5]]), 1.0, 100)]:
        r, mubar, g, _ = _gpu_backward(x, h, lambda s: rng.standard_normal(size=s), max_iter=mi)
        res, tape = gs_oracle.fit_tape(x, h, mi)
        np.testing.assert_array_equal(_bits(g), _bits(tape.point_adjoint(mubar)))


def test_backward_batched():
    sizes = [5000, 0, 1, 120000, 800]
    xs = [_blobs(720 + i, s, 3, k=30 if s > 100000 else 8, scale=8.0 if s > 100000 else 5.0,
                 spread=20.0 if s > 100000 else 12.0) for i, s in enumerate(sizes)]
    hs = [2.0, 1.0, 1.0, 1.0, 3.0]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs, axis=0)).to(DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(True)
    br = gridshift.fit_batched(X, off, hs, 100, ctx=ctx)
    rng = np.random.default_rng(5)
    mubar = rng.standard_normal(size=tuple(br.modes.shape))
    g = gridshift.backward_modes(ctx, torch.from_numpy(mubar).to(DEV), X.shape[0], 3).cpu().numpy()
    for b, (x, h) in enumerate(zip(xs, hs)):
        _say(f"batched adjoint instance {b} n={len(x)}")
        res, tape = gs_oracle.fit_tape(x, h)
        mb = mubar[br.k_offsets[b]:br.k_offsets[b + 1]]
        np.testing.assert_array_equal(_bits(g[off[b]:off[b + 1]]), _bits(tape.point_adjoint(mb)))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_loss_and_gradient_bitwise(dtype):
    x = _blobs(730, 40000, 5).astype(dtype)
    xt = torch.from_numpy(x).to(DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(True)
    r = gridshift.fit(xt, 4.0, 100, ctx=ctx)
    L = gridshift.point_mode_loss_values(ctx, xt, r.labels, 1).cpu().numpy()
    g = gridshift.point_mode_loss_grad(ctx, xt, r.labels, torch.ones(1, dtype=torch.float64, device=DEV))
    Lo, go, res, tape = gs_oracle.loss_and_grad(x.astype(np.float64), 4.0)
    assert _bits(L[0]) == _bits(Lo)
    np.testing.assert_array_equal(_bits(g.cpu().numpy()), _bits(go))


def test_loss_batched_against_oracle():
    sizes = [3000, 7000, 1]
    xs = [_blobs(740 + i, s, 2) for i, s in enumerate(sizes)]
    hs = [2.0, 3.0, 1.0]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = torch.from_numpy(np.concatenate(xs, axis=0)).to(DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(True)
    br = gridshift.fit_batched(X, off, hs, 100, ctx=ctx)
    L = gridshift.point_mode_loss_values(ctx, X, br.labels, len(sizes)).cpu().numpy()
    gl = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device=DEV)
    g = gridshift.point_mode_loss_grad(ctx, X, br.labels, gl).cpu().numpy()
    for b, (x, h) in enumerate(zip(xs, hs)):
        Lo, go, res, tape = gs_oracle.loss_and_grad(x, h)
        assert _bits(L[b]) == _bits(Lo)
        np.testing.assert_allclose(g[off[b]:off[b + 1]], float(gl[b]) * go, rtol=1e-13, atol=1e-13)


def test_gradient_against_binary128_finite_differences():
    # a small (x, y, L, a, b) Voronoi image with colour ramps
    rgb = synth.voronoi_rgb(48, 64, 6, 6.0, 64.0, seed=5077)
    x32 = synth.xy_lab_features(48, 64, rgb, 1.0)
    x = x32.astype(np.float64)
    h = 16.0
    xt = torch.from_numpy(x32).to(DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(True)
    r = gridshift.fit(xt, h, 100, ctx=ctx)
    assert r.info["n_iter"] >= 1
    g = gridshift.point_mode_loss_grad(ctx, xt, r.labels, torch.ones(1, dtype=torch.float64, device=DEV)).cpu().numpy()
    res, tape = gs_oracle.fit_tape(x, h)
    eps = 1e-4
    rng = np.random.default_rng(11)
    checked, worst = 0, 0.0
    for i in rng.choice(len(x), size=40, replace=False):
        for k in range(5):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += eps
            xm[i, k] -= eps
            _, tp = gs_oracle.fit_tape(xp, h)
            _, tm = gs_oracle.fit_tape(xm, h)
            if not (tape.same_trajectory(tp) and tape.same_trajectory(tm)):
                continue
            fd = tape.fd_q(x, i, k, eps)
            rel = abs(fd - g[i, k]) / max(abs(fd), 1e-30)
            worst = max(worst, rel if abs(fd) > 1e-8 else abs(fd - g[i, k]))
            checked += 1
    _say(f"finite differences checked={checked} worst={worst:.3e}")
    assert checked >= 50
    assert worst <= 1e-6


def test_autograd_functions():
    x = torch.from_numpy(_blobs(750, 20000, 3).astype(np.float32)).to(DEV).requires_grad_(True)
    loss = gridshift.point_mode_loss(x, 3.0)
    loss.sum().backward()
    assert x.grad is not None and x.grad.dtype == torch.float32
    ctx = gridshift.Context(0)
    ctx.set_tape(True)
    r = gridshift.fit(x.detach(), 3.0, 100, ctx=ctx)
    g = gridshift.point_mode_loss_grad(ctx, x.detach(), r.labels, torch.ones(1, dtype=torch.float64, device=DEV))
    assert torch.equal(x.grad, g.to(torch.float32))

    x2 = x.detach().double().requires_grad_(True)
    modes, labels, counts = gridshift.gridshift_modes(x2, 3.0)
    w = torch.randn_like(modes)
    (modes * w).sum().backward()
    ctx2 = gridshift.Context(0)
    ctx2.set_tape(True)
    gridshift.fit(x2.detach(), 3.0, 100, ctx=ctx2)
    g2 = gridshift.backward_modes(ctx2, w, x2.shape[0], 3)
    assert torch.equal(x2.grad, g2)
    assert not labels.requires_grad and not counts.requires_grad


def test_backward_needs_a_recorded_fit():
    ctx = gridshift.Context(0)
    x = torch.from_numpy(_blobs(760, 100, 2)).to(DEV)
    r = gridshift.fit(x, 2.0, 100, ctx=ctx)
    with pytest.raises(gridshift.GridShiftError) as e:
        gridshift.backward_modes(ctx, torch.ones_like(r.modes), 100, 2)
    assert e.value.code == 7


# ---------------------------------------------------------------------------
# checkpointed tail: segments recomputed in the backward pass
# ---------------------------------------------------------------------------
def _grads(x, off, hs, tape_mode, mubar_seed=6, max_iter=100):
    X = torch.from_numpy(x).to(DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(tape_mode)
    if off is None:
        r = gridshift.fit(X, hs, max_iter, ctx=ctx)
        K, labels, B = r.modes.shape[0], r.labels, 1
    else:
        r = gridshift.fit_batched(X, off, hs, max_iter, ctx=ctx)
        K, labels, B = r.modes.shape[0], r.labels, len(off) - 1
    mubar = np.random.default_rng(mubar_seed).standard_normal(size=(K, x.shape[1]))
    g = gridshift.backward_modes(ctx, torch.from_numpy(mubar).to(DEV), x.shape[0], x.shape[1]).cpu().numpy()
    gl = torch.linspace(0.5, 2.0, B, dtype=torch.float64, device=DEV)
    gL = gridshift.point_mode_loss_grad(ctx, X, labels, gl).cpu().numpy()
    ctx.close()
    return g, gL, mubar


@pytest.mark.parametrize("k", [2, 3, 8, 1000])
def test_checkpointed_backward_equals_full_tape(k):
    x = _blobs(770, 20000, 3)
    g1, gL1, mubar = _grads(x, None, 2.0, 1)
    gk, gLk, _ = _grads(x, None, 2.0, k)
    np.testing.assert_array_equal(_bits(gk), _bits(g1))
    np.testing.assert_array_equal(_bits(gLk), _bits(gL1))
    res, tape = gs_oracle.fit_tape(x, 2.0)
    _say(f"ckpt k={k}: rounds={res.n_iter}")
    assert res.n_iter >= 3
    np.testing.assert_array_equal(_bits(gk), _bits(tape.point_adjoint(mubar)))


def test_checkpointed_backward_batched_wide_and_capped():
    sizes = [120000, 0, 1, 5000, 800, 3000]
    xs = [_blobs(780 + i, s, 3, k=30 if s > 100000 else 8, scale=8.0 if s > 100000 else 5.0,
                 spread=20.0 if s > 100000 else 12.0) for i, s in enumerate(sizes)]
    hs = [1.0, 1.0, 1.0, 2.0, 3.0, 1.5]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = np.concatenate(xs, axis=0).astype(np.float32)
    for mi in [100, 7]:
        g1, gL1, _ = _grads(x, off, hs, 1, max_iter=mi)
        for k in [2, 5, 8]:
            _say(f"batched ckpt k={k} max_iter={mi}")
            gk, gLk, _ = _grads(x, off, hs, k, max_iter=mi)
            np.testing.assert_array_equal(_bits(gk), _bits(g1))
            np.testing.assert_array_equal(_bits(gLk), _bits(gL1))


def test_checkpointed_autograd_and_invalid_interval():
    x = torch.from_numpy(_blobs(790, 20000, 5).astype(np.float32)).to(DEV)
    xa = x.clone().requires_grad_(True)
    gridshift.point_mode_loss(xa, 3.0).sum().backward()
    xb = x.clone().requires_grad_(True)
    gridshift.point_mode_loss(xb, 3.0, ckpt_every=8).sum().backward()
    assert torch.equal(xa.grad, xb.grad)
    ctx = gridshift.Context(0)
    with pytest.raises(gridshift.GridShiftError) as e:
        ctx.set_tape(-1)
    assert e.value.code == 1
