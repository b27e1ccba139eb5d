"""GPU parity at the full sizes of the benchmarked workloads.

* Gaussian mixtures: n = 10^7 float32 points, d = 2..6, h = 4 — every output
  bit-exact against the oracle (the whole set; the oracle takes seconds).
* Batched: the 256 uneven Voronoi images (1.87e8 points) in one batched call,
  generated on the device exactly as the benchmark does.  Every instance is
  compared bitwise with a plain fit of the same rows; sampled instances (the
  smallest, the largest, the longest-running, a capped one and eight seeded
  picks) are compared with the oracle; every instance's counts sum to its size.
* Forward + backward: the 64 images of 512x512 (x, y, L, a, b), recorded with
  tail checkpoints every 8 rounds; the loss of every instance and the
  gradient rows of sampled instances are compared
  bitwise with the oracle's adjoint; on one full image the gradient is checked
  against binary128 central differences (eps 1e-4) at perturbations whose
  FP64 fits keep the identical trajectory (bar 1e-6 relative).
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


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_gmm_1e7_full_size(d):
    _say(f"gmm n=1e7 d={d}")
    w = synth.gmm_f32(10_000_000, d, seed=40 + d)
    x = torch.from_numpy(w.x).to(DEV)
    g = gridshift.fit(x, w.h, w.max_iter, with_sums=True, with_keys=True)
    labels = g.labels.cpu().numpy()
    del x
    o = gs_oracle.fit(w.x.astype(np.float64), w.h, w.max_iter)
    _say(f"  cells0={o.m_hist[0]} rounds={o.n_iter} K={o.K} flags={o.flags}")
    assert g.info["n_cells0"] == o.m_hist[0]
    assert (g.info["n_clusters"], g.info["n_iter"], g.info["flags"]) == (o.K, o.n_iter, o.flags)
    np.testing.assert_array_equal(labels, o.labels)
    np.testing.assert_array_equal(g.counts.cpu().numpy(), o.counts)
    np.testing.assert_array_equal(g.keys.cpu().numpy(), o.keys)
    np.testing.assert_array_equal(_bits(g.sums.cpu().numpy()), _bits(o.sums))
    np.testing.assert_array_equal(_bits(g.modes.cpu().numpy()), _bits(o.modes))


def test_batched_256_images_full_size():
    specs = synth.batch_specs()
    X, off, hs = synth.batch_rgb_torch(specs, DEV)
    B = len(specs)
    _say(f"batched full size: B={B} n={int(off[-1])}")
    ctx = gridshift.Context(0)
    br = gridshift.fit_batched(X, off, hs, 100, ctx=ctx, with_sums=True)
    torch.cuda.synchronize()
    rounds = np.array([i["n_iter"] for i in br.infos])
    counts = br.counts.cpu().numpy()
    sums = br.sums.cpu().numpy()
    for b in range(B):
        ko = slice(br.k_offsets[b], br.k_offsets[b + 1])
        assert counts[ko].sum() == off[b + 1] - off[b]
    # every instance: bitwise the plain form on the same rows
    pctx = gridshift.Context(0)
    for b in range(B):
        p = gridshift.fit(X[off[b]:off[b + 1]], float(hs[b]), 100, ctx=pctx, with_sums=True)
        ko = slice(br.k_offsets[b], br.k_offsets[b + 1])
        assert p.info["n_clusters"] == br.infos[b]["n_clusters"], b
        assert p.info["n_iter"] == br.infos[b]["n_iter"] and p.info["flags"] == br.infos[b]["flags"], b
        assert torch.equal(p.labels, br.labels[off[b]:off[b + 1]]), b
        np.testing.assert_array_equal(_bits(p.sums.cpu().numpy()), _bits(sums[ko]), err_msg=str(b))
    # sampled instances: against the oracle
    sizes = np.diff(off)
    capped = [b for b in range(B) if br.infos[b]["flags"] & 4]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes)), int(np.argmax(rounds))}
    if capped:
        pick.add(capped[0])
    pick |= set(int(v) for v in np.random.default_rng(91).choice(B, size=8, replace=False))
    labels = br.labels
    for b in sorted(pick):
        x = X[off[b]:off[b + 1]].cpu().numpy().astype(np.float64)
        _say(f"  oracle instance {b}: n={len(x)} h={hs[b]} rounds={rounds[b]}")
        o = gs_oracle.fit(x, float(hs[b]), 100)
        ko = slice(br.k_offsets[b], br.k_offsets[b + 1])
        assert br.infos[b]["n_cells0"] == o.m_hist[0]
        assert (br.infos[b]["n_clusters"], br.infos[b]["n_iter"], br.infos[b]["flags"]) == (o.K, o.n_iter, o.flags)
        np.testing.assert_array_equal(labels[off[b]:off[b + 1]].cpu().numpy(), o.labels)
        np.testing.assert_array_equal(counts[ko], o.counts)
        np.testing.assert_array_equal(_bits(sums[ko]), _bits(o.sums))
    ctx.close()
    pctx.close()


@pytest.fixture(scope="module")
def diff_batch():
    X, off = synth.diff_batch_torch(64, DEV)
    ctx = gridshift.Context(0)
    ctx.set_tape(8)  # tail checkpoints every 8 rounds, segments recomputed in the backward
    br = gridshift.fit_batched(X, off, np.full(64, 16.0), 100, ctx=ctx)
    L = gridshift.point_mode_loss_values(ctx, X, br.labels, 64).cpu().numpy()
    g = gridshift.point_mode_loss_grad(ctx, X, br.labels, torch.ones(64, dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    yield X, off, br, L, g
    ctx.close()


def test_fwd_bwd_64_images_full_size(diff_batch):
    X, off, br, L, g = diff_batch
    _say(f"fwd+bwd full size: n={int(off[-1])}")
    assert np.all(np.isfinite(L)) and torch.isfinite(g).all()
    for b in [0, 17, 40, 63]:
        x = X[off[b]:off[b + 1]].cpu().numpy().astype(np.float64)
        Lo, go, res, _ = gs_oracle.loss_and_grad(x, 16.0)
        _say(f"  instance {b}: rounds={res.n_iter} K={res.K} loss={Lo!r}")
        assert br.infos[b]["n_iter"] == res.n_iter and br.infos[b]["n_clusters"] == res.K
        assert _bits(L[b]) == _bits(Lo)
        np.testing.assert_array_equal(_bits(g[off[b]:off[b + 1]].cpu().numpy()), _bits(go))


def test_fwd_bwd_full_image_finite_differences(diff_batch):
    X, off, br, L, g = diff_batch
    x = X[off[0]:off[1]].cpu().numpy().astype(np.float64)
    gb = g[off[0]:off[1]].cpu().numpy()
    res, tape = gs_oracle.fit_tape(x, 16.0)
    eps = 1e-4
    rng = np.random.default_rng(12)
    checked, worst = 0, 0.0
    for i in rng.choice(len(x), size=6, replace=False):
        for k in range(5):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += eps
            xm[i, k] -= eps
            _, tp = gs_oracle.fit_tape(xp, 16.0)
            _, tm = gs_oracle.fit_tape(xm, 16.0)
            if not (tape.same_trajectory(tp) and tape.same_trajectory(tm)):
                continue
            fd = tape.fd_q(x, i, k, eps)
            rel = abs(fd - gb[i, k]) / max(abs(fd), 1e-30)
            worst = max(worst, rel if abs(fd) > 1e-8 else abs(fd - gb[i, k]))
            checked += 1
    _say(f"full-image finite differences: checked={checked} worst={worst:.3e}")
    assert checked >= 20
    assert worst <= 1e-6
