"""GPU tracker (gs_track, Algorithm 2) against the tracking oracle: every
emitted window (o_x, o_y, l, w) bit-exact, on moving-disc videos (float32 and
float64 frames, one or two selected clusters, the bench's full-size video),
exact rectangles, a disappearing object (empty R, the window grows) and a
window reaching past the frame's borders."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from oracle import track_oracle as tr  # noqa: E402
from paper_2206_02200_amd import gridshift, synth  # noqa: E402

DEV = torch.device("cuda:0")


def _check(frames, o0, l0, w0, f, h, eta, max_inner, n_select=1, what=""):
    print(f"track case {what}: frames={frames.shape} {frames.dtype} o0={tuple(o0)} l0={l0} w0={w0} f={f} "
          f"h={h} n_select={n_select}", flush=True)
    sys.stdout.flush()
    g = gridshift.track(torch.from_numpy(np.ascontiguousarray(frames)).to(DEV), o0, l0, w0, f, h, eta, max_inner,
                        n_select)
    o = tr.track(frames, o0, l0, w0, f, h, eta, max_inner, n_select)
    np.testing.assert_array_equal(g.view(np.uint64), o.view(np.uint64), err_msg=what)
    return g


@pytest.mark.parametrize("seed", [7, 8, 9, 10])
def test_moving_disc_f32(seed):
    fr, c = synth.moving_blob_video(T=14, H=96, W=128, radius=11.0, seed=seed)
    _check(fr, c[0], 18.0, 18.0, 0.75, 16.0, 0.5, 20, what=f"disc seed {seed}")


def test_moving_disc_f64_two_clusters():
    fr, c = synth.moving_blob_video(T=10, H=90, W=120, radius=10.0, seed=11, dtype=np.float64)
    _check(fr, c[0], 30.0, 30.0, 0.8, 24.0, 0.25, 15, n_select=2, what="f64 two clusters")


def test_single_channel_frames():
    fr, c = synth.moving_blob_video(T=8, H=64, W=80, radius=8.0, seed=12)
    _check(np.ascontiguousarray(fr[..., :1]), c[0], 14.0, 14.0, 0.7, 16.0, 0.5, 10, what="dc=1")


def _rect_video(T, H, W, x0, y0, rw, rh, vx=0, vy=0):
    fr = np.empty((T, H, W, 3), np.float32)
    fr[:] = (10.0, 120.0, 200.0)
    for t in range(T):
        xs, ys = x0 + vx * t, y0 + vy * t
        fr[t, max(ys, 0):max(ys + rh, 0), max(xs, 0):max(xs + rw, 0)] = (200.0, 50.0, 50.0)
    return fr


def test_rectangles_exact_centres():
    fr = _rect_video(8, 90, 140, 20, 15, 21, 17, vx=6, vy=4)
    g = _check(fr, (30.0, 23.0), 16.0, 12.0, 0.6, 16.0, 0.25, 20, what="moving rectangle")
    np.testing.assert_array_equal(g[1:, :2], [[20 + 6 * t + 10.0, 15 + 4 * t + 8.0] for t in range(1, 8)])


def test_object_gone_and_window_past_the_borders():
    fr = _rect_video(6, 60, 70, 2, 3, 12, 12, vx=-3, vy=-2)  # leaves through the top-left corner
    fr[4:] = (10.0, 120.0, 200.0)
    _check(fr, (8.0, 9.0), 10.0, 10.0, 0.9, 16.0, 0.5, 9, what="object gone")


def test_full_size_video():
    fr, c = synth.moving_blob_video(T=40, H=480, W=640, radius=28.0, seed=7)
    g = _check(fr, c[0], 48.0, 48.0, 0.8, 16.0, 0.5, 20, what="640x480 x40")
    assert np.abs(g[:, :2] - c).max() < 4.0


def test_errors():
    fr = torch.zeros((2, 8, 8, 5), dtype=torch.float32, device=DEV)
    with pytest.raises(RuntimeError, match="GS_ERR_UNSUPPORTED"):
        gridshift.track(fr, (4.0, 4.0), 4.0, 4.0, 1.0, 1.0, 0.5)
    fr = torch.zeros((2, 8, 8, 3), dtype=torch.float32, device=DEV)
    with pytest.raises(RuntimeError, match="GS_ERR_INVALID_ARG"):
        gridshift.track(fr, (4.0, 4.0), -1.0, 4.0, 1.0, 1.0, 0.5)
    big = torch.full((2, 8, 8, 3), 1e9, dtype=torch.float32, device=DEV)
    with pytest.raises(RuntimeError, match="GS_ERR_KEY_RANGE"):
        gridshift.track(big, (4.0, 4.0), 4.0, 4.0, 1.0, 1.0, 0.5)


def test_batched_tracks_equal_single_tracks_and_oracle():
    fr, c = synth.moving_blob_video(T=10, H=96, W=128, radius=9.0, seed=13, discs=3)
    o0 = np.concatenate([c[0], [[-40.0, -40.0]]])  # the last window lies outside the frame: empty
    l0 = np.array([16.0, 20.0, 14.0, 10.0])
    w0 = np.array([16.0, 14.0, 20.0, 10.0])
    print(f"batched track case: frames={fr.shape} tracks={len(o0)}", flush=True)
    g = gridshift.track_batched(torch.from_numpy(fr).to(DEV), o0, l0, w0, 0.75, 16.0, 0.5, 15)
    for t in range(len(o0)):
        o = tr.track(fr, o0[t], l0[t], w0[t], 0.75, 16.0, 0.5, 15)
        np.testing.assert_array_equal(g[t].view(np.uint64), o.view(np.uint64), err_msg=f"track {t}")
        one = gridshift.track(torch.from_numpy(fr).to(DEV), o0[t], l0[t], w0[t], 0.75, 16.0, 0.5, 15)
        np.testing.assert_array_equal(g[t].view(np.uint64), one.view(np.uint64), err_msg=f"track {t} single")
    assert np.abs(g[:3, :, :2] - np.transpose(c, (1, 0, 2))).max() < 4.0
