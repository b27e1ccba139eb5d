"""Tracking oracle (Algorithm 2, Section 2.3) against its pins.

* A uniform rectangle on a background of another colour cell: R is exactly
  the rectangle's pixels, so the centre is the rectangle's centre (integer
  sums), and l, w follow the 0.99 / 1.01 rule step by step.
* The same rectangle moving by whole pixels: every emitted centre is the
  rectangle's centre in that frame.
* The object gone: R stays empty, the window grows by 1.1 per inner step.
* Initial selection: the largest cluster, or the two largest.
* A second, vectorised implementation (numpy masks over the whole frame, not
  loops over the window) on textured moving-disc videos: identical windows.
"""
import numpy as np
import pytest

from oracle import track_oracle as tr
from paper_2206_02200_amd import synth

FG = (200.0, 50.0, 50.0)
BG = (10.0, 120.0, 200.0)


def _rect_video(T, H, W, x0, y0, rw, rh, vx=0, vy=0):
    fr = np.empty((T, H, W, 3), np.float64)
    fr[:] = BG
    for t in range(T):
        xs, ys = x0 + vx * t, y0 + vy * t
        fr[t, ys:ys + rh, xs:xs + rw] = FG
    return fr


def _grow(v, factor, k):
    for _ in range(k):
        v = factor * v
    return v


def test_static_rectangle_centre_is_exact():
    fr = _rect_video(3, 80, 100, 30, 20, 30, 30)
    out = tr.track(fr, (45.0, 35.0), 28.0, 28.0, 0.8, 16.0, 0.5, 10)
    # window 0 lies inside the rectangle: B = {cell of FG}; R = the rectangle
    np.testing.assert_array_equal(out[1:, :2], [[44.5, 34.5], [44.5, 34.5]])
    # frame 1: two inner steps (the centre moves by (-0.5, -0.5), then not at
    # all); the extent 29 >= 28 grows l, 29 >= 28.28 grows it again
    l1 = _grow(28.0, 1.01, 2)
    assert out[1, 2] == l1 and out[1, 3] == l1
    # frame 2: one step; 29 < l1 = 28.5628 is false, so l grows again
    assert out[2, 2] == 1.01 * l1


def test_moving_rectangle_centres():
    fr = _rect_video(8, 90, 140, 20, 15, 21, 17, vx=6, vy=4)
    out = tr.track(fr, (30.0, 23.0), 16.0, 12.0, 0.6, 16.0, 0.25, 20)
    want = np.array([[20 + 6 * t + 10.0, 15 + 4 * t + 8.0] for t in range(1, 8)])
    np.testing.assert_array_equal(out[1:, :2], want)


def test_object_gone_grows_the_window():
    fr = _rect_video(3, 60, 60, 20, 20, 12, 12)
    fr[1:] = BG
    out = tr.track(fr, (26.0, 26.0), 10.0, 10.0, 1.0, 16.0, 0.5, 7)
    assert out[1, 0] == 26.0 and out[1, 1] == 26.0
    assert out[1, 2] == _grow(10.0, 1.1, 7) and out[2, 3] == _grow(10.0, 1.1, 14)


def test_initial_selection():
    fr = np.empty((1, 20, 20, 3))
    fr[:] = BG
    fr[0, :, :12] = FG  # 12 of 20 columns: FG is the larger cluster
    B1, r = tr.init_cells(fr[0], (9.5, 9.5), 100.0, 100.0, 16.0, 100, 1)
    assert r.K == 2
    assert B1 == {tr.colour_cell(FG, 16.0)}
    B2, _ = tr.init_cells(fr[0], (9.5, 9.5), 100.0, 100.0, 16.0, 100, 2)
    assert B2 == {tr.colour_cell(FG, 16.0), tr.colour_cell(BG, 16.0)}


def _track_vectorised(frames, o0, l0, w0, f, h, eta, max_inner, n_select=1):
    T, H, W, dc = frames.shape
    B, _ = tr.init_cells(frames[0], o0, l0, w0, h, 100, n_select)
    px = np.arange(W, dtype=np.float64)[None, :]
    py = np.arange(H, dtype=np.float64)[:, None]
    ox, oy, l, w = float(o0[0]), float(o0[1]), float(l0), float(w0)
    out = [(ox, oy, l, w)]
    for i in range(1, T):
        cells = np.floor(frames[i].astype(np.float64) / h).astype(np.int64)
        inB = np.zeros((H, W), bool)
        for b in B:
            inB |= np.all(cells == np.array(b), axis=-1)
        for _ in range(max_inner):
            win = (np.abs(px - ox) <= 0.5 * (l / f)) & (np.abs(py - oy) <= 0.5 * (w / f))
            m = win & inB
            ys, xs = np.nonzero(m)
            if xs.size == 0:
                l, w = 1.1 * l, 1.1 * w
                continue
            nx = float(xs.sum()) / float(xs.size)
            ny = float(ys.sum()) / float(ys.size)
            B = {tuple(int(v) for v in cells[y, x]) for y, x in zip(ys, xs)}
            inB = np.zeros((H, W), bool)
            for b in B:
                inB |= np.all(cells == np.array(b), axis=-1)
            l = 0.99 * l if float(xs.max() - xs.min()) < l else 1.01 * l
            w = 0.99 * w if float(ys.max() - ys.min()) < w else 1.01 * w
            dx, dy = nx - ox, ny - oy
            ox, oy = nx, ny
            if dx * dx + dy * dy < eta * eta:
                break
        out.append((ox, oy, l, w))
    return np.array(out)


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_against_vectorised_formulation(seed):
    fr, c = synth.moving_blob_video(T=8, H=72, W=96, radius=9.0, seed=seed, dtype=np.float64)
    a = tr.track(fr, c[0], 16.0, 16.0, 0.75, 16.0, 0.5, 15)
    b = _track_vectorised(fr, c[0], 16.0, 16.0, 0.75, 16.0, 0.5, 15)
    np.testing.assert_array_equal(a, b)
    assert np.abs(a[:, :2] - c).max() < 4.0  # and it follows the disc (clipped at borders)
