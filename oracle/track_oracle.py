"""GridShift object tracking (Algorithm 2, Section 2.3), FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY.  The plain, slow reference the GPU tracker is
checked against; only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library (the
initial clustering calls this package's own GridShift oracle).

Frames are images of colour features: frame i, pixel (px, py) (column, row)
holds the colour vector c = frames[i, py, px, :].  The readings of the parts
of Algorithm 2 the paper leaves open:

* window W(o, l, w): the pixels of the frame with |px - o_x| <= l/2 and
  |py - o_y| <= w/2 (binary64: fabs(px - o_x) <= 0.5 * l), so l runs along x
  and w along y;
* initialisation: GridShift (the oracle's fit, bandwidth h, max_iter rounds)
  on the colours of W(o0, l0, w0) in frame 0 in raster order; the n_select
  largest clusters (count descending, then cluster id) are "selected"; B is the
  set of colour cells floor(fl(c / h)) of their pixels;
* each frame i >= 1 repeats, at most max_inner times:
    W' = W(o, fl(l / f), fl(w / f));
    R = the pixels of W' whose colour cell is in B;
    R empty: l = fl(1.1 * l), w = fl(1.1 * w), and the loop goes on;
    otherwise o' = (fl(sum px / |R|), fl(sum py / |R|)) (integer sums, exact),
    B = the colour cells of R, and with the extents e_x = max px - min px and
    e_y = max py - min py of R (the paper's garbled "max(l) - min(l)"):
    l = fl(0.99 * l) if e_x < l else fl(1.01 * l), likewise w with e_y;
    the loop stops once |o' - o|^2 = (dx*dx + dy*dy) < eta * eta, o = o' either way;
* the emitted window of frame i is (o_x, o_y, l, w) after that loop; frame 0
  emits (o0, l0, w0).
"""
from __future__ import annotations

import math

import numpy as np

from . import gs_oracle


def window_ranges(ox: float, oy: float, l: float, w: float, W: int, H: int):
    """Columns and rows of W(o, l, w) inside a W x H frame, by the per-pixel
    test (the set is a rectangle since the test separates)."""
    hl, hw = 0.5 * l, 0.5 * w
    cols = [px for px in range(W) if math.fabs(float(px) - ox) <= hl]
    rows = [py for py in range(H) if math.fabs(float(py) - oy) <= hw]
    return cols, rows


def colour_cell(c, h: float):
    return tuple(int(math.floor(float(v) / h)) for v in c)


def init_cells(frame0, o0, l0: float, w0: float, h: float, max_iter: int, n_select: int):
    """The initial set B of Algorithm 2: GridShift on the window's colours,
    the n_select largest clusters, their pixels' colour cells."""
    H, W, dc = frame0.shape
    cols, rows = window_ranges(o0[0], o0[1], l0, w0, W, H)
    if not cols or not rows:
        return set(), None
    pix = np.array([[frame0[py, px, k] for k in range(dc)] for py in rows for px in cols], dtype=np.float64)
    r = gs_oracle.fit(pix, h, max_iter)
    order = sorted(range(r.K), key=lambda c: (-int(r.counts[c]), c))
    sel = set(order[:n_select])
    B = {colour_cell(pix[i], h) for i in range(len(pix)) if int(r.labels[i]) in sel}
    return B, r


def track(frames, o0, l0: float, w0: float, f: float, h: float, eta: float, max_inner: int,
          n_select: int = 1, max_iter: int = 100):
    """Windows (o_x, o_y, l, w) of every frame, float64 [T, 4]."""
    frames = np.asarray(frames)
    T, H, W, dc = frames.shape
    B, _ = init_cells(frames[0], o0, l0, w0, h, max_iter, n_select)
    ox, oy, l, w = float(o0[0]), float(o0[1]), float(l0), float(w0)
    out = [(ox, oy, l, w)]
    for i in range(1, T):
        fr = frames[i]
        for _ in range(max_inner):
            cols, rows = window_ranges(ox, oy, l / f, w / f, W, H)
            members = [(px, py) for py in rows for px in cols if colour_cell(fr[py, px], h) in B]
            if not members:
                l = 1.1 * l
                w = 1.1 * w
                continue
            sx = sum(px for px, _ in members)
            sy = sum(py for _, py in members)
            nx = float(sx) / float(len(members))
            ny = float(sy) / float(len(members))
            B = {colour_cell(fr[py, px], h) for px, py in members}
            ex = max(px for px, _ in members) - min(px for px, _ in members)
            ey = max(py for _, py in members) - min(py for _, py in members)
            l = 0.99 * l if float(ex) < l else 1.01 * l
            w = 0.99 * w if float(ey) < w else 1.01 * w
            dx, dy = nx - ox, ny - oy
            ox, oy = nx, ny
            if dx * dx + dy * dy < eta * eta:
                break
        out.append((ox, oy, l, w))
    return np.array(out, dtype=np.float64)
