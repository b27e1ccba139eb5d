"""Exact-rational brute-force GridShift for tiny inputs (test helper).

Written from the paper independently of the FP64 oracle, in exact rational
arithmetic (fractions.Fraction), so it pins the mathematics apart from
floating-point rounding:

* keys are floor(x / h) of the exact quotient (Section 2.1 (i));
* the neighbour relation is the supplement's cell distance
  M(z, x; h) = max_k |floor(x_k/h) - floor(z_k/h)| <= 1, evaluated over all
  pairs of active cells (no 3^d offset enumeration);
* the shift is the exact count-weighted mean of Eq. 1-2, parallel form Eq. 6,
  or (``rule``) the sequential form of Eq. 5, written on centroids: the cells
  are visited one after another and the centroid of a visited cell is
  replaced by its new value for the cells visited after it, the weights
  staying the counts of the round ("sequential_key": ascending key;
  "sequential": ascending colour, the colour being the tuple of coordinate
  parities with dimension 0 first, then ascending key);
* merges use the exact weighted mean of Eq. 3-4;
* stopping follows Section 2.1 (v) / Theorem 2, capped at max_iter, with the
  same early exit on an unchanged state.

It also records the smallest distance of any floor decision to an integer,
so that a test can tell when FP64 rounding could legitimately flip a key.
"""
from __future__ import annotations

from fractions import Fraction
from math import floor


def _cheb_adjacent(a, b):
    return max(abs(x - y) for x, y in zip(a, b)) <= 1


def _visit_order(ks, rule):
    if rule == "sequential_key":
        return list(ks)
    return sorted(ks, key=lambda k: (tuple(v % 2 for v in k), k))


def exact_fit(x, h, max_iter=100, rule="parallel"):
    hq = Fraction(h)
    pts = [[Fraction(float(v)) for v in row] for row in x]
    n = len(pts)
    d = len(pts[0]) if n else 0
    margin = [None]

    def key(vec):
        out = []
        for v in vec:
            q = v / hq
            f = floor(q)
            frac = q - f
            dist = min(frac, 1 - frac)
            if margin[0] is None or dist < margin[0]:
                margin[0] = dist
            out.append(f)
        return tuple(out)

    # cells: key -> [count, sum vector, member point indices]
    cells = {}
    for i, p in enumerate(pts):
        k = key(p)
        if k not in cells:
            cells[k] = [0, [Fraction(0)] * d, []]
        c = cells[k]
        c[0] += 1
        c[1] = [s + v for s, v in zip(c[1], p)]
        c[2].append(i)

    t = 0
    flags = 0
    while True:
        ks = sorted(cells)
        any_nb = any(_cheb_adjacent(a, b) for a in ks for b in ks if a != b)
        if not any_nb:
            flags |= 1
            break
        if t == max_iter:
            flags |= 4
            break
        # new centroid of every cell
        newc = {}
        if rule == "parallel":
            for j in ks:
                nb = [k for k in ks if _cheb_adjacent(j, k)]
                W = sum(cells[k][0] for k in nb)
                newc[j] = [sum(cells[k][1][dd] for k in nb) / W for dd in range(d)]
        else:
            cent = {k: [s / cells[k][0] for s in cells[k][1]] for k in ks}
            for j in _visit_order(ks, rule):
                nb = [k for k in ks if _cheb_adjacent(j, k)]
                W = sum(cells[k][0] for k in nb)
                cent[j] = [sum(cells[k][0] * cent[k][dd] for k in nb) / W for dd in range(d)]
                newc[j] = cent[j]
        moved = {}
        for j in ks:
            p = newc[j]
            kap = key(p)
            C = cells[j][0]
            if kap not in moved:
                moved[kap] = [0, [Fraction(0)] * d, []]
            m = moved[kap]
            m[0] += C
            m[1] = [s + C * v for s, v in zip(m[1], p)]
            m[2].extend(cells[j][2])
        same = sorted(moved) == ks and all(
            moved[k][0] == cells[k][0] and moved[k][1] == cells[k][1] for k in ks)
        cells = moved
        t += 1
        if same:
            flags |= 2
            break

    ks = sorted(cells)
    labels = [0] * n
    for cid, k in enumerate(ks):
        for i in cells[k][2]:
            labels[i] = cid
    modes = [[s / cells[k][0] for s in cells[k][1]] for k in ks]
    counts = [cells[k][0] for k in ks]
    return {
        "labels": labels, "modes": modes, "counts": counts, "keys": [list(k) for k in ks],
        "n_iter": t, "flags": flags, "margin": margin[0],
    }


def exact_jacobian(x, h, max_iter=100):
    """Exact Jacobian of the modes with respect to the points, with the
    trajectory of the exact fit held fixed: every cell carries, besides its
    count, the weight vector w over the points such that its sum is
    S = sum_i w_i x_i (the same weights for every coordinate).  Binning gives
    indicator weights; a shift gives (sum of neighbour weights) / W; a merge
    gives sum C_j * (shifted weights).  Mode c = S_c / C_c, so J_c = w_c / C_c.
    Returns (J [K][n] of Fractions, margin)."""
    hq = Fraction(h)
    pts = [[Fraction(float(v)) for v in row] for row in x]
    n = len(pts)
    margin = [None]

    def key(vec):
        out = []
        for v in vec:
            q = v / hq
            f = floor(q)
            frac = q - f
            dist = min(frac, 1 - frac)
            if margin[0] is None or dist < margin[0]:
                margin[0] = dist
            out.append(f)
        return tuple(out)

    cells = {}
    for i, p in enumerate(pts):
        k = key(p)
        if k not in cells:
            cells[k] = [0, [Fraction(0)] * len(p), [Fraction(0)] * n]
        c = cells[k]
        c[0] += 1
        c[1] = [s + v for s, v in zip(c[1], p)]
        c[2][i] += 1
    t = 0
    while True:
        ks = sorted(cells)
        if not any(_cheb_adjacent(a, b) for a in ks for b in ks if a != b):
            break
        if t == max_iter:
            break
        moved = {}
        for j in ks:
            nb = [k for k in ks if _cheb_adjacent(j, k)]
            W = sum(cells[k][0] for k in nb)
            p = [sum(cells[k][1][dd] for k in nb) / W for dd in range(len(cells[j][1]))]
            pw = [sum(cells[k][2][i] for k in nb) / W for i in range(n)]
            kap = key(p)
            C = cells[j][0]
            if kap not in moved:
                moved[kap] = [0, [Fraction(0)] * len(p), [Fraction(0)] * n]
            m = moved[kap]
            m[0] += C
            m[1] = [s + C * v for s, v in zip(m[1], p)]
            m[2] = [s + C * v for s, v in zip(m[2], pw)]
        same = sorted(moved) == ks and all(moved[k][0] == cells[k][0] and moved[k][1] == cells[k][1] for k in ks)
        cells = moved
        t += 1
        if same:
            break
    J = [[w / cells[k][0] for w in cells[k][2]] for k in sorted(cells)]
    return J, margin[0]
