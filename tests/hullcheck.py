"""Independent 2D hull checks used to pin the oracle and to check GPU output.

Nothing here calls the oracle or the library.  Three kinds of check:

* ``brute_hull2d``: O(n^3) definition of the hull of a tiny point set: (i, j)
  is a counter-clockwise hull edge iff no point lies strictly to its right and
  every point on its line lies on the closed segment [i, j];
* ``monotone_chain``: Andrew's monotone chain, a textbook O(n log n)
  algorithm unrelated to Quickhull;
* ``check_hull2d``: a certificate, O(n log h): the reported polygon is
  strictly convex, counter-clockwise from the lexicographic minimum, its
  vertices are input points with the lowest index among duplicates, and it
  contains every input point.  A polygon with these properties is the convex
  hull and its vertices are exactly the extreme points.
"""
from __future__ import annotations

import numpy as np


def _lowest_index_of_coords(pts):
    """dict (x, y) -> lowest index carrying those coordinates."""
    x = pts[0].astype(np.int64)
    y = pts[1].astype(np.int64)
    key = (x << 32) ^ (y & 0xFFFFFFFF)
    order = np.argsort(key, kind="stable")
    k_sorted = key[order]
    first = np.ones(len(key), bool)
    first[1:] = k_sorted[1:] != k_sorted[:-1]
    return {(int(x[i]), int(y[i])): int(i) for i in order[first]}


def brute_hull2d(pts) -> list:
    """Hull by the O(n^3) edge definition; CCW from the lexicographic min."""
    pts = np.asarray(pts, np.int64)
    n = pts.shape[1]
    if n == 0:
        return []
    low = _lowest_index_of_coords(pts)
    coords = sorted(low.keys())
    m = len(coords)
    if m == 1:
        return [low[coords[0]]]
    P = np.array(coords, np.int64)          # distinct, lexicographically sorted
    px, py = P[:, 0], P[:, 1]
    nxt = {}
    for i in range(m):
        for j in range(m):
            if i == j:
                continue
            ex, ey = px[j] - px[i], py[j] - py[i]
            d = (px - px[i]) * ey - (py - py[i]) * ex     # > 0: strictly right
            if np.any(d > 0):
                continue
            on = d == 0
            t = (px - px[i]) * ex + (py - py[i]) * ey
            L = ex * ex + ey * ey
            if np.any(on & ((t < 0) | (t > L))):
                continue
            nxt[i] = j
    start = 0  # lexicographic minimum
    out = [start]
    cur = nxt[start]
    while cur != start:
        out.append(cur)
        cur = nxt[cur]
        if len(out) > m:
            raise AssertionError("brute force did not close a cycle")
    return [low[(int(px[i]), int(py[i]))] for i in out]


def monotone_chain(pts) -> list:
    """Andrew's monotone chain, strictly convex vertices, CCW from lex-min."""
    pts = np.asarray(pts, np.int64)
    if pts.shape[1] == 0:
        return []
    low = _lowest_index_of_coords(pts)
    P = sorted(low.keys())
    if len(P) == 1:
        return [low[P[0]]]

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower = []
    for p in P:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    upper = []
    for p in reversed(P):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    chain = lower[:-1] + upper[:-1]
    return [low[p] for p in chain]


def _lowest_index_per_point(pts):
    """For every point, the lowest index carrying its coordinates."""
    x = pts[0].astype(np.int64)
    y = pts[1].astype(np.int64)
    n = len(x)
    order = np.lexsort((np.arange(n), y, x))
    xs, ys = x[order], y[order]
    start = np.ones(n, bool)
    start[1:] = (xs[1:] != xs[:-1]) | (ys[1:] != ys[:-1])
    low = np.empty(n, np.int64)
    low[order] = order[start][np.cumsum(start) - 1]
    return low


def _orient(ax, ay, bx, by, px, py):
    """(b - a) x (p - a): > 0 when p is strictly left of a -> b."""
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax)


def check_hull2d(pts, idx) -> None:
    """Raise AssertionError unless ``idx`` is the CCW hull of ``pts``."""
    pts = np.asarray(pts, np.int64)
    idx = np.asarray(idx, np.int64)
    n = pts.shape[1]
    assert np.abs(pts).max(initial=0) < (1 << 29), "checker needs |coord| < 2^29"
    if n == 0:
        assert len(idx) == 0
        return
    h = len(idx)
    assert h >= 1
    assert np.all((idx >= 0) & (idx < n)), "index out of range"
    assert len(np.unique(idx)) == h, "repeated vertex"
    x, y = pts[0], pts[1]
    vx, vy = x[idx], y[idx]
    # lowest index among exact duplicates
    assert (_lowest_index_per_point(pts)[idx] == idx).all(), "not the lowest duplicate index"
    # start at the lexicographic minimum
    lex = np.lexsort((y, x))
    first = lex[0]
    assert (vx[0], vy[0]) == (x[first], y[first]), "does not start at the lexicographic min"
    if h == 1:
        assert np.all((x == vx[0]) & (y == vy[0])), "h = 1 but points differ"
        return
    if h == 2:
        last = lex[-1]
        assert (vx[1], vy[1]) == (x[last], y[last]), "h = 2 must end at the lex max"
        o = _orient(vx[0], vy[0], vx[1], vy[1], x, y)
        assert np.all(o == 0), "h = 2 but points are not collinear"
        return
    # strictly convex, counter-clockwise, one lower and one upper chain
    nx_, ny_ = np.roll(vx, -1), np.roll(vy, -1)
    nnx, nny = np.roll(vx, -2), np.roll(vy, -2)
    turn = _orient(vx, vy, nx_, ny_, nnx, nny)
    assert np.all(turn > 0), "not strictly convex / not counter-clockwise"
    key = vx * (1 << 32) + vy
    m = int(np.argmax(key))
    assert np.all(np.diff(key[: m + 1]) > 0), "lower chain not lexicographically increasing"
    assert np.all(np.diff(key[m:]) < 0), "upper chain not lexicographically decreasing"
    # containment: fan from vertex 0, binary search for the wedge
    ax, ay = vx[0], vy[0]
    o1 = _orient(ax, ay, vx[1], vy[1], x, y)
    oh = _orient(ax, ay, vx[h - 1], vy[h - 1], x, y)
    assert np.all(o1 >= 0) and np.all(oh <= 0), "point outside the fan of vertex 0"
    lo = np.ones(n, np.int64)
    hi = np.full(n, h - 1, np.int64)
    while True:
        active = hi - lo > 1
        if not active.any():
            break
        mid = (lo + hi) // 2
        om = _orient(ax, ay, vx[mid], vy[mid], x, y)
        go = active & (om >= 0)
        lo = np.where(go, mid, lo)
        hi = np.where(active & ~go, mid, hi)
    e = _orient(vx[lo], vy[lo], vx[lo + 1], vy[lo + 1], x, y)
    assert np.all(e >= 0), "an input point lies outside the polygon"
