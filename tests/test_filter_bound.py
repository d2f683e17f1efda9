"""The FP32 filters decide a sign only when it is certain.

2D: d = (px - ax)(by - ay) - (py - ay)(bx - ax) with exact int32 differences
rounded to float, the two products and the difference rounded once each
(no fused multiply-add), decided iff |fl(d)| > 5 eps (|p1| + |p2|).
3D: d = n.p - off with the int64 normal components and offset rounded to
float, |coordinate| <= 2^19 exact, three products, two sums and one
difference rounded once each, decided iff |fl(d)| > 8 eps (|fx| + |fy| +
|fz| + |fo|).

Every decided sign must equal the exact integer sign, on adversarial inputs
(points on, and one unit off, long edges and planes) and random ones.  numpy
float32 arithmetic is IEEE round-to-nearest, the rounding the kernels use.
"""
import numpy as np

EPS = np.float32(2.0 ** -24)
F = np.float32


def filt2(px, py, ax, ay, bx, by):
    dx, dy = px - ax, py - ay          # int64, exact
    ex, ey = bx - ax, by - ay
    p1 = F(dx.astype(np.float32) * ey.astype(np.float32))
    p2 = F(dy.astype(np.float32) * ex.astype(np.float32))
    d = F(p1 - p2)
    bound = F(F(np.abs(p1) + np.abs(p2)) * F(5.0 * EPS))
    exact = dx * ey - dy * ex
    return d, bound, exact


def check2(px, py, ax, ay, bx, by):
    d, bound, exact = filt2(px, py, ax, ay, bx, by)
    pos = d > bound
    neg = d < -bound
    assert (exact[pos] > 0).all()
    assert (exact[neg] < 0).all()
    return int((~pos & ~neg).sum())


def test_2d_on_and_near_long_edges():
    rng = np.random.default_rng(0)
    C = (1 << 30) - 1
    und = 0
    for _ in range(40):
        a = rng.integers(-C, C, size=2, endpoint=True)
        b = rng.integers(-C, C, size=2, endpoint=True)
        g = np.gcd(abs(b[0] - a[0]), abs(b[1] - a[1]))
        if g == 0:
            continue
        step = (b - a) // g
        t = rng.integers(-3 * g, 3 * g, size=4000)
        px = a[0] + t * step[0] + rng.integers(-2, 3, size=t.size)
        py = a[1] + t * step[1] + rng.integers(-2, 3, size=t.size)
        keep = (np.abs(px) <= C) & (np.abs(py) <= C)
        und += check2(px[keep], py[keep], a[0], a[1], b[0], b[1])
    assert und > 0  # the adversarial points do reach the fallback


def test_2d_random_full_range():
    rng = np.random.default_rng(1)
    C = (1 << 30) - 1
    P = rng.integers(-C, C, size=(6, 200000), endpoint=True)
    check2(*P)


def filt3(n, off, p):
    nf = n.astype(np.float32)
    pf = p.astype(np.float32)       # exact: |p| <= 2^19
    fx = F(nf[0] * pf[0])
    fy = F(nf[1] * pf[1])
    fz = F(nf[2] * pf[2])
    fo = off.astype(np.float32)
    d = F(F(F(fx + fy) + fz) - fo)
    bound = F(F(F(F(np.abs(fx) + np.abs(fy)) + np.abs(fz)) + np.abs(fo)) * F(8.0 * EPS))
    exact = n[0] * p[0] + n[1] * p[1] + n[2] * p[2] - off
    return d, bound, exact


def test_3d_on_and_near_planes():
    rng = np.random.default_rng(2)
    C = 1 << 19
    und = 0
    for _ in range(60):
        a, b, c = (rng.integers(-C, C, size=3, endpoint=True) for _ in range(3))
        n = np.cross(b - a, c - a)
        if not n.any():
            continue
        off = int(n @ a)
        # lattice points of the plane near a, and one unit off it
        u, v = b - a, c - a
        s = rng.integers(-2, 3, size=(2, 3000))
        pts = a[:, None] + s[0] * u[:, None] + s[1] * v[:, None]
        pts = pts + rng.integers(-1, 2, size=pts.shape) * (rng.random(pts.shape[1]) < 0.5)
        keep = (np.abs(pts) <= C).all(axis=0)
        pts = pts[:, keep]
        d, bound, exact = filt3(n[:, None], np.int64(off), pts)
        pos, neg = d > bound, d < -bound
        assert (exact[pos] > 0).all() and (exact[neg] < 0).all()
        und += int((~pos & ~neg).sum())
    assert und > 0


def test_3d_random():
    rng = np.random.default_rng(3)
    C = 1 << 19
    for _ in range(20):
        a, b, c = (rng.integers(-C, C, size=3, endpoint=True) for _ in range(3))
        n = np.cross(b - a, c - a)
        off = np.int64(n @ a)
        p = rng.integers(-C, C, size=(3, 50000), endpoint=True)
        d, bound, exact = filt3(n[:, None], off, p)
        assert (exact[d > bound] > 0).all() and (exact[d < -bound] < 0).all()
