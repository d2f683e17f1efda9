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


# --- the argmax filters ------------------------------------------------------
# The later rounds keep per point the interval [fl(d - 2B), fl(d + 2B)] (B the
# per-point bound above) and offer a point to the exact argmax only when its
# upper end reaches the best lower end.  The first split and the round after
# it use one bound for every point instead: with |coordinate| <= C,
# B = fl(fl(2C) fl(|ex| + |ey|)) 5 eps, and a point is offered when
# fl(d) >= fl(max fl(d) - 2B) over its child.  Both are safe only if the
# rounding of these expressions keeps the exact distance inside.

def interval2(px, py, ax, ay, bx, by):
    d, bound, exact = filt2(px, py, ax, ay, bx, by)
    lo = F(d - F(2.0) * bound)
    hi = F(d + F(2.0) * bound)
    return lo, hi, exact


def test_2d_per_point_interval_holds_the_exact_distance():
    rng = np.random.default_rng(4)
    C = (1 << 30) - 1
    for _ in range(30):
        a = rng.integers(-C, C, size=2, endpoint=True)
        b = rng.integers(-C, C, size=2, endpoint=True)
        # near the edge's line and anywhere in the range
        g = max(1, int(np.gcd(abs(b[0] - a[0]), abs(b[1] - a[1]))))
        step = (b - a) // g
        t = rng.integers(-3 * g, 3 * g, size=3000)
        near = np.stack([a[0] + t * step[0], a[1] + t * step[1]]) + rng.integers(-3, 4, size=(2, t.size))
        far = rng.integers(-C, C, size=(2, 3000), endpoint=True)
        P = np.concatenate([near, far], axis=1)
        P = P[:, (np.abs(P) <= C).all(axis=0)]
        lo, hi, exact = interval2(P[0], P[1], a[0], a[1], b[0], b[1])
        ex = exact.astype(np.float64)
        assert (lo.astype(np.float64) <= ex).all() and (ex <= hi.astype(np.float64)).all()


def static_bound(ex, ey, C):
    c2 = F(2.0 * C)
    s = F(F(np.abs(F(ex))) + F(np.abs(F(ey))))
    return F(F(c2 * s) * F(5.0 * EPS))


def estimate(px, py, ax, ay, ex, ey):
    dx, dy = px - ax, py - ay
    p1 = F(dx.astype(np.float32) * np.float32(ey))
    p2 = F(dy.astype(np.float32) * np.float32(ex))
    return F(p1 - p2), dx * ey - dy * ex


def _static_cases(rng, C, count):
    for _ in range(count):
        a = rng.integers(-C, C, size=2, endpoint=True)
        b = rng.integers(-C, C, size=2, endpoint=True)
        if (a == b).all():
            continue
        ex, ey = int(b[0] - a[0]), int(b[1] - a[1])
        g = max(1, int(np.gcd(abs(ex), abs(ey))))
        # lattice points on the edge's line, one unit off it, on the farthest
        # lines parallel to it, and anywhere in the range
        t = rng.integers(-2 * g, 2 * g, size=2000)
        line = np.stack([a[0] + t * (ex // g), a[1] + t * (ey // g)])
        line = line + rng.integers(-1, 2, size=line.shape)
        anyw = rng.integers(-C, C, size=(2, 4000), endpoint=True)
        P = np.concatenate([line, anyw], axis=1)
        P = P[:, (np.abs(P) <= C).all(axis=0)]
        yield a, ex, ey, P


def test_2d_static_bound_decides_signs_and_leaves_margin():
    rng = np.random.default_rng(5)
    for C in ((1 << 20), (1 << 30) - 1, 1000):
        und = 0
        for a, ex, ey, P in _static_cases(rng, C, 25):
            e, d = estimate(P[0], P[1], a[0], a[1], ex, ey)
            B = static_bound(ex, ey, C)
            err = np.abs(e.astype(np.float64) - d.astype(np.float64))
            # the error stays below 4/5 of the bound (the candidate test
            # relies on this margin)
            assert (err <= 0.8 * np.float64(B)).all()
            assert (d[e > B] > 0).all() and (d[e < -B] < 0).all()
            und += int(((e <= B) & (e >= -B)).sum())
        assert und > 0


def test_2d_static_candidates_keep_the_farthest_point():
    rng = np.random.default_rng(6)
    for C in ((1 << 20), (1 << 30) - 1):
        for a, ex, ey, P in _static_cases(rng, C, 40):
            e, d = estimate(P[0], P[1], a[0], a[1], ex, ey)
            B = static_bound(ex, ey, C)
            pos = e > B
            if pos.sum() < 2:
                continue
            ep, dp = e[pos], d[pos]
            # every point with the largest exact distance is a candidate,
            # against the largest estimate of any subset that holds it
            thr = F(ep.max() - F(2.0) * B)
            best = dp == dp.max()
            assert (ep[best] >= thr).all()
            # also with a second, larger group: points on the line parallel to
            # the edge through the farthest point (many exact ties)
            k = int(np.argmax(dp))
            g = max(1, int(np.gcd(abs(ex), abs(ey))))
            t = rng.integers(-50, 50, size=200)
            Q = np.stack([P[0][pos][k] + t * (ex // g), P[1][pos][k] + t * (ey // g)])
            Q = Q[:, (np.abs(Q) <= C).all(axis=0)]
            if Q.shape[1] == 0:
                continue
            eq, dq = estimate(Q[0], Q[1], a[0], a[1], ex, ey)
            assert (dq == dp.max()).all()
            thr2 = F(max(ep.max(), eq.max()) - F(2.0) * B)
            assert (eq >= thr2).all() and (ep[best] >= thr2).all()
