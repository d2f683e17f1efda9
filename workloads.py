"""Seeded synthetic point sets for the segmented Quickhull.

This module only draws integer points.  It holds no orientation test, no
distance, no hull: the oracle and the HIP path both take their inputs from
here and nothing else is shared between them.

The paper times points in, on and near the unit circle and sphere (Section 5).
These generators stand in for those distributions on an integer grid, so every
predicate of the method can be decided exactly:

* ``disk``      uniform integer points in the disk x^2 + y^2 <= R^2
                (rejection from the integer square, candidates drawn in
                batches of 2n, kept in draw order).
* ``square``    uniform integer points in [-R, R]^2 (inclusive).
* ``circle``    rint(R cos t), rint(R sin t) for t ~ U[0, 2 pi), kept distinct
                in first-draw order: the "points on the circle" regime, with a
                very large hull.
* ``ball``      uniform integer points in x^2 + y^2 + z^2 <= R^2.
* ``sphere``    rint(R g / |g|), g ~ N(0, I_3), duplicates kept.

Arrays are structure-of-arrays: a 2D set is int32[2, n] (row 0 = x, row 1 =
y), a 3D set int32[3, n].  The point index is the column.
"""
from __future__ import annotations

import math

import numpy as np

R2D = 1 << 20  # 2D radius / half-width of the grid workloads
R3D = 1 << 16  # 3D radius

# Sizes of the five workloads.
N_DISK_SMALL = 65_536
N_SQUARE = 16_777_216
N_CIRCLE_MIX = 4_194_304
N_CIRCLE_PART = 2_076_181
N_DISK_PART = 2_076_180
N_LINE_PART = N_CIRCLE_MIX - N_CIRCLE_PART - N_DISK_PART  # 41,943
N_LINES = 64
N_BALL = 4_194_304
N_SPHERE = 1_048_576
N_INSTANCES = 4_096
INST_MIN, INST_MAX = 256, 1_048_576


def rng_for(seed) -> np.random.Generator:
    """PCG64 generator; ``seed`` may be an int or a SeedSequence."""
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# basic distributions
# --------------------------------------------------------------------------
def disk(rng: np.random.Generator, n: int, r: int = R2D) -> np.ndarray:
    """n integer points uniform in x^2 + y^2 <= r^2, in draw order."""
    out_x = np.empty(n, np.int64)
    out_y = np.empty(n, np.int64)
    got = 0
    r2 = r * r
    while got < n:
        m = 2 * max(n - got, 1)
        cx = rng.integers(-r, r, size=m, endpoint=True, dtype=np.int64)
        cy = rng.integers(-r, r, size=m, endpoint=True, dtype=np.int64)
        keep = cx * cx + cy * cy <= r2
        cx, cy = cx[keep], cy[keep]
        take = min(len(cx), n - got)
        out_x[got:got + take] = cx[:take]
        out_y[got:got + take] = cy[:take]
        got += take
    return np.stack([out_x, out_y]).astype(np.int32)


def square(rng: np.random.Generator, n: int, r: int = R2D) -> np.ndarray:
    """n integer points uniform in [-r, r]^2 (inclusive)."""
    x = rng.integers(-r, r, size=n, endpoint=True, dtype=np.int64)
    y = rng.integers(-r, r, size=n, endpoint=True, dtype=np.int64)
    return np.stack([x, y]).astype(np.int32)


def circle(rng: np.random.Generator, n: int, r: int = R2D) -> np.ndarray:
    """n distinct grid points rint(r cos t), rint(r sin t), first-draw order."""
    chunks_x, chunks_y = [], []
    got = 0
    seen = np.empty(0, np.int64)
    while got < n:
        m = 2 * (n - got) + 1024
        t = rng.uniform(0.0, 2.0 * math.pi, size=m)
        cx = np.rint(r * np.cos(t)).astype(np.int64)
        cy = np.rint(r * np.sin(t)).astype(np.int64)
        key = (cx + (1 << 31)) << 32 | (cy + (1 << 31))
        # first occurrence inside this batch, in draw order
        _, first = np.unique(key, return_index=True)
        first.sort()
        key, cx, cy = key[first], cx[first], cy[first]
        fresh = ~np.isin(key, seen)
        key, cx, cy = key[fresh], cx[fresh], cy[fresh]
        take = min(len(key), n - got)
        chunks_x.append(cx[:take])
        chunks_y.append(cy[:take])
        seen = np.concatenate([seen, key[:take]])
        got += take
    return np.stack([np.concatenate(chunks_x), np.concatenate(chunks_y)]).astype(np.int32)


def ball(rng: np.random.Generator, n: int, r: int = R3D) -> np.ndarray:
    """n integer points uniform in x^2 + y^2 + z^2 <= r^2, in draw order."""
    out = np.empty((3, n), np.int64)
    got = 0
    r2 = r * r
    while got < n:
        m = 2 * max(n - got, 1)
        c = rng.integers(-r, r, size=(3, m), endpoint=True, dtype=np.int64)
        keep = (c * c).sum(axis=0) <= r2
        c = c[:, keep]
        take = min(c.shape[1], n - got)
        out[:, got:got + take] = c[:, :take]
        got += take
    return out.astype(np.int32)


def sphere(rng: np.random.Generator, n: int, r: int = R3D) -> np.ndarray:
    """n points rint(r g/|g|), g ~ N(0, I_3); duplicates are kept."""
    g = rng.standard_normal(size=(3, n))
    g /= np.sqrt((g * g).sum(axis=0))
    return np.rint(r * g).astype(np.int32)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def disk_65k() -> np.ndarray:
    """2D, n = 65,536 uniform in the disk of radius 2^20 (seed 1)."""
    return disk(rng_for(1), N_DISK_SMALL)


def square_16m() -> np.ndarray:
    """2D, n = 16,777,216 uniform in [-2^20, 2^20]^2 (seed 2)."""
    return square(rng_for(2), N_SQUARE)


def _support_lines(pts: np.ndarray, rng: np.random.Generator,
                   counts: list) -> np.ndarray:
    """Collinear points on 64 supporting lines of ``pts``.

    Line k has the primitive integer normal n_k ~ 32 (cos p_k, sin p_k),
    p_k = 2 pi (k + 1/2) / 64.  Its offset is the support value
    H_k = max_p n_k . p over ``pts`` and it passes through the point q_k that
    attains it.  The new points are q_k + t (-n_k.y, n_k.x) for integers t
    drawn uniformly in [-T_k, T_k] (T_k |n_k| <= 20000), so they lie exactly on
    the line n_k . p = H_k, repeats included.  The extent is small enough that
    no line reaches past another line's support value; this is checked.
    """
    x = pts[0].astype(np.int64)
    y = pts[1].astype(np.int64)
    normals = []
    for k in range(N_LINES):
        phi = 2.0 * math.pi * (k + 0.5) / N_LINES
        a, b = int(round(32 * math.cos(phi))), int(round(32 * math.sin(phi)))
        g = math.gcd(abs(a), abs(b))
        normals.append((a // g, b // g))
    lx, ly = [], []
    support = []
    for k, (a, b) in enumerate(normals):
        val = a * x + b * y
        q = int(np.argmax(val))
        h = int(val[q])
        support.append(h)
        tmax = int(20000 // math.hypot(a, b))
        t = rng.integers(-tmax, tmax, size=counts[k], endpoint=True, dtype=np.int64)
        lx.append(x[q] - t * b)
        ly.append(y[q] + t * a)
    lx = np.concatenate(lx)
    ly = np.concatenate(ly)
    ax = np.concatenate([x, lx])
    ay = np.concatenate([y, ly])
    for (a, b), h in zip(normals, support):
        if int((a * ax + b * ay).max()) != h:
            raise AssertionError("collinear lines reach past a support line")
    return np.stack([lx, ly]).astype(np.int32)


def disk_4m() -> np.ndarray:
    """2D, n = 4,194,304 uniform in the disk of radius 2^20 (seed 11): the
    points-in-a-disk input at the size of circle_mix_4m, so the two regimes
    compare at one size."""
    return disk(rng_for(11), N_CIRCLE_MIX)


def circle_mix_4m() -> np.ndarray:
    """2D, n = 4,194,304: snapped circle + disk + 64 exactly collinear lines.

    2,076,181 distinct snapped points on the circle of radius 2^20, 2,076,180
    uniform in the disk, and 41,943 points (about 1%) on 64 supporting lines
    of that set, all shuffled (seed 3).
    """
    rng = rng_for(3)
    c = circle(rng, N_CIRCLE_PART)
    d = disk(rng, N_DISK_PART)
    base = np.concatenate([c, d], axis=1)
    per = [N_LINE_PART // N_LINES + (1 if k < N_LINE_PART % N_LINES else 0)
           for k in range(N_LINES)]
    lines = _support_lines(base, rng, per)
    pts = np.concatenate([base, lines], axis=1)
    perm = rng.permutation(pts.shape[1])
    return np.ascontiguousarray(pts[:, perm])


def ball_sphere_5m() -> np.ndarray:
    """3D, n = 5,242,880: 4,194,304 in the ball of radius 2^16 plus 1,048,576
    snapped to its sphere, shuffled (seed 4)."""
    rng = rng_for(4)
    b = ball(rng, N_BALL)
    s = sphere(rng, N_SPHERE)
    pts = np.concatenate([b, s], axis=1)
    perm = rng.permutation(pts.shape[1])
    return np.ascontiguousarray(pts[:, perm])


def instance_sizes(k: int = N_INSTANCES) -> np.ndarray:
    """Sizes floor(exp(U(ln 256, ln 2^20))) of the batched workload (seed 5)."""
    rng = rng_for(5)
    u = rng.uniform(math.log(INST_MIN), math.log(INST_MAX), size=k)
    return np.floor(np.exp(u)).astype(np.int64)


def batched_disks(k: int = N_INSTANCES, sizes: np.ndarray | None = None):
    """k independent disks of radius 2^20 concatenated (seed 5).

    Returns (pts int32[2, N], offsets int64[k + 1]).  Instance i is drawn from
    SeedSequence(5).spawn(k)[i].
    """
    if sizes is None:
        sizes = instance_sizes(k)
    sizes = np.asarray(sizes, np.int64)
    offsets = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pts = np.empty((2, int(offsets[-1])), np.int32)
    children = np.random.SeedSequence(5).spawn(len(sizes))
    for i, ss in enumerate(children):
        pts[:, offsets[i]:offsets[i + 1]] = disk(rng_for(ss), int(sizes[i]))
    return pts, offsets


def batched_balls3d(k: int = 512):
    """k independent 3D point sets (seed 6): sizes floor(exp(U(ln 64, ln 16384))),
    instance i (from SeedSequence(6).spawn(k)[i]) is three quarters uniform in
    the ball of radius 2^16 and one quarter snapped to its sphere.

    Returns (pts int32[3, N], offsets int64[k + 1])."""
    rng = rng_for(6)
    sizes = np.floor(np.exp(rng.uniform(np.log(64), np.log(16384), size=k))).astype(np.int64)
    offsets = np.zeros(k + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pts = np.empty((3, int(offsets[-1])), np.int32)
    for i, ss in enumerate(np.random.SeedSequence(6).spawn(k)):
        g = rng_for(ss)
        m = int(sizes[i])
        pts[:, offsets[i]:offsets[i + 1]] = np.concatenate([ball(g, m - m // 4), sphere(g, m // 4)], axis=1)
    return pts, offsets


WORKLOADS = {
    "disk_65k": disk_65k,
    "square_16m": square_16m,
    "disk_4m": disk_4m,
    "circle_mix_4m": circle_mix_4m,
    "ball_sphere_5m": ball_sphere_5m,
}


# --------------------------------------------------------------------------
# small adversarial sets for tests
# --------------------------------------------------------------------------
def small_random(seed: int, n: int, r: int) -> np.ndarray:
    rng = rng_for(seed)
    return square(rng, n, r)


def small_grid(seed: int, n: int, side: int) -> np.ndarray:
    """n points drawn (with repeats) from the (side+1)^2 lattice square."""
    rng = rng_for(seed)
    return rng.integers(0, side, size=(2, n), endpoint=True, dtype=np.int64).astype(np.int32)


def small_collinear(seed: int, n: int, span: int = 50) -> np.ndarray:
    """n points on one random lattice line (repeats allowed)."""
    rng = rng_for(seed)
    dx, dy = (int(v) for v in rng.integers(-5, 5, size=2, endpoint=True))
    if dx == 0 and dy == 0:
        dx = 1
    ox, oy = (int(v) for v in rng.integers(-1000, 1000, size=2, endpoint=True))
    t = rng.integers(-span, span, size=n, endpoint=True, dtype=np.int64)
    return np.stack([ox + t * dx, oy + t * dy]).astype(np.int32)


def small_ball3(seed: int, n: int, r: int) -> np.ndarray:
    return ball(rng_for(seed), n, r)


def small_grid3(seed: int, n: int, side: int) -> np.ndarray:
    rng = rng_for(seed)
    return rng.integers(0, side, size=(3, n), endpoint=True, dtype=np.int64).astype(np.int32)
