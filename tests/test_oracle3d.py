"""Pins of the 3D oracle against what the mathematics fixes.

Brute force on tiny sets, closed forms (lattice cube, lattice paraboloid,
lattice sphere, polytope corners with interior points), invariants and
shuffle / translation invariance, and Qhull (through SciPy) as an unrelated
library routine on points in general position.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from hullcheck3d import brute_vertices3d, check_hull3d


def _hull(pts):
    return oracle.hull3d(np.ascontiguousarray(pts, dtype=np.int32))


def _rand(seed, n, r):
    rng = np.random.default_rng(seed)
    return rng.integers(-r, r, size=(3, n), endpoint=True).astype(np.int32)


@pytest.mark.parametrize("seed", range(150))
def test_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 26))
    r = int(rng.choice([1, 2, 3, 10, 1000, (1 << 19) - 1]))
    pts = _rand(seed, n, r)
    want = brute_vertices3d(pts)
    if want is None:
        with pytest.raises(oracle.Degenerate):
            _hull(pts)
        return
    fac, ver = _hull(pts)
    assert ver.tolist() == want
    check_hull3d(pts, fac, ver)


@pytest.mark.parametrize("seed", range(60))
def test_brute_force_lattice_duplicates(seed):
    # few distinct coordinates: heavy coplanarity, collinearity, duplicates
    rng = np.random.default_rng(10_000 + seed)
    n = int(rng.integers(8, 30))
    side = int(rng.integers(1, 4))
    pts = rng.integers(0, side, size=(3, n), endpoint=True).astype(np.int32)
    want = brute_vertices3d(pts)
    if want is None:
        with pytest.raises(oracle.Degenerate):
            _hull(pts)
        return
    fac, ver = _hull(pts)
    assert ver.tolist() == want
    check_hull3d(pts, fac, ver)


def test_degenerate_inputs():
    cases = [
        np.zeros((3, 0), np.int32),
        np.array([[1, 2, 3], [0, 0, 0], [5, 5, 5]], np.int32),
        np.full((3, 10), 7, np.int32),
        np.array([[0, 1, 2, 3, 4], [0, 2, 4, 6, 8], [0, 3, 6, 9, 12]], np.int32),
        np.array([[0, 1, 0, 1, 5], [0, 0, 1, 1, 7], [0, 0, 0, 0, 0]], np.int32),
    ]
    for pts in cases:
        with pytest.raises(oracle.Degenerate):
            _hull(pts)


@pytest.mark.parametrize("m", [1, 2, 5, 17])
def test_lattice_cube(m):
    g = np.array(np.meshgrid(*[np.arange(m + 1)] * 3, indexing="ij")).reshape(3, -1)
    perm = np.random.default_rng(m).permutation(g.shape[1])
    pts = g[:, perm].astype(np.int32)
    fac, ver = _hull(pts)
    corners = [(x, y, z) for x in (0, m) for y in (0, m) for z in (0, m)]
    got = sorted(tuple(int(c) for c in pts[:, v]) for v in ver)
    assert got == sorted(corners)
    assert len(fac) == 12
    check_hull3d(pts, fac, ver)


@pytest.mark.parametrize("m", [2, 6, 20])
def test_lattice_paraboloid_all_points(m):
    xs, ys = np.meshgrid(np.arange(-m, m + 1), np.arange(-m, m + 1), indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel(), (xs ** 2 + ys ** 2).ravel()]).astype(np.int32)
    perm = np.random.default_rng(m).permutation(pts.shape[1])
    pts = np.ascontiguousarray(pts[:, perm])
    fac, ver = _hull(pts)
    # z = x^2 + y^2 is strictly convex: its tangent plane at any lattice
    # point has every other point strictly above it, so all are vertices
    assert ver.tolist() == list(range(pts.shape[1]))
    check_hull3d(pts, fac, ver)


def test_lattice_sphere_all_points():
    r2 = 105 * 105  # every lattice point on this sphere is a vertex
    pts = []
    r = int(math.isqrt(r2)) + 1
    for x in range(-r, r + 1):
        for y in range(-r, r + 1):
            z2 = r2 - x * x - y * y
            if z2 < 0:
                continue
            z = math.isqrt(z2)
            if z * z == z2:
                pts.append((x, y, z))
                if z:
                    pts.append((x, y, -z))
    pts = np.array(pts, np.int32).T
    assert pts.shape[1] > 50
    perm = np.random.default_rng(0).permutation(pts.shape[1])
    pts = np.ascontiguousarray(pts[:, perm])
    fac, ver = _hull(pts)
    assert ver.tolist() == list(range(pts.shape[1]))
    check_hull3d(pts, fac, ver)


@pytest.mark.parametrize("shape", ["octahedron", "cube", "tetra"])
def test_corners_plus_interior(shape):
    R = 1000
    if shape == "octahedron":
        corners = [(R, 0, 0), (-R, 0, 0), (0, R, 0), (0, -R, 0), (0, 0, R), (0, 0, -R)]
    elif shape == "cube":
        corners = [(x, y, z) for x in (-R, R) for y in (-R, R) for z in (-R, R)]
    else:
        corners = [(0, 0, 0), (3 * R, 0, 0), (0, 3 * R, 0), (0, 0, 3 * R)]
    rng = np.random.default_rng(5)
    inner = []
    while len(inner) < 3000:
        p = rng.integers(-R, 3 * R, size=3)
        if shape == "octahedron" and abs(p).sum() <= R:
            inner.append(p)
        elif shape == "cube" and (abs(p) <= R).all():
            inner.append(p)
        elif shape == "tetra" and (p >= 0).all() and p.sum() <= 3 * R:
            inner.append(p)
    allp = np.array(list(corners) + [tuple(p) for p in inner], np.int64).T
    perm = rng.permutation(allp.shape[1])
    pts = np.ascontiguousarray(allp[:, perm]).astype(np.int32)
    fac, ver = _hull(pts)
    got = sorted(tuple(int(c) for c in pts[:, v]) for v in ver)
    assert got == sorted(corners)
    check_hull3d(pts, fac, ver)


@pytest.mark.parametrize("seed", range(8))
def test_shuffle_translation_invariance(seed):
    pts = workloads.ball(workloads.rng_for(seed), 3000, 200)
    fac, ver = _hull(pts)
    check_hull3d(pts, fac, ver)
    coords = sorted(tuple(int(c) for c in pts[:, v]) for v in ver)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(pts.shape[1])
    p2 = np.ascontiguousarray(pts[:, perm])
    _, v2 = _hull(p2)
    assert sorted(tuple(int(c) for c in p2[:, v]) for v in v2) == coords
    t = rng.integers(-5000, 5000, size=(3, 1))
    p3 = (pts.astype(np.int64) + t).astype(np.int32)
    f3, v3 = _hull(p3)
    assert v3.tolist() == ver.tolist() and f3.tolist() == fac.tolist()


@pytest.mark.parametrize("seed", range(6))
def test_qhull_general_position(seed):
    spatial = pytest.importorskip("scipy.spatial")
    rng = np.random.default_rng(seed)
    pts = rng.integers(-(1 << 19) + 1, 1 << 19, size=(3, 4000)).astype(np.int32)
    fac, ver = _hull(pts)
    h = spatial.ConvexHull(pts.T.astype(np.float64))
    assert ver.tolist() == sorted(h.vertices.tolist())
    check_hull3d(pts, fac, ver)


def test_sphere_snapped_with_duplicates():
    rng = workloads.rng_for(99)
    s = workloads.sphere(rng, 4000, 300)
    b = workloads.ball(rng, 4000, 300)
    pts = np.ascontiguousarray(np.concatenate([s, b, s[:, :500]], axis=1))
    fac, ver = _hull(pts)
    check_hull3d(pts, fac, ver)
    assert ver.max() < 8000  # the repeated sphere points carry the higher indices


@pytest.mark.slow
def test_ball_sphere_5m_certificate():
    pts = workloads.ball_sphere_5m()
    fac, ver = _hull(pts)
    rng = np.random.default_rng(0)
    sample = rng.choice(pts.shape[1], size=300, replace=False)
    check_hull3d(pts, fac, ver, sample=sample)
