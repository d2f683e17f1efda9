"""Pins of the 2D oracle against brute force, closed forms, a textbook
algorithm and a hull certificate (none of which calls the oracle)."""
import math

import numpy as np
import pytest

import oracle
import workloads
from hullcheck import brute_hull2d, check_hull2d, monotone_chain


def _as_list(a):
    return [int(v) for v in a]


# --------------------------------------------------------------------------
# brute force on tiny inputs, random and adversarial
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(300))
def test_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 41))
    r = int(rng.choice([3, 10, 1000, 1 << 20]))
    pts = workloads.small_random(seed, n, r)
    assert _as_list(oracle.hull2d(pts)) == brute_hull2d(pts)


@pytest.mark.parametrize("seed", range(200))
def test_brute_force_grid_duplicates(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 41))
    side = int(rng.integers(1, 6))
    pts = workloads.small_grid(seed, n, side)
    assert _as_list(oracle.hull2d(pts)) == brute_hull2d(pts)


@pytest.mark.parametrize("seed", range(100))
def test_brute_force_collinear(seed):
    pts = workloads.small_collinear(seed, 1 + seed % 40)
    got = _as_list(oracle.hull2d(pts))
    assert got == brute_hull2d(pts)
    assert len(got) <= 2


@pytest.mark.parametrize("seed", range(100))
def test_brute_force_collinear_plus_one(seed):
    base = workloads.small_collinear(seed, 20)
    extra = workloads.small_random(seed, 3, 2000)
    pts = np.concatenate([base, extra], axis=1)
    assert _as_list(oracle.hull2d(pts)) == brute_hull2d(pts)


# --------------------------------------------------------------------------
# degenerate cases of the output convention
# --------------------------------------------------------------------------
def test_empty_single_equal():
    assert _as_list(oracle.hull2d(np.zeros((2, 0), np.int32))) == []
    assert _as_list(oracle.hull2d(np.array([[5], [7]], np.int32))) == [0]
    pts = np.full((2, 9), 3, np.int32)
    assert _as_list(oracle.hull2d(pts)) == [0]


def test_two_points_and_duplicates():
    pts = np.array([[4, 1, 4, 1], [0, 2, 0, 2]], np.int32)
    # lex min (1,2) first seen at index 1; lex max (4,0) first at index 0
    assert _as_list(oracle.hull2d(pts)) == [1, 0]


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------
def test_lattice_square_corners():
    m = 37
    xs, ys = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()]).astype(np.int32)
    perm = np.random.default_rng(0).permutation(pts.shape[1])
    pts = pts[:, perm]
    got = oracle.hull2d(pts)
    corners = [(0, 0), (m, 0), (m, m), (0, m)]          # CCW from lex min
    assert [(int(pts[0, i]), int(pts[1, i])) for i in got] == corners


def test_parabola_all_points():
    x = np.arange(-1024, 1025, dtype=np.int64)
    pts = np.stack([x, x * x]).astype(np.int32)
    perm = np.random.default_rng(1).permutation(pts.shape[1])
    pts = pts[:, perm]
    got = oracle.hull2d(pts)
    # every point is a vertex; CCW from the lex min = ascending x
    assert len(got) == len(x)
    assert np.all(np.diff(pts[0, got]) > 0)


def _circle_lattice(r):
    pts = []
    for xx in range(-r, r + 1):
        yy2 = r * r - xx * xx
        yy = math.isqrt(yy2)
        if yy * yy == yy2:
            pts.append((xx, yy))
            if yy:
                pts.append((xx, -yy))
    return pts


def test_circle_lattice_points_all_extreme():
    r = 801125  # 5^3 * 13 * 17 * 29: 4 * 7 * 3 * 3 * 3 = 756 lattice points
    P = _circle_lattice(r)
    assert len(P) == 756
    pts = np.array(P, np.int64).T.astype(np.int32)
    perm = np.random.default_rng(2).permutation(pts.shape[1])
    pts = pts[:, perm]
    got = oracle.hull2d(pts)
    assert len(got) == 756
    ang = np.arctan2(pts[1, got].astype(float), pts[0, got].astype(float))
    # CCW from the lex min (-r, 0): angles increase from -pi (wrapping once)
    ang = np.unwrap(ang)
    assert np.all(np.diff(ang) > 0)


def test_polygon_with_interior():
    k = 40
    rng = np.random.default_rng(3)
    R = 1 << 20
    corners = [(int(round(R * math.cos(2 * math.pi * i / k))),
                int(round(R * math.sin(2 * math.pi * i / k)))) for i in range(k)]
    inner = workloads.disk(rng, 5000, R // 2)
    pts = np.concatenate([np.array(corners, np.int64).T.astype(np.int32), inner], axis=1)
    got = _as_list(oracle.hull2d(pts))
    assert sorted(got) == list(range(k))
    check_hull2d(pts, got)


# --------------------------------------------------------------------------
# textbook algorithm and certificate at moderate size
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(6))
def test_monotone_chain_agrees(seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(1000, 40000))
    gen = [workloads.small_random(seed, n, 1 << 20),
           workloads.small_grid(seed, n, 60),
           workloads.disk(rng, n, 1 << 20)][seed % 3]
    assert _as_list(oracle.hull2d(gen)) == monotone_chain(gen)


def test_disk_65k_monotone_chain_and_certificate():
    pts = workloads.disk_65k()
    got = _as_list(oracle.hull2d(pts))
    assert got == monotone_chain(pts)
    check_hull2d(pts, got)


def test_invariance_shuffle_translate():
    pts = workloads.disk(workloads.rng_for(11), 20000, 1 << 18)
    got = oracle.hull2d(pts)
    perm = np.random.default_rng(4).permutation(pts.shape[1])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    got_p = oracle.hull2d(pts[:, perm])
    assert sorted(inv[got].tolist()) == sorted(got_p.tolist())
    shifted = pts + np.array([[12345], [-999]], np.int32)
    assert _as_list(oracle.hull2d(shifted)) == _as_list(got)


def test_batched_matches_single():
    pts, off = workloads.batched_disks(sizes=np.array([300, 0, 1, 5000, 2, 777]))
    idx, out_off = oracle.hull2d_batched(pts, off)
    for i in range(len(off) - 1):
        sl = pts[:, off[i]:off[i + 1]]
        assert _as_list(idx[out_off[i]:out_off[i + 1]]) == _as_list(oracle.hull2d(sl))


@pytest.mark.slow
@pytest.mark.parametrize("name", ["square_16m", "circle_mix_4m"])
def test_full_workloads_certificate(name):
    pts = workloads.WORKLOADS[name]()
    got = oracle.hull2d(pts)
    check_hull2d(pts, got)
