"""Parity of the HIP 2D path with the oracle (through the C ABI).

Results must be identical element by element: the same hull vertex indices in
the same counter-clockwise order.  Both arithmetic modes (exact int64 and the
FP32 filter with int64 fallback) must give the oracle's output bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from hullcheck import check_hull2d

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# bit 0: the arithmetic (0 exact int64, 1 FP32 filter); bit 1: every level
# as a round of the round kernels (no one-workgroup finishing of small segments)
MODES = [0, 1, 2, 3]


def _kw(m):
    return dict(mode=m & 1, finish=not (m & 2))


@pytest.fixture(scope="module")
def qhm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1201_2936_amd import qh
    qh.load()
    return qh


@pytest.fixture(scope="module")
def ctx(qhm):
    c = qhm.Context()
    yield c
    c.close()


def _gpu_hull(qhm, ctx, pts, mode):
    t = torch.from_numpy(np.ascontiguousarray(pts)).to("cuda")
    idx, stats = qhm.qh_hull2d(t, ctx=ctx, **_kw(mode))
    return idx.cpu().numpy(), stats


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", MODES)
def test_tiny_cases(qhm, ctx, mode):
    cases = [
        np.array([[5], [7]], np.int32),
        np.full((2, 9), 3, np.int32),
        np.array([[4, 1, 4, 1], [0, 2, 0, 2]], np.int32),
        np.array([[0, 10, 0], [0, 0, 10]], np.int32),
        np.array([[0, 1, 2, 3, 4], [0, 1, 2, 3, 4]], np.int32),
    ]
    for pts in cases:
        _say(f"tiny n={pts.shape[1]} mode={mode}")
        got, _ = _gpu_hull(qhm, ctx, pts, mode)
        assert got.tolist() == oracle.hull2d(pts).tolist()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(12))
def test_random_small(qhm, ctx, mode, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    r = int(rng.choice([5, 100, 1 << 20, (1 << 30) - 1]))
    pts = workloads.small_random(seed, n, r)
    _say(f"random seed={seed} n={n} r={r} mode={mode}")
    got, _ = _gpu_hull(qhm, ctx, pts, mode)
    assert got.tolist() == oracle.hull2d(pts).tolist()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [2047, 2048, 2049, 4095, 4097, 6144 + 3, 20000, 65536 + 17])
def test_tile_boundaries(qhm, ctx, mode, n):
    pts = workloads.disk(workloads.rng_for(n), n, 1 << 20)
    _say(f"disk n={n} mode={mode}")
    got, _ = _gpu_hull(qhm, ctx, pts, mode)
    assert got.tolist() == oracle.hull2d(pts).tolist()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(6))
def test_grid_duplicates_collinear(qhm, ctx, mode, seed):
    n = 5000 + 997 * seed
    for pts in (workloads.small_grid(seed, n, 3 + seed),
                workloads.small_collinear(seed, n, 400)):
        _say(f"grid/collinear seed={seed} n={n} mode={mode}")
        got, _ = _gpu_hull(qhm, ctx, pts, mode)
        assert got.tolist() == oracle.hull2d(pts).tolist()


def _range_edge_points(seed, C, n):
    """Snapped points of the circle of radius C (many hull vertices, nearly
    collinear triples) and points of its disk, with the four points of the
    axes at distance C; with C = 2^22 - 1 the differences reach 2^23 - 2,
    the end of the 24-bit product range."""
    rng = np.random.default_rng(seed)
    P = [workloads.circle(rng, n // 2, C).astype(np.int64),
         workloads.disk(rng, n - n // 2 - 4, C).astype(np.int64),
         np.array([[-C, C, 0, 0], [0, 0, -C, C]], np.int64)]
    pts = np.concatenate(P, axis=1)
    pts = pts[:, rng.permutation(pts.shape[1])]
    return np.ascontiguousarray(pts.astype(np.int32))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("C", [(1 << 22) - 1, 1 << 22, (1 << 30) - 1])
def test_coordinate_range_edges(qhm, ctx, mode, C):
    # |c| < 2^22 takes the 24-bit product path of the exact form, larger
    # coordinates the 64-bit one; both must give the oracle's output
    for seed in range(3):
        pts = _range_edge_points(seed, C, 60000 + 1001 * seed)
        _say(f"range edges C={C} seed={seed} n={pts.shape[1]} mode={mode}")
        got, _ = _gpu_hull(qhm, ctx, pts, mode)
        assert got.tolist() == oracle.hull2d(pts).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_many_segments(qhm, ctx, mode):
    # every point on a parabola is a vertex: segments shrink to single points
    x = np.arange(-30000, 30000, dtype=np.int64)
    pts = np.stack([x, x * x // 1024]).astype(np.int32)
    perm = np.random.default_rng(5).permutation(pts.shape[1])
    pts = np.ascontiguousarray(pts[:, perm])
    _say(f"parabola mode={mode}")
    got, _ = _gpu_hull(qhm, ctx, pts, mode)
    assert got.tolist() == oracle.hull2d(pts).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_circle_lattice(qhm, ctx, mode):
    r = 801125
    P = []
    import math
    for xx in range(-r, r + 1):
        yy2 = r * r - xx * xx
        yy = math.isqrt(yy2)
        if yy * yy == yy2:
            P.append((xx, yy))
            if yy:
                P.append((xx, -yy))
    inner = workloads.disk(workloads.rng_for(9), 100000, r - 10)
    pts = np.concatenate([np.array(P, np.int64).T.astype(np.int32), inner], axis=1)
    perm = np.random.default_rng(6).permutation(pts.shape[1])
    pts = np.ascontiguousarray(pts[:, perm])
    _say(f"circle lattice mode={mode}")
    got, _ = _gpu_hull(qhm, ctx, pts, mode)
    want = oracle.hull2d(pts)
    assert len(want) == 756
    assert got.tolist() == want.tolist()


def test_range_error(qhm, ctx):
    pts = np.array([[0, 1 << 30, 5], [0, 0, 9]], np.int32)
    with pytest.raises(qhm.QhError) as e:
        _gpu_hull(qhm, ctx, pts, 0)
    assert e.value.status == qhm.QH_ERANGE
    # the context stays usable
    ok, _ = _gpu_hull(qhm, ctx, np.array([[0, 3], [0, 4]], np.int32), 0)
    assert ok.tolist() == [0, 1]


def test_misaligned_and_odd_sizes(qhm, ctx):
    # a view that starts one element in: not 16-byte aligned
    base = workloads.disk(workloads.rng_for(12), 10001, 1 << 20)
    t = torch.from_numpy(base).to("cuda")
    for mode in MODES:
        sub = t[:, 1:]
        idx, _ = qhm.qh_hull2d(sub.contiguous(), ctx=ctx, **_kw(mode))
        assert idx.cpu().numpy().tolist() == oracle.hull2d(base[:, 1:]).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_finish_round_reported(qhm, ctx, mode):
    """Inputs of at most QH_FINISH_CAP points are finished at the first split;
    larger ones later; never with the option off."""
    for n, first in [(1, True), (700, True), (1024, True), (1025, False), (30000, False)]:
        pts = workloads.disk(workloads.rng_for(40 + n), n, 1 << 20)
        got, st = _gpu_hull(qhm, ctx, pts, mode)
        assert got.tolist() == oracle.hull2d(pts).tolist()
        if mode & 2:
            assert st["finish_round"] == -1
        elif first:
            assert st["finish_round"] == 0
        else:
            assert st["finish_round"] >= 1


@pytest.mark.parametrize("mode", [0, 1])
def test_finish_hint_same_shape(qhm, ctx, mode):
    """A call of the same shape as the context's last one launches the
    finishing kernel only from the round that call finished in; inputs that
    could finish earlier, later or never must still give the oracle's hull."""
    n = 40000
    rng = workloads.rng_for(77)
    sets = [workloads.disk(rng, n, 1 << 20),
            workloads.circle(rng, n, 1 << 20),
            workloads.disk(rng, n, 1 << 20),
            workloads.small_collinear(3, n, 400),
            workloads.disk(rng, n, 1 << 20)]
    for i, pts in enumerate(sets):
        _say(f"finish hint call {i} n={n} mode={mode}")
        got, st = _gpu_hull(qhm, ctx, np.ascontiguousarray(pts), mode)
        assert got.tolist() == oracle.hull2d(pts).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_circle_300k_finish(qhm, ctx, mode):
    """One instance of 300,000 grid points on a circle (174,915 of them hull
    vertices): segments shrink by half a round, so the round that first
    holds no segment above QH_FINISH_CAP points holds few enough of them to
    finish them one per workgroup (runs of segments need many more, which
    batches of instances give)."""
    pts = workloads.circle(workloads.rng_for(91), 300000, (1 << 30) - 1)
    _say(f"circle 300k mode={mode}")
    got, st = _gpu_hull(qhm, ctx, pts, mode)
    assert got.tolist() == oracle.hull2d(pts).tolist()
    if mode & 2:
        assert st["finish_round"] == -1 and st["finish_runs"] == 0
    else:
        assert st["finish_round"] >= 2 and st["finish_runs"] == 0


def test_deterministic_and_no_ctx(qhm):
    pts = workloads.disk(workloads.rng_for(13), 50000, 1 << 20)
    t = torch.from_numpy(pts).to("cuda")
    a, _ = qhm.qh_hull2d(t, mode=1)
    b, _ = qhm.qh_hull2d(t, mode=1)
    assert torch.equal(a, b)


@pytest.mark.parametrize("mode", MODES)
def test_disk_65k(qhm, ctx, mode):
    pts = workloads.disk_65k()
    _say(f"disk_65k mode={mode}")
    got, stats = _gpu_hull(qhm, ctx, pts, mode)
    assert got.tolist() == oracle.hull2d(pts).tolist()
    if mode & 2:
        assert stats["rounds"] >= 2 and stats["finish_round"] == -1
    else:
        assert stats["finish_round"] >= 1


@pytest.mark.parametrize("mode", MODES)
def test_disk_4m(qhm, ctx, mode):
    """The disk input of the regimes benchmark (4,194,304 points)."""
    pts = workloads.disk_4m()
    _say(f"disk_4m mode={mode}")
    got, _ = _gpu_hull(qhm, ctx, pts, mode)
    assert got.tolist() == oracle.hull2d(pts).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_square_16m(qhm, ctx, mode):
    pts = workloads.square_16m()
    _say(f"square_16m mode={mode}")
    got, stats = _gpu_hull(qhm, ctx, pts, mode)
    want = oracle.hull2d(pts)
    assert got.tolist() == want.tolist()
    if mode & 1:
        assert stats["filter_tests"] > 0
        _say(f"fallback rate {stats['filter_fallbacks'] / stats['filter_tests']:.3e}")


@pytest.mark.parametrize("mode", MODES)
def test_circle_mix_4m(qhm, ctx, mode):
    pts = workloads.circle_mix_4m()
    _say(f"circle_mix_4m mode={mode}")
    got, stats = _gpu_hull(qhm, ctx, pts, mode)
    want = oracle.hull2d(pts)
    assert got.tolist() == want.tolist()
    check_hull2d(pts, got)
    if mode & 1:
        # the exactly collinear support lines force undecided FP32 signs
        assert stats["filter_fallbacks"] > 0


# ---------------------------------------------------------------------------
# batched form: k instances in one call
# ---------------------------------------------------------------------------
def _gpu_batched(qhm, ctx, pts, offsets, mode):
    t = torch.from_numpy(np.ascontiguousarray(pts)).to("cuda")
    o = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to("cuda")
    idx, hoff, stats = qhm.qh_hull2d_batched(t, o, ctx=ctx, **_kw(mode))
    return idx.cpu().numpy(), hoff.cpu().numpy(), stats


def _small_instance(rng, kind):
    if kind == 0:
        return np.zeros((2, 0), np.int32)
    if kind == 1:
        n = int(rng.integers(1, 4))
        return workloads.small_random(int(rng.integers(1 << 30)), n, 50)
    if kind == 2:
        return workloads.small_collinear(int(rng.integers(1 << 30)), int(rng.integers(2, 300)))
    if kind == 3:
        return workloads.small_grid(int(rng.integers(1 << 30)), int(rng.integers(1, 3000)), 7)
    if kind == 4:
        return np.full((2, int(rng.integers(1, 500))), int(rng.integers(-9, 9)), np.int32)
    n = int(rng.integers(1, 9000))
    return workloads.small_random(int(rng.integers(1 << 30)), n, int(rng.choice([30, 1 << 20, (1 << 30) - 1])))


def _concat(insts):
    sizes = np.array([p.shape[1] for p in insts], np.int64)
    offsets = np.zeros(len(insts) + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pts = np.concatenate(insts, axis=1) if offsets[-1] else np.zeros((2, 0), np.int32)
    return np.ascontiguousarray(pts.astype(np.int32)), offsets


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(6))
def test_batched_small_mixed(qhm, ctx, mode, seed):
    rng = np.random.default_rng(1000 + seed)
    k = int(rng.integers(1, 80))
    insts = [_small_instance(rng, int(rng.integers(0, 6))) for _ in range(k)]
    pts, offsets = _concat(insts)
    _say(f"batched seed={seed} k={k} N={offsets[-1]} mode={mode}")
    want, want_off = oracle.hull2d_batched(pts, offsets)
    got, got_off, _ = _gpu_batched(qhm, ctx, pts, offsets, mode)
    assert got_off.tolist() == want_off.tolist()
    assert got.tolist() == want.tolist()
    # and each instance alone
    for i, p in enumerate(insts):
        assert got[got_off[i]:got_off[i + 1]].tolist() == oracle.hull2d(p).tolist()


@pytest.mark.parametrize("mode", MODES)
def test_batched_many_tiny_instances(qhm, ctx, mode):
    rng = np.random.default_rng(77)
    insts = []
    for _ in range(5000):
        n = int(rng.integers(0, 40))
        insts.append(workloads.small_random(int(rng.integers(1 << 30)), n, 1000) if n else
                     np.zeros((2, 0), np.int32))
    pts, offsets = _concat(insts)
    _say(f"batched tiny k=5000 N={offsets[-1]} mode={mode}")
    want, want_off = oracle.hull2d_batched(pts, offsets)
    got, got_off, _ = _gpu_batched(qhm, ctx, pts, offsets, mode)
    assert got_off.tolist() == want_off.tolist()
    assert got.tolist() == want.tolist()


@pytest.mark.parametrize("mode", MODES)
def test_batched_finish_runs(qhm, ctx, mode):
    """Thousands of instances: the rounds soon hold tens of thousands of small
    segments, which the finishing kernel takes in runs of consecutive
    segments (runs that end at region and workgroup boundaries, circles whose
    every point is a vertex, collinear and duplicate points); the second call
    of the same shape starts finishing where the first one did."""
    rng = np.random.default_rng(4242)
    insts = []
    for i in range(2500):
        kind = i % 10
        n = int(np.exp(rng.uniform(np.log(16), np.log(20000))))
        if kind < 7:
            insts.append(workloads.disk(rng, n, 1 << 20))
        elif kind == 7:
            insts.append(workloads.circle(rng, min(n, 3000), 1 << 20))
        elif kind == 8:
            insts.append(workloads.small_collinear(int(rng.integers(1 << 30)), min(n, 500)))
        else:
            insts.append(workloads.small_grid(int(rng.integers(1 << 30)), min(n, 4000), 9))
    pts, offsets = _concat(insts)
    _say(f"batched finish runs k=2500 N={offsets[-1]} mode={mode}")
    want, want_off = oracle.hull2d_batched(pts, offsets)
    for call in range(2):
        got, got_off, st = _gpu_batched(qhm, ctx, pts, offsets, mode)
        assert got_off.tolist() == want_off.tolist()
        assert got.tolist() == want.tolist()
        if mode & 2:
            assert st["finish_round"] == -1 and st["finish_runs"] == 0
        else:
            assert st["finish_round"] >= 2 and st["finish_runs"] == 1


def _polygon_instance(rng, m, r):
    """m vertices of a strictly convex polygon (a regular m-gon of radius r,
    rounded to the grid) and 3m points strictly inside, shuffled."""
    t = 2 * np.pi * np.arange(m) / m
    ring = np.stack([np.rint(r * np.cos(t)), np.rint(r * np.sin(t))]).astype(np.int64)
    inner = rng.integers(-r // 3, r // 3, size=(2, 3 * m), endpoint=True)
    pts = np.concatenate([ring, inner], axis=1)
    return np.ascontiguousarray(pts[:, rng.permutation(pts.shape[1])]).astype(np.int32)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k", [511, 512, 513])
def test_batched_hull_ids_around_rank_cap(qhm, ctx, mode, k):
    """16 hull vertices per instance: 8,176, 8,192 and 8,208 hull ids in all,
    on both sides of the 8,192 ids the output ranks in one block's LDS."""
    rng = np.random.default_rng(880 + k)
    insts = [_polygon_instance(rng, 16, 1000) for _ in range(k)]
    pts, offsets = _concat(insts)
    _say(f"batched rank cap k={k} mode={mode}")
    want, want_off = oracle.hull2d_batched(pts, offsets)
    got, got_off, _ = _gpu_batched(qhm, ctx, pts, offsets, mode)
    assert int(want_off[-1]) == 16 * k
    assert got_off.tolist() == want_off.tolist()
    assert got.tolist() == want.tolist()


@pytest.mark.parametrize("mode", MODES)
def test_batched_equals_single_calls(qhm, ctx, mode):
    sizes = np.array([256, 300, 5000, 70000, 2048, 2049, 1 << 17, 999], np.int64)
    pts, offsets = workloads.batched_disks(len(sizes), sizes)
    _say(f"batched vs single N={offsets[-1]} mode={mode}")
    got, got_off, _ = _gpu_batched(qhm, ctx, pts, offsets, mode)
    for i in range(len(sizes)):
        single, _ = _gpu_hull(qhm, ctx, pts[:, offsets[i]:offsets[i + 1]], mode)
        assert got[got_off[i]:got_off[i + 1]].tolist() == single.tolist()
    want, want_off = oracle.hull2d_batched(pts, offsets)
    assert got.tolist() == want.tolist()


def test_batched_bad_offsets(qhm, ctx):
    pts = torch.zeros((2, 10), dtype=torch.int32, device="cuda")
    for off in ([0, 5, 3, 10], [0, 5, 11], [1, 5, 10], [0, 4, 9]):
        o = torch.tensor(off, dtype=torch.int64, device="cuda")
        with pytest.raises(qhm.QhError) as ei:
            qhm.qh_hull2d_batched(pts, o, ctx=ctx)
        assert ei.value.status == qhm.QH_EINVAL
    # still usable afterwards
    o = torch.tensor([0, 4, 10], dtype=torch.int64, device="cuda")
    idx, hoff, _ = qhm.qh_hull2d_batched(pts, o, ctx=ctx)
    assert hoff.cpu().tolist() == [0, 1, 2] and idx.cpu().tolist() == [0, 0]


@pytest.mark.parametrize("mode", MODES)
def test_batched_disks_4096(qhm, ctx, mode, batched_full):
    """The full batched workload: 4,096 disks, about 5.1e8 points."""
    pts_t, off_t, want, want_off = batched_full
    _say(f"batched_disks full N={int(off_t[-1])} mode={mode}")
    idx, hoff, st = qhm.qh_hull2d_batched(pts_t, off_t, ctx=ctx, **_kw(mode))
    assert hoff.cpu().numpy().tolist() == want_off.tolist()
    assert np.array_equal(idx.cpu().numpy(), want)


@pytest.fixture(scope="module")
def batched_full(qhm):
    _say("generating the 4,096-disk batch")
    pts, offsets = workloads.batched_disks()
    _say("oracle on the 4,096-disk batch")
    want, want_off = oracle.hull2d_batched(pts, offsets)
    pts_t = torch.from_numpy(pts).to("cuda")
    off_t = torch.from_numpy(offsets).to("cuda")
    del pts
    yield pts_t, off_t, want, want_off
    del pts_t, off_t
    torch.cuda.empty_cache()
