"""Parity of the batched 3D call (qh_hull3d_batched) with the 3D oracle run
on every instance alone, through the C ABI.

Every instance's vertices and canonical triangulation (local indices) must
equal the oracle's element by element; an instance with fewer than four
affinely independent points has neither.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = [0, 1]


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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _concat(insts):
    sizes = np.array([p.shape[1] for p in insts], np.int64)
    offsets = np.zeros(len(insts) + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pts = np.concatenate(insts, axis=1) if offsets[-1] else np.zeros((3, 0), np.int32)
    return np.ascontiguousarray(pts.astype(np.int32)), offsets


def _want(p):
    if p.shape[1] < 4:
        return None
    try:
        return oracle.hull3d(p)
    except oracle.Degenerate:
        return None


def _check(qhm, ctx, insts, mode):
    pts, off = _concat(insts)
    t = torch.from_numpy(pts).to("cuda")
    o = torch.from_numpy(off).to("cuda")
    fac, foff, ver, voff, st = qhm.qh_hull3d_batched(t, o, mode=mode, ctx=ctx)
    fac, foff, ver, voff = fac.cpu().numpy(), foff.cpu().numpy(), ver.cpu().numpy(), voff.cpu().numpy()
    assert foff[0] == 0 and voff[0] == 0
    degen = 0
    for i, p in enumerate(insts):
        w = _want(p)
        gf = fac[foff[i]:foff[i + 1]]
        gv = ver[voff[i]:voff[i + 1]]
        if w is None:
            degen += 1
            assert gf.size == 0 and gv.size == 0, i
            continue
        assert gv.tolist() == w[1].tolist(), i
        assert gf.tolist() == w[0].tolist(), i
    assert st["degenerate_instances"] == degen
    return st


def _small(rng):
    kind = int(rng.integers(0, 6))
    n = int(rng.integers(0, 2500))
    if kind == 0:
        r = int(rng.choice([1, 3, 100, 1 << 19]))
        return rng.integers(-r, r, size=(3, n), endpoint=True).astype(np.int32)
    if kind == 1:   # coplanar (z = 0): degenerate
        p = rng.integers(-50, 50, size=(3, n), endpoint=True).astype(np.int32)
        p[2] = 0
        return p
    if kind == 2:   # tiny
        return rng.integers(-5, 5, size=(3, int(rng.integers(0, 5))), endpoint=True).astype(np.int32)
    if kind == 3:   # lattice cube with duplicates
        return rng.integers(0, 4, size=(3, n)).astype(np.int32)
    g = workloads.rng_for(int(rng.integers(1 << 30)))
    m = max(n, 8)
    return np.ascontiguousarray(np.concatenate(
        [workloads.ball(g, m - m // 3, 1 << 12), workloads.sphere(g, m // 3, 1 << 12)], axis=1)).astype(np.int32)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(4))
def test_batched3d_mixed(qhm, ctx, mode, seed):
    rng = np.random.default_rng(500 + seed)
    k = int(rng.integers(1, 40))
    insts = [_small(rng) for _ in range(k)]
    _say(f"3d batched seed={seed} k={k} N={sum(p.shape[1] for p in insts)} mode={mode}")
    _check(qhm, ctx, insts, mode)


@pytest.mark.parametrize("mode", MODES)
def test_batched3d_equals_single_calls(qhm, ctx, mode):
    sizes = [4097, 60000, 300, 20000, 5]
    insts = []
    for j, n in enumerate(sizes):
        g = workloads.rng_for(900 + j)
        insts.append(np.ascontiguousarray(np.concatenate(
            [workloads.ball(g, n - n // 4, 1 << 16), workloads.sphere(g, n // 4, 1 << 16)], axis=1)).astype(np.int32))
    _say(f"3d batched vs single mode={mode}")
    st = _check(qhm, ctx, insts, mode)
    assert st["rounds"] >= 1
    pts, off = _concat(insts)
    fac, foff, ver, voff, _ = qhm.qh_hull3d_batched(torch.from_numpy(pts).to("cuda"),
                                                    torch.from_numpy(off).to("cuda"), mode=mode, ctx=ctx)
    for i, p in enumerate(insts):
        if p.shape[1] < 4:
            continue
        f1, v1, _ = qhm.qh_hull3d(torch.from_numpy(p).to("cuda"), mode=mode, ctx=ctx)
        assert f1.cpu().tolist() == fac[foff[i]:foff[i + 1]].cpu().tolist()
        assert v1.cpu().tolist() == ver[voff[i]:voff[i + 1]].cpu().tolist()


def test_batched3d_many_instances(qhm, ctx):
    rng = np.random.default_rng(77)
    insts = [rng.integers(-20, 20, size=(3, int(rng.integers(0, 60))), endpoint=True).astype(np.int32)
             for _ in range(600)]
    _say("3d batched k=600")
    _check(qhm, ctx, insts, 1)


def test_batched3d_empty_and_bad(qhm, ctx):
    # no points at all: every instance is degenerate
    pts = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
    off = torch.zeros(4, dtype=torch.int64, device="cuda")
    fac, foff, ver, voff, st = qhm.qh_hull3d_batched(pts, off, ctx=ctx)
    assert foff.cpu().tolist() == [0, 0, 0, 0] and voff.cpu().tolist() == [0, 0, 0, 0]
    assert st["degenerate_instances"] == 3
    pts = torch.zeros((3, 10), dtype=torch.int32, device="cuda")
    for bad in ([0, 5, 3, 10], [0, 5, 11], [1, 5, 10]):
        o = torch.tensor(bad, dtype=torch.int64, device="cuda")
        with pytest.raises(qhm.QhError) as ei:
            qhm.qh_hull3d_batched(pts, o, ctx=ctx)
        assert ei.value.status == qhm.QH_EINVAL
    # a coordinate out of range in one instance
    a = np.array([[0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]], np.int32)
    b = np.array([[0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, (1 << 19) + 1]], np.int32)
    p, o = _concat([a, b])
    with pytest.raises(qhm.QhError) as ei:
        qhm.qh_hull3d_batched(torch.from_numpy(p).to("cuda"), torch.from_numpy(o).to("cuda"), ctx=ctx)
    assert ei.value.status == qhm.QH_ERANGE


@pytest.mark.parametrize("mode", MODES)
def test_batched3d_init_paths(qhm, ctx, mode):
    """Instances at and above the size where the first simplex stops being
    found by one block each, and the smallest ones, in one call."""
    insts = []
    for j, n in enumerate([32768, 32769, 4, 7, 16]):
        g = workloads.rng_for(950 + j)
        insts.append(np.ascontiguousarray(np.concatenate(
            [workloads.ball(g, n - n // 4, 1 << 19), workloads.sphere(g, n // 4, 1 << 19)], axis=1)).astype(np.int32))
    _say(f"3d batched init paths mode={mode}")
    _check(qhm, ctx, insts, mode)
