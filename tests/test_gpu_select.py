"""Parity of the GPU compact primitive (Algorithm 3) and of the order
statistics built from flagPermute and compact (Section 6, k-median finding)
with the oracle's.

Positions, head flags and selected values are integers: bit-exact.
"""
import sys

import numpy as np
import pytest

from oracle import segmented

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qhm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1201_2936_amd import qh
    qh.load()
    return qh


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compact(qhm, b, s):
    bt = torch.tensor(np.asarray(b, np.uint8), device="cuda")
    st = torch.tensor(np.asarray(s, np.uint8), device="cuda")
    p, sn, m = qhm.qh_test_compact(bt, st)
    return p.cpu().numpy(), sn.cpu().numpy(), m


def test_compact_scenarios(qhm):
    s = np.array([1, 0, 0, 1, 0, 1, 0])
    b = np.array([0, 1, 1, 0, 0, 1, 1])
    p, sn, m = _compact(qhm, b, s)
    wp, wm, _, wsn = segmented.compact(b, s)
    assert m == wm == 4
    assert p.tolist() == wp.tolist()
    assert sn.tolist() == wsn.tolist()


@pytest.mark.parametrize("seed", range(12))
def test_compact_random_vs_oracle(qhm, seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.choice([1, 5, 1023, 1024, 1025, 3000, 20000]))
    s = (rng.random(n) < rng.choice([0.001, 0.05, 0.5])).astype(np.int64)
    s[0] = 1
    b = (rng.random(n) < rng.choice([0.0, 0.3, 0.9, 1.0])).astype(np.int64)
    _say(f"compact seed={seed} n={n}")
    p, sn, m = _compact(qhm, b, s)
    wp, wm, _, wsn = segmented.compact(b, s)
    assert m == wm
    assert p.tolist() == wp.tolist()
    assert sn.tolist() == wsn.tolist()


def _select(qhm, vals, offsets, ranks):
    v = torch.tensor(np.asarray(vals, np.int32), device="cuda")
    o = torch.tensor(np.asarray(offsets, np.int64), device="cuda")
    r = torch.tensor(np.asarray(ranks, np.int64), device="cuda")
    return qhm.qh_select(v, o, r).cpu().numpy()


def test_select_worked_example(qhm):
    vals = np.array([7, 1, 5, 3, 9, 4, 4, 8, 2])
    offsets = np.array([0, 5, 9])
    for ranks in ([2, 0], [4, 3], [0, 1], [1, 2]):
        assert _select(qhm, vals, offsets, ranks).tolist() == segmented.select(vals, offsets, ranks).tolist()


@pytest.mark.parametrize("seed", range(10))
def test_select_random_vs_oracle(qhm, seed):
    rng = np.random.default_rng(3000 + seed)
    k = int(rng.integers(1, 200))
    big = rng.random() < 0.3
    sizes = rng.integers(1, 30000 if big else 600, size=k)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    spread = int(rng.choice([1, 3, 1000, 1 << 30]))
    vals = rng.integers(-spread, spread, size=int(offsets[-1]), endpoint=True).astype(np.int32)
    ranks = np.array([rng.integers(0, sz) for sz in sizes], np.int64)
    ranks[0] = 0
    ranks[-1] = sizes[-1] - 1
    _say(f"select seed={seed} k={k} n={offsets[-1]} spread={spread}")
    got = _select(qhm, vals, offsets, ranks)
    want = np.array([np.sort(vals[offsets[i]:offsets[i + 1]])[ranks[i]] for i in range(k)])
    assert got.tolist() == want.tolist()


def test_select_one_large_segment_medians(qhm):
    rng = np.random.default_rng(7)
    n = 300_000
    vals = rng.integers(-(1 << 30), 1 << 30, size=n).astype(np.int32)
    srt = np.sort(vals)
    for r in (0, n // 2, n - 1):
        _say(f"select n={n} rank={r}")
        got = _select(qhm, vals, np.array([0, n]), np.array([r]))
        assert got.tolist() == [srt[r]]


def test_select_bad_arguments(qhm):
    vals = np.arange(10, dtype=np.int32)
    for offsets, ranks in (([0, 5, 5, 10], [0, 0, 0]),   # an empty segment
                           ([0, 5, 10], [5, 0]),           # rank past the segment
                           ([0, 5, 10], [-1, 0]),
                           ([0, 5, 11], [0, 0])):          # offsets past n
        with pytest.raises(qhm.QhError) as ei:
            _select(qhm, vals, offsets, ranks)
        assert ei.value.status == qhm.QH_EINVAL
