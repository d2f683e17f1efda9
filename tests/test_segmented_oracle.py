"""Pins of the segmented primitives (Sections 4.1-4.2) against the worked
example of Figure 1 and against brute-force definitions."""
import os

import numpy as np
import pytest

from oracle import segmented

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "figure1_flagpermute.txt")


def _figure1():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            name, *vals = line.split()
            rows[name] = np.array([int(v) for v in vals], np.int64)
    return rows


def test_figure1_rows():
    fig = _figure1()
    rows = segmented.figure1_rows(fig["f"], fig["s"], 3)
    for name in ["s_t", "s_h", "mask[0]", "scan[0]", "mask[1]", "scan[1]",
                 "mask[2]", "scan[2]", "p", "s'"]:
        assert rows[name].tolist() == fig[name].tolist(), name
    p, s_new = segmented.flag_permute(fig["f"], fig["s"], 3)
    assert p.tolist() == fig["p"].tolist()
    assert s_new.tolist() == fig["s'"].tolist()


def test_figure1_printed_backscan_reading():
    """The printed backscan rows count a state over the segment without its
    last element (reading R1); the p and s' rows need the full count."""
    fig = _figure1()
    rows = segmented.figure1_rows(fig["f"], fig["s"], 3)
    for i in (0, 1):
        assert rows[f"backscan[{i}]"].tolist() == fig[f"backscan[{i}]"].tolist()


def _brute_partition(f, s, k):
    """stable grouping by state inside every segment, by definition"""
    n = len(f)
    heads = [i for i in range(n) if s[i] == 1 or i == 0] + [n]
    p = np.zeros(n, np.int64)
    s_new = np.zeros(n, np.int64)
    for a, b in zip(heads[:-1], heads[1:]):
        pos = a
        for st in range(k):
            first = True
            for i in range(a, b):
                if f[i] == st:
                    p[i] = pos
                    if first:
                        s_new[pos] = 1
                        first = False
                    pos += 1
    return p, s_new


@pytest.mark.parametrize("seed", range(200))
def test_flag_permute_is_stable_partition(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 30))
    k = int(rng.integers(1, 5))
    f = rng.integers(0, k, size=n)
    s = (rng.random(n) < 0.3).astype(np.int64)
    s[0] = 1
    p, s_new = segmented.flag_permute(f, s, k)
    bp, bs = _brute_partition(f, s, k)
    assert p.tolist() == bp.tolist()
    assert s_new.tolist() == bs.tolist()
    assert sorted(p.tolist()) == list(range(n))


@pytest.mark.parametrize("seed", range(100))
def test_flag_permute_matches_stable_sort(seed):
    """A second formulation through a library primitive: sorting the
    elements stably by (segment, state) lists them in their new order."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 400))
    k = int(rng.integers(1, 17))
    f = rng.integers(0, k, size=n)
    s = (rng.random(n) < rng.choice([0.0, 0.05, 0.5])).astype(np.int64)
    s[0] = 1
    seg = np.cumsum(s) - 1
    order = np.lexsort((np.arange(n), f, seg))
    p, s_new = segmented.flag_permute(f, s, k)
    assert (order[p] == np.arange(n)).all()
    # new heads: where the (segment, state) pair changes along the new order
    key = seg[order] * 64 + f[order]
    want = np.ones(n, np.int64)
    want[1:] = (key[1:] != key[:-1]).astype(np.int64)
    assert s_new.tolist() == want.tolist()


def test_compact_scenarios():
    # segment 0: first element dropped -> head moves to the first kept one;
    # segment 1: every element dropped -> the segment and its head vanish;
    # segment 2: all kept -> untouched.
    s = np.array([1, 0, 0, 1, 0, 1, 0])
    b = np.array([0, 1, 1, 0, 0, 1, 1])
    p, n_new, sp, s_new = segmented.compact(b, s)
    assert n_new == 4
    assert [int(p[i]) for i in range(7) if b[i]] == [0, 1, 2, 3]
    assert sp[0] == 0 and sp[3] == segmented.INF and sp[5] == 2
    assert s_new.tolist() == [1, 0, 1, 0]


@pytest.mark.parametrize("seed", range(200))
def test_compact_brute(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 30))
    s = (rng.random(n) < 0.3).astype(np.int64)
    s[0] = 1
    b = (rng.random(n) < 0.5).astype(np.int64)
    p, n_new, sp, s_new = segmented.compact(b, s)
    kept = [i for i in range(n) if b[i]]
    assert n_new == len(kept)
    assert [int(p[i]) for i in kept] == list(range(len(kept)))
    heads = [i for i in range(n) if s[i] == 1] + [n]
    exp_heads = np.zeros(len(kept), np.int64)
    for a, c in zip(heads[:-1], heads[1:]):
        ks = [i for i in range(a, c) if b[i]]
        if ks:
            assert sp[a] == p[ks[0]]
            exp_heads[p[ks[0]]] = 1
        else:
            assert sp[a] == segmented.INF
    assert s_new.tolist() == exp_heads.tolist()


@pytest.mark.parametrize("seed", range(50))
def test_select_by_counting(seed):
    """The order statistic v of rank r is the value with
    #{x < v} <= r < #{x <= v} (brute force over the segment)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 6))
    sizes = rng.integers(1, 25, size=k)
    offsets = np.concatenate([[0], np.cumsum(sizes)])
    vals = rng.integers(-5, 5, size=int(offsets[-1]))
    ranks = np.array([rng.integers(0, sz) for sz in sizes])
    got = segmented.select(vals, offsets, ranks)
    for i in range(k):
        seg = vals[offsets[i]:offsets[i + 1]]
        v = got[i]
        assert v in seg
        assert (seg < v).sum() <= ranks[i] < (seg <= v).sum()


def test_select_worked_example():
    # the median of an odd segment, and the extremes of an even one
    vals = np.array([7, 1, 5, 3, 9, 4, 4, 8, 2])
    offsets = np.array([0, 5, 9])
    assert segmented.select(vals, offsets, [2, 0]).tolist() == [5, 2]
    assert segmented.select(vals, offsets, [4, 3]).tolist() == [9, 8]
