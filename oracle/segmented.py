"""Reference segmented primitives of the permute-and-segment framework.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Plain Python loops over small arrays, written from Section 4.1 (``flagPermute``,
Algorithm 2) and Section 4.2 (``compact``, Algorithm 3).  Segments are
contiguous runs of the array; a head flag ``s[i] = 1`` starts one.

Readings of the printed pseudocode (each one is listed in the design notes):

* The per-segment count of state i is the backward inclusive max of the
  forward *inclusive* sum of ``mask[i]``.  The printed Algorithm 2 takes the
  backward max of the *exclusive* sum instead; that reproduces the printed
  ``backscan`` rows of Figure 1 but not its ``p`` and ``s'`` rows, which are
  the stable per-segment partition and are taken as the definition.
* ``flagPermuteKernel`` adds ``scan[f[id]][id]`` (the element's rank among its
  own state in its segment) to the counts of all lower states and to the
  segment head position ``s_h``.
* ``addSegKernel`` loops over states 0 .. k-2 and marks the first position of
  the next state group, s_h + (count of states <= i); targets at or beyond the
  segment end are ignored.
* ``compact`` runs ``segmentMaskKernel`` over the old n; the backward min scan
  takes that kernel's output; a segment whose elements are all false keeps no
  head (identity of min = +inf).
"""
from __future__ import annotations

import numpy as np

INF = np.iinfo(np.int64).max


def _segments(s):
    s = np.asarray(s)
    n = len(s)
    heads = [i for i in range(n) if s[i] == 1 or i == 0]
    bounds = heads + [n]
    return [(bounds[j], bounds[j + 1]) for j in range(len(heads))]


def segmented_scan(values, s, op: str, inclusive: bool, backward: bool = False):
    """Segmented scan of ``values`` with head flags ``s`` (Blelloch).

    op is "sum", "max" or "min".  A forward exclusive scan starts every
    segment at the identity; a backward scan runs from each segment's end.
    """
    v = np.asarray(values, np.int64)
    out = np.zeros(len(v), np.int64)
    ident = {"sum": 0, "max": -INF, "min": INF}[op]
    f = {"sum": lambda a, b: a + b, "max": max, "min": min}[op]
    for lo, hi in _segments(s):
        order = range(hi - 1, lo - 1, -1) if backward else range(lo, hi)
        acc = ident
        for i in order:
            if inclusive:
                acc = f(acc, int(v[i]))
                out[i] = acc
            else:
                out[i] = acc
                acc = f(acc, int(v[i]))
    return out


def flag_permute(f, s, k: int):
    """k-state ``flagPermute`` (Section 4.1).

    Returns (p, s_new, rows): ``p[id]`` is the new position of element id,
    ``s_new`` the head flags after the permutation, ``rows`` the intermediate
    arrays named as in Figure 1.
    """
    f = np.asarray(f, np.int64)
    s = np.asarray(s, np.int64)
    n = len(f)
    ids = np.arange(n, dtype=np.int64)
    s_t = np.where(s == 1, ids, 0)
    s_h = segmented_scan(s_t, s, "sum", inclusive=True)
    rows = {"s": s, "s_t": s_t, "s_h": s_h, "f": f}
    scan = []
    count = []
    for i in range(k):
        mask = (f == i).astype(np.int64)
        sc = segmented_scan(mask, s, "sum", inclusive=False)
        incl = segmented_scan(mask, s, "sum", inclusive=True)
        cnt = segmented_scan(incl, s, "max", inclusive=True, backward=True)
        rows[f"mask[{i}]"] = mask
        rows[f"scan[{i}]"] = sc
        rows[f"count[{i}]"] = cnt
        scan.append(sc)
        count.append(cnt)
    # flagPermuteKernel
    p = np.zeros(n, np.int64)
    for i_d in range(n):
        loc = 0
        for i in range(int(f[i_d])):
            loc += int(count[i][i_d])
        p[i_d] = loc + int(s_h[i_d]) + int(scan[f[i_d]][i_d])
    # addSegKernel: original heads stay, plus the first slot of each later group
    s_new = s.copy()
    if n:
        s_new[0] = 1
    seg_end = np.zeros(n, np.int64)
    for lo, hi in _segments(s):
        seg_end[lo:hi] = hi
    for i_d in range(n):
        cum = 0
        for i in range(k - 1):
            cum += int(count[i][i_d])
            target = int(s_h[i_d]) + cum
            if target == i_d and target < seg_end[i_d]:
                s_new[i_d] = 1
    rows["p"] = p
    rows["s'"] = s_new
    return p, s_new, rows


def literal_backscan(f, s, i: int):
    """Backward inclusive max of the exclusive sum of mask[i], exactly as the
    printed Algorithm 2 states it (these are the printed backscan rows)."""
    mask = (np.asarray(f, np.int64) == i).astype(np.int64)
    sc = segmented_scan(mask, s, "sum", inclusive=False)
    return segmented_scan(sc, s, "max", inclusive=True, backward=True)


def compact(b, s):
    """``compact`` (Section 4.2): drop elements with b = 0.

    Returns (p, n_new, sp, s_new): ``p`` is the exclusive scan of b (the new
    position of every kept element), ``sp[head]`` the new position of the
    segment's first kept element or +inf when the segment is removed, and
    ``s_new`` the head flags of the compacted array.
    """
    b = np.asarray(b, np.int64)
    s = np.asarray(s, np.int64)
    n = len(b)
    p = np.zeros(n, np.int64)
    acc = 0
    for i in range(n):
        p[i] = acc
        acc += int(b[i])
    n_new = acc
    masked = np.where(b == 1, p, INF)          # segmentMaskKernel (old n)
    sp = segmented_scan(masked, s, "min", inclusive=True, backward=True)
    s_new = np.zeros(n_new, np.int64)
    for lo, _hi in _segments(s):
        if sp[lo] != INF:
            s_new[sp[lo]] = 1
    return p, n_new, sp, s_new


def select(vals, offsets, ranks):
    """Order statistics (Section 6, k-median finding): the ranks[i]-th
    smallest value, counted from 0, of every segment [offsets[i],
    offsets[i+1]) -- by definition, the entry at that rank of the segment in
    sorted order."""
    vals = np.asarray(vals, np.int64)
    out = np.zeros(len(ranks), np.int64)
    for i, r in enumerate(ranks):
        seg = sorted(vals[int(offsets[i]):int(offsets[i + 1])].tolist())
        out[i] = seg[int(r)]
    return out


def apply_permutation(values, p):
    out = np.empty_like(np.asarray(values))
    out[np.asarray(p)] = values
    return out
