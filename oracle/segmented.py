"""Reference segmented primitives of the permute-and-segment framework.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Each function is the plain definition of what the primitive computes, written
out as counting loops over small arrays; none follows the scan-and-map
pipeline the paper uses to compute it on its GPU.  Segments are contiguous
runs of the array; a head flag ``s[i] != 0`` starts one, and element 0 always
starts one.

* ``flag_permute`` (Section 4.1, Figure 1): a stable partition of every
  segment by state.  Element i of state c = f[i] in the segment [h, e) moves
  to  h + #{j in [h, e): f[j] < c} + #{j in [h, i): f[j] = c},  and the new
  head flags mark the first slot of every non-empty state group of every
  segment (the segment's own head stays, as the first group starts there).
* ``figure1_rows``: the named rows of Figure 1 by their definitions (segment
  head index, per-state masks, the element's rank among the earlier elements
  of its state in its segment); the printed ``backscan`` rows count a state
  over the segment without its last element (reading R1).
* ``compact`` (Section 4.2): the kept elements keep their order; element i
  moves to #{j < i : kept}, and a segment keeps a head at the new position of
  its first kept element, or vanishes when it keeps none.
* ``select`` (Section 6, k-median finding): the entry of the wanted rank of
  the segment in sorted order.
"""
from __future__ import annotations

import numpy as np

INF = np.iinfo(np.int64).max


def _segments(s):
    """[(h, e)] of every segment: element 0 and every flagged element start one."""
    s = np.asarray(s)
    n = len(s)
    heads = [i for i in range(n) if s[i] != 0 or i == 0]
    bounds = heads + [n]
    return [(bounds[j], bounds[j + 1]) for j in range(len(heads))]


def flag_permute(f, s, k: int):
    """k-state ``flagPermute`` (Section 4.1) by its counting definition.

    Returns (p, s_new): ``p[i]`` is the new position of element i and
    ``s_new`` the head flags after the permutation.
    """
    f = [int(v) for v in np.asarray(f).tolist()]
    n = len(f)
    p = np.zeros(n, np.int64)
    s_new = np.zeros(n, np.int64)
    for h, e in _segments(s):
        # the first slot of state c's group: the segment head plus the
        # elements of the lower states
        count = [0] * k
        for i in range(h, e):
            count[f[i]] += 1
        first = [0] * k
        acc = h
        for c in range(k):
            first[c] = acc
            acc += count[c]
        # each element after the earlier elements of its own state
        seen = [0] * k
        for i in range(h, e):
            c = f[i]
            p[i] = first[c] + seen[c]
            seen[c] += 1
        for c in range(k):
            if count[c] > 0:
                s_new[first[c]] = 1
    return p, s_new


def figure1_rows(f, s, k: int):
    """The rows Figure 1 names, each by its definition: ``s_t`` (the index at
    a head, else 0), ``s_h`` (the head index of the element's segment),
    ``mask[c]`` (the element has state c), ``scan[c]`` (elements of state c
    before it in its segment) and ``backscan[c]`` as the printed rows read
    (elements of state c in its segment, its last element left out)."""
    f = np.asarray(f, np.int64)
    s = np.asarray(s, np.int64)
    n = len(f)
    rows = {"s": s.copy(), "f": f.copy()}
    s_t = np.zeros(n, np.int64)
    s_h = np.zeros(n, np.int64)
    for h, e in _segments(s):
        if s[h] != 0:
            s_t[h] = h
        s_h[h:e] = h
    rows["s_t"] = s_t
    rows["s_h"] = s_h
    for c in range(k):
        mask = np.zeros(n, np.int64)
        before = np.zeros(n, np.int64)
        back = np.zeros(n, np.int64)
        for h, e in _segments(s):
            without_last = sum(1 for j in range(h, e - 1) if f[j] == c)
            for i in range(h, e):
                mask[i] = 1 if f[i] == c else 0
                before[i] = sum(1 for j in range(h, i) if f[j] == c)
                back[i] = without_last
        rows[f"mask[{c}]"] = mask
        rows[f"scan[{c}]"] = before
        rows[f"backscan[{c}]"] = back
    p, s_new = flag_permute(f, s, k)
    rows["p"] = p
    rows["s'"] = s_new
    return rows


def compact(b, s):
    """``compact`` (Section 4.2) by its definition: drop elements with b = 0.

    Returns (p, n_new, sp, s_new): ``p[i]`` is the number of kept elements
    before i (the new position of a kept element), ``sp[h]`` at every segment
    head h the new position of the segment's first kept element, or ``INF``
    when it keeps none (and ``INF`` elsewhere), and ``s_new`` the head flags
    of the compacted array.
    """
    b = [int(v) != 0 for v in np.asarray(b).tolist()]
    n = len(b)
    p = np.zeros(n, np.int64)
    kept = 0
    for i in range(n):
        p[i] = kept
        kept += 1 if b[i] else 0
    sp = np.full(n, INF, np.int64)
    s_new = np.zeros(kept, np.int64)
    for h, e in _segments(s):
        ks = [i for i in range(h, e) if b[i]]
        if ks:
            sp[h] = p[ks[0]]
            s_new[p[ks[0]]] = 1
    return p, kept, sp, s_new


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
