"""Independent 3D hull checks used to pin the 3D oracle and to check GPU output.

Nothing here calls the oracle or the library.

* ``brute_vertices3d``: O(n^4) definition of the vertex set of a tiny point
  set: a plane through three non-collinear points with every point on one
  side supports the hull; the extreme points of the points on that plane
  (Andrew's monotone chain in a coordinate projection) are hull vertices, and
  every vertex lies on such a plane;
* ``check_hull3d``: invariants of a reported hull: every input point on the
  inner side of (or on) every facet plane, a closed oriented 2-manifold
  (each directed edge once, with its reverse), Euler V - E + F = 2,
  F = 2V - 4, facet corners equal the vertex set, no zero-area facet, at
  least three distinct facet planes at every vertex (it is extreme), the
  lowest index among duplicate coordinates, and the canonical triangulation
  (every face fanned from its lowest-index vertex).
"""
from __future__ import annotations

import numpy as np

from hullcheck import monotone_chain


def _lowest_index3(pts):
    P = np.asarray(pts, np.int64)
    low = {}
    for i in range(P.shape[1]):
        low.setdefault((int(P[0, i]), int(P[1, i]), int(P[2, i])), i)
    return low


def brute_vertices3d(pts):
    """Sorted hull vertex indices (lowest index per coordinate triple), or
    None when the points span less than three dimensions."""
    low = _lowest_index3(pts)
    keys = sorted(low.keys())
    Q = np.array(keys, np.int64)
    m = len(Q)
    verts = set()
    full = False
    for i in range(m):
        for j in range(i + 1, m):
            for k in range(j + 1, m):
                nrm = np.cross(Q[j] - Q[i], Q[k] - Q[i])
                if not nrm.any():
                    continue
                d = (Q - Q[i]) @ nrm
                if (d != 0).any():
                    full = True
                if not ((d <= 0).all() or (d >= 0).all()):
                    continue
                on = np.nonzero(d == 0)[0]
                drop = int(np.argmax(np.abs(nrm)))
                keep = [c for c in range(3) if c != drop]
                proj = Q[on][:, keep].T
                for e in monotone_chain(proj):
                    verts.add(low[keys[on[e]]])
    if not full:
        return None
    return sorted(verts)


def check_hull3d(pts, facets, verts, sample=None):
    """Assert the invariants above.  ``sample``: check only these point
    indices against every facet (None = all points).  Array operations
    throughout: facet planes are compared by their primitive normals (the
    normal divided by the gcd of its components), which are equal exactly
    when the planes have the same outward direction."""
    P = np.asarray(pts, np.int64)
    F = np.asarray(facets, np.int64).reshape(-1, 3)
    V = np.asarray(verts, np.int64)
    n = P.shape[1]
    assert len(V) >= 4 and len(F) == 2 * len(V) - 4
    assert (np.diff(V) > 0).all(), "vertices not ascending"
    assert np.array_equal(np.unique(F.ravel()), V), "facet corners != vertex set"
    A = P[:, F[:, 0]].T
    B = P[:, F[:, 1]].T
    C = P[:, F[:, 2]].T
    N = np.cross(B - A, C - A)
    assert N.any(axis=1).all(), "zero-area facet"
    off = np.einsum("ij,ij->i", N, A)
    idx = np.arange(n) if sample is None else np.asarray(sample)
    for s in range(0, len(idx), 4096):
        q = P[:, idx[s:s + 4096]]
        d = N @ q - off[:, None]
        assert (d <= 0).all(), "a point lies outside a facet"
    # closed oriented 2-manifold: each directed edge once, with its reverse
    u = F.ravel()
    w = F[:, [1, 2, 0]].ravel()
    key = np.sort(u * n + w)
    assert (np.diff(key) > 0).all(), "directed edge used twice"
    rev = w * n + u
    pos = np.searchsorted(key, rev)
    assert (pos < len(key)).all() and (key[np.minimum(pos, len(key) - 1)] == rev).all(), \
        "edge without its reverse"
    E = len(key) // 2
    assert len(V) - E + len(F) == 2, "Euler characteristic"
    # the facet planes by primitive outward normal
    g = np.gcd.reduce(np.abs(N), axis=1)
    prim = N // g[:, None]
    _, pid = np.unique(prim, axis=0, return_inverse=True)
    pid = pid.ravel()
    # every vertex is extreme: >= 3 distinct planes around it
    pairs = np.unique(u * (pid.max() + 1) + np.repeat(pid, 3))
    verts_of_pairs = pairs // (pid.max() + 1)
    vv, cnt = np.unique(verts_of_pairs, return_counts=True)
    assert np.array_equal(vv, V) and (cnt >= 3).all(), "a vertex is not extreme"
    # lowest index among duplicates
    order = np.lexsort((np.arange(n), P[2], P[1], P[0]))
    Ps = P[:, order]
    start = np.ones(n, bool)
    start[1:] = (Ps[:, 1:] != Ps[:, :-1]).any(axis=0)
    grp = np.cumsum(start) - 1
    low_of_grp = order[start]
    lowest = np.empty(n, np.int64)
    lowest[order] = low_of_grp[grp]
    assert (lowest[V] == V).all(), "not the lowest index"
    # canonical triangulation: each face (the facets of one plane) fanned from
    # its lowest vertex
    minv = np.full(pid.max() + 1, np.iinfo(np.int64).max)
    np.minimum.at(minv, np.repeat(pid, 3), u)
    assert (F[:, 0] == minv[pid]).all(), "face not fanned from its lowest vertex"
    dF = F[1:] - F[:-1]
    first = np.argmax(dF != 0, axis=1)
    lead = dF[np.arange(len(dF)), first]
    assert ((lead > 0) | (dF == 0).all(axis=1)).all(), "facets not sorted"
