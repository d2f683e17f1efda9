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

from collections import defaultdict

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


def _planes_equal(n1, n2):
    c = np.cross(n1, n2)
    return not c.any() and int(np.dot(n1, n2)) > 0


def check_hull3d(pts, facets, verts, sample=None):
    """Assert the invariants above.  ``sample``: check only these point
    indices against every facet (None = all points)."""
    P = np.asarray(pts, np.int64)
    F = np.asarray(facets, np.int64).reshape(-1, 3)
    V = np.asarray(verts, np.int64)
    assert len(V) >= 4 and len(F) == 2 * len(V) - 4
    assert (np.diff(V) > 0).all(), "vertices not ascending"
    assert set(F.ravel().tolist()) == set(V.tolist()), "facet corners != vertex set"
    A = P[:, F[:, 0]].T
    B = P[:, F[:, 1]].T
    C = P[:, F[:, 2]].T
    N = np.cross(B - A, C - A)
    assert N.any(axis=1).all(), "zero-area facet"
    off = np.einsum("ij,ij->i", N, A)
    idx = np.arange(P.shape[1]) if sample is None else np.asarray(sample)
    for s in range(0, len(idx), 4096):
        q = P[:, idx[s:s + 4096]]
        d = N @ q - off[:, None]
        assert (d <= 0).all(), "a point lies outside a facet"
    # closed oriented 2-manifold
    edges = {}
    for f, (a, b, c) in enumerate(F.tolist()):
        for u, w in ((a, b), (b, c), (c, a)):
            assert (u, w) not in edges, "directed edge used twice"
            edges[(u, w)] = f
    for (u, w) in edges:
        assert (w, u) in edges, "edge without its reverse"
    E = len(edges) // 2
    assert len(V) - E + len(F) == 2, "Euler characteristic"
    # every vertex is extreme: >= 3 distinct planes around it
    inc = defaultdict(list)
    for f, tri in enumerate(F.tolist()):
        for v in tri:
            inc[v].append(f)
    for v, fs in inc.items():
        reps = []
        for f in fs:
            if not any(_planes_equal(N[f], N[r]) for r in reps):
                reps.append(f)
            if len(reps) >= 3:
                break
        assert len(reps) >= 3, f"vertex {v} is not extreme"
    # lowest index among duplicates
    low = _lowest_index3(P)
    for v in V.tolist():
        assert low[(int(P[0, v]), int(P[1, v]), int(P[2, v]))] == v, "not the lowest index"
    # canonical triangulation: each face fanned from its lowest vertex
    parent = list(range(len(F)))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for (u, w), f in edges.items():
        g = edges[(w, u)]
        if _planes_equal(N[f], N[g]):
            parent[find(f)] = find(g)
    faces = defaultdict(list)
    for f in range(len(F)):
        faces[find(f)].append(f)
    for fs in faces.values():
        lowest = min(int(v) for f in fs for v in F[f])
        assert all(int(F[f, 0]) == lowest for f in fs), "face not fanned from its lowest vertex"
    assert [tuple(t) for t in F.tolist()] == sorted(tuple(t) for t in F.tolist()), "facets not sorted"
