"""The oracle: plain, slow, obviously correct CPU Quickhull and segmented
primitives, written from the paper (Tzeng & Owens, Sections 3-4).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the library and its Python binding
never do.  It shares no code with the HIP path: the only thing both sides use
is the seeded input generator module ``workloads``, which holds none of the
method's arithmetic.

* ``hull2d`` / ``hull2d_batched``: the C oracle in ``qh_oracle.c`` (Algorithm
  1 in 2D, first split of Algorithm 4), exact 128-bit predicates.
* ``hull3d``: the C oracle in ``qh_oracle3d.c`` (Algorithm 1 in 3D with
  outside sets, visible facets and horizons), exact 128-bit predicates,
  canonical triangulation of every face.
* ``segmented``: ``flagPermute`` and ``compact`` (Algorithms 2 and 3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "qh_oracle.c"), os.path.join(_HERE, "qh_oracle3d.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the C oracle with gcc into ``oracle/liboracle.so``."""
    srcs = [s for s in _SRC if os.path.exists(s)]
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    stale = (not os.path.exists(_LIB)) or any(
        os.path.exists(s) and os.path.getmtime(s) > os.path.getmtime(_LIB) for s in _SRC)
    if stale:
        build()
    lib = ctypes.CDLL(_LIB)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.qho_hull2d.restype = ctypes.c_int64
    lib.qho_hull2d.argtypes = [i32p, i32p, ctypes.c_int64, i32p]
    lib.qho_hull2d_batched.restype = ctypes.c_int64
    lib.qho_hull2d_batched.argtypes = [i32p, i32p, i64p, ctypes.c_int64, i32p, i64p]
    if hasattr(lib, "qho_hull3d"):
        lib.qho_hull3d.restype = ctypes.c_int
        lib.qho_hull3d.argtypes = [i32p, i32p, i32p, ctypes.c_int64, i32p, i64p,
                                   i32p, i64p]
    _lib = lib
    return lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def hull2d(pts) -> np.ndarray:
    """CCW hull vertex indices of int32[2, n] points, from the lexicographic
    minimum."""
    lib = _load()
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    n = pts.shape[1]
    x = np.ascontiguousarray(pts[0])
    y = np.ascontiguousarray(pts[1])
    out = np.empty(max(n, 1), np.int32)
    h = lib.qho_hull2d(_p32(x), _p32(y), n, _p32(out))
    if h < 0:
        raise MemoryError("oracle ran out of memory")
    return out[:h].copy()


def hull2d_batched(pts, offsets):
    """Hulls of the instances [offsets[i], offsets[i+1]); returns
    (indices local to each instance, int64 output offsets[k + 1])."""
    lib = _load()
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    k = len(offsets) - 1
    x = np.ascontiguousarray(pts[0])
    y = np.ascontiguousarray(pts[1])
    out = np.empty(max(pts.shape[1], 1), np.int32)
    out_off = np.zeros(k + 1, np.int64)
    h = lib.qho_hull2d_batched(_p32(x), _p32(y), _p64(offsets), k, _p32(out), _p64(out_off))
    if h < 0:
        raise MemoryError("oracle ran out of memory")
    return out[:h].copy(), out_off


class Degenerate(ValueError):
    """Fewer than four affinely independent points (no 3D hull)."""


def hull3d(pts):
    """3D hull of int32[3, n] points: (facets int32[F, 3], vertices int32[V]).

    Facets are the canonical triangulation (every face fanned from its
    lowest-index vertex, counter-clockwise seen from outside), triples sorted;
    vertices ascending.  Raises Degenerate when the points span less than 3D.
    """
    lib = _load()
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    n = pts.shape[1]
    x = np.ascontiguousarray(pts[0])
    y = np.ascontiguousarray(pts[1])
    z = np.ascontiguousarray(pts[2])
    fac = np.empty(3 * max(2 * n - 4, 4), np.int32)
    ver = np.empty(max(n, 1), np.int32)
    nf = ctypes.c_int64(0)
    nv = ctypes.c_int64(0)
    rc = lib.qho_hull3d(_p32(x), _p32(y), _p32(z), n, _p32(fac), ctypes.byref(nf),
                        _p32(ver), ctypes.byref(nv))
    if rc == -4:
        raise Degenerate("fewer than four affinely independent points")
    if rc != 0:
        raise MemoryError("oracle ran out of memory")
    return fac[: 3 * nf.value].reshape(-1, 3).copy(), ver[: nv.value].copy()
