"""Thin ctypes binding of ``include/qh.h`` (argument marshalling only).

Every step of the hull runs in the HIP library ``libqh.so``; PyTorch is used
here only to own device memory and to name the current stream.  If the
library is missing this module raises: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqh.so")

QH_OK = 0
QH_EINVAL = -1
QH_ERANGE = -2
QH_ENOMEM = -3
QH_EDEGENERATE = -4
QH_EDEVICE = -5
QH_ECAPACITY = -6

QH_EXACT_INT64 = 0
QH_FP32_FILTER = 1
QH_FLAG_TIMING = 1
QH_FLAG_NO_FINISH = 2
QH_FLAG_GRAPH = 4
QH_FLAG_AUTOTUNE = 8
QH_FINISH_CAP = 1024

EXPORTED = ["qh_ctx_create", "qh_ctx_destroy", "qh_status_str", "qh_version",
            "qh_hull2d", "qh_hull2d_batched", "qh_hull3d", "qh_hull3d_batched",
            "qh_test_flag_permute", "qh_test_flag_permute_noalloc", "qh_test_compact", "qh_select"]


class QhStats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int64),
        ("round_launches", ctypes.c_int64),
        ("round_points_in", ctypes.c_int64),
        ("round_points_out", ctypes.c_int64),
        ("split_points_out", ctypes.c_int64),
        ("hull_bytes", ctypes.c_int64),
        ("round_kernel_bytes", ctypes.c_int64),
        ("kernel_ms", ctypes.c_double),
        ("round_kernel_ms", ctypes.c_double),
        ("split_ms", ctypes.c_double),
        ("extremes_ms", ctypes.c_double),
        ("segment_ms", ctypes.c_double),
        ("filter_tests", ctypes.c_int64),
        ("filter_fallbacks", ctypes.c_int64),
        ("argmax_candidates", ctypes.c_int64),
        ("max_segments", ctypes.c_int64),
        ("grid_blocks", ctypes.c_int64),
        ("host_syncs", ctypes.c_int64),
        ("host_ms", ctypes.c_double),
        ("host_output_ms", ctypes.c_double),
        ("finish_round", ctypes.c_int64),
        ("multi_blocks", ctypes.c_int64),
        ("finish_segments", ctypes.c_int64),
        ("graph_launches", ctypes.c_int64),
        ("tuned_configs", ctypes.c_int64),
        ("degenerate_instances", ctypes.c_int64),
        ("finish_runs", ctypes.c_int64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class QhOpts(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_void_p),
        ("mode", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("ctx", ctypes.c_void_p),
        ("stats", ctypes.POINTER(QhStats)),
    ]


class QhError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libqh.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run __graft_entry__.build()")
    # torch first: it brings its own HIP runtime (the same soname), and the
    # library must bind to that one, the runtime of the device memory and
    # streams it is given; loaded before torch, the library would start a
    # second runtime, which then finds no device
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.qh_ctx_create.restype = ctypes.c_int
    lib.qh_ctx_create.argtypes = [ctypes.POINTER(vp)]
    lib.qh_ctx_destroy.restype = None
    lib.qh_ctx_destroy.argtypes = [vp]
    lib.qh_status_str.restype = ctypes.c_char_p
    lib.qh_status_str.argtypes = [ctypes.c_int]
    lib.qh_version.restype = ctypes.c_char_p
    lib.qh_version.argtypes = []
    lib.qh_hull2d.restype = ctypes.c_int
    lib.qh_hull2d.argtypes = [vp, i64, vp, ctypes.POINTER(i64), ctypes.POINTER(QhOpts)]
    lib.qh_hull2d_batched.restype = ctypes.c_int
    lib.qh_hull2d_batched.argtypes = [vp, i64, vp, ctypes.c_int32, vp, vp,
                                      ctypes.POINTER(i64), ctypes.POINTER(QhOpts)]
    lib.qh_test_flag_permute.restype = ctypes.c_int
    lib.qh_test_flag_permute.argtypes = [vp, vp, i64, ctypes.c_int32, vp, vp, vp]
    lib.qh_test_flag_permute_noalloc.restype = ctypes.c_int
    lib.qh_test_flag_permute_noalloc.argtypes = [vp, vp, i64, ctypes.c_int32, vp, vp, vp]
    lib.qh_test_compact.restype = ctypes.c_int
    lib.qh_test_compact.argtypes = [vp, vp, i64, vp, vp, ctypes.POINTER(i64), vp]
    lib.qh_select.restype = ctypes.c_int
    lib.qh_select.argtypes = [vp, i64, vp, ctypes.c_int32, vp, vp, vp]
    lib.qh_hull3d_batched.restype = ctypes.c_int
    lib.qh_hull3d_batched.argtypes = [vp, i64, vp, ctypes.c_int32, vp, vp, vp, vp, ctypes.POINTER(QhOpts)]
    lib.qh_hull3d.restype = ctypes.c_int
    lib.qh_hull3d.argtypes = [vp, i64, vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64),
                              ctypes.POINTER(QhOpts)]
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load().qh_status_str(int(status)).decode()


def version() -> str:
    return load().qh_version().decode()


# Contexts still open when the interpreter exits are closed by an exit hook,
# while the HIP runtime is certainly alive, not by their finalizers during
# interpreter teardown.
_open_contexts = weakref.WeakSet()


def _close_open_contexts():
    for c in list(_open_contexts):
        c.close()


atexit.register(_close_open_contexts)


class Context:
    """A workspace context (device memory reused across calls)."""

    def __init__(self):
        self.ptr = None
        lib = load()
        p = ctypes.c_void_p()
        st = lib.qh_ctx_create(ctypes.byref(p))
        if st != QH_OK:
            raise QhError(st, "qh_ctx_create")
        self.ptr = p
        _open_contexts.add(self)

    def close(self):
        if self.ptr is not None and self.ptr.value:
            load().qh_ctx_destroy(self.ptr)
        self.ptr = None
        _open_contexts.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts(ctx, mode, timing, stream, finish=True, graph=False, autotune=False):
    import torch
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    stats = QhStats()
    flags = ((QH_FLAG_TIMING if timing else 0) | (0 if finish else QH_FLAG_NO_FINISH)
             | (QH_FLAG_GRAPH if graph else 0) | (QH_FLAG_AUTOTUNE if autotune else 0))
    o = QhOpts(ctypes.c_void_p(st), mode, flags,
               ctx.ptr if ctx is not None else None, ctypes.pointer(stats))
    return o, stats


def _check_points(pts, dims):
    import torch
    if not isinstance(pts, torch.Tensor) or not pts.is_cuda:
        raise TypeError("points must be a CUDA (HIP) tensor")
    if pts.dtype != torch.int32 or pts.dim() != 2 or pts.shape[0] != dims:
        raise TypeError(f"points must be int32 of shape ({dims}, n)")
    return pts.contiguous()


def _out_buffer(out, size, dtype, device, name):
    import torch
    if out is None:
        return torch.empty(size, dtype=dtype, device=device)
    if (not isinstance(out, torch.Tensor) or out.dtype != dtype or out.device != device
            or out.dim() != 1 or out.shape[0] < size or not out.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} tensor of at least {size} "
                        f"elements on {device}")
    return out


def qh_hull2d(pts, mode: int = QH_EXACT_INT64, ctx: Context | None = None,
              timing: bool = False, stream=None, finish: bool = True, graph: bool = False,
              autotune: bool = False, out=None):
    """Counter-clockwise hull vertex indices (int32 tensor on the device) of
    int32[2, n] device points; returns (indices, stats dict).  ``out`` is an
    optional int32 output buffer of at least max(n, 1) elements (graph replay
    needs the same buffers on every call)."""
    lib = load()
    pts = _check_points(pts, 2)
    n = pts.shape[1]
    import torch
    out = _out_buffer(out, max(n, 1), torch.int32, pts.device, "out")
    h = ctypes.c_int64(0)
    o, stats = _opts(ctx, mode, timing, stream, finish, graph, autotune)
    st = lib.qh_hull2d(ctypes.c_void_p(pts.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                       ctypes.byref(h), ctypes.byref(o))
    if st != QH_OK:
        raise QhError(st, "qh_hull2d")
    return out[: h.value], stats.as_dict()


def qh_hull2d_batched(pts, offsets, mode: int = QH_EXACT_INT64, ctx: Context | None = None,
                      timing: bool = False, stream=None, finish: bool = True,
                      graph: bool = False, autotune: bool = False, out=None,
                      hull_offsets=None):
    """Hulls of the instances [offsets[i], offsets[i+1]) of int32[2, N] device
    points; offsets is an int64[k + 1] device tensor.  Returns (indices local
    to each instance, int64[k + 1] device hull offsets, stats dict).  ``out``
    (int32, at least max(N, 1)) and ``hull_offsets`` (int64, k + 1) are
    optional output buffers."""
    import torch
    lib = load()
    pts = _check_points(pts, 2)
    if offsets.dtype != torch.int64 or not offsets.is_cuda or offsets.dim() != 1:
        raise TypeError("offsets must be an int64 CUDA tensor of shape (k + 1,)")
    offsets = offsets.contiguous()
    k = offsets.shape[0] - 1
    n = pts.shape[1]
    out = _out_buffer(out, max(n, 1), torch.int32, pts.device, "out")
    hoff = _out_buffer(hull_offsets, k + 1, torch.int64, pts.device, "hull_offsets")[: k + 1]
    ht = ctypes.c_int64(0)
    o, stats = _opts(ctx, mode, timing, stream, finish, graph, autotune)
    st = lib.qh_hull2d_batched(ctypes.c_void_p(pts.data_ptr()), n,
                               ctypes.c_void_p(offsets.data_ptr()), k,
                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(hoff.data_ptr()),
                               ctypes.byref(ht), ctypes.byref(o))
    if st != QH_OK:
        raise QhError(st, "qh_hull2d_batched")
    return out[: ht.value], hoff, stats.as_dict()


def qh_hull3d(pts, mode: int = QH_EXACT_INT64, ctx: Context | None = None,
              timing: bool = False, stream=None):
    """3D hull of int32[3, n] device points: (facets int32[F, 3] on the device,
    vertices int32[V] on the device, stats dict)."""
    import torch
    lib = load()
    pts = _check_points(pts, 3)
    n = pts.shape[1]
    fac = torch.empty(3 * max(2 * n - 4, 4), dtype=torch.int32, device=pts.device)
    ver = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
    nf = ctypes.c_int64(0)
    nv = ctypes.c_int64(0)
    o, stats = _opts(ctx, mode, timing, stream)
    st = lib.qh_hull3d(ctypes.c_void_p(pts.data_ptr()), n, ctypes.c_void_p(fac.data_ptr()),
                       ctypes.byref(nf), ctypes.c_void_p(ver.data_ptr()), ctypes.byref(nv),
                       ctypes.byref(o))
    if st != QH_OK:
        raise QhError(st, "qh_hull3d")
    return fac[: 3 * nf.value].view(-1, 3), ver[: nv.value], stats.as_dict()


def qh_hull3d_batched(pts, offsets, mode: int = QH_EXACT_INT64, ctx: Context | None = None,
                      timing: bool = False, stream=None):
    """3D hulls of the instances [offsets[i], offsets[i+1]) of int32[3, N]
    device points; offsets is an int64[k + 1] device tensor.  Returns
    (facets int32[F, 3], facet offsets int64[k + 1], vertices int32[V],
    vertex offsets int64[k + 1], stats dict), all on the device, indices local
    to each instance."""
    import torch
    lib = load()
    pts = _check_points(pts, 3)
    if offsets.dtype != torch.int64 or not offsets.is_cuda or offsets.dim() != 1:
        raise TypeError("offsets must be an int64 CUDA tensor of shape (k + 1,)")
    offsets = offsets.contiguous()
    k = offsets.shape[0] - 1
    n = pts.shape[1]
    fac = torch.empty(max(6 * n, 3), dtype=torch.int32, device=pts.device)
    ver = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
    foff = torch.empty(k + 1, dtype=torch.int64, device=pts.device)
    voff = torch.empty(k + 1, dtype=torch.int64, device=pts.device)
    o, stats = _opts(ctx, mode, timing, stream)
    st = lib.qh_hull3d_batched(ctypes.c_void_p(pts.data_ptr()), n, ctypes.c_void_p(offsets.data_ptr()), k,
                               ctypes.c_void_p(fac.data_ptr()), ctypes.c_void_p(foff.data_ptr()),
                               ctypes.c_void_p(ver.data_ptr()), ctypes.c_void_p(voff.data_ptr()),
                               ctypes.byref(o))
    if st != QH_OK:
        raise QhError(st, "qh_hull3d_batched")
    nf = int(foff[-1].item())
    nv = int(voff[-1].item())
    return fac[: 3 * nf].view(-1, 3), foff, ver[: nv], voff, stats.as_dict()


def qh_test_flag_permute(f, s, k: int, stream=None, noalloc: bool = False):
    """k-state segmented stable partition of device int32 states f and uint8
    head flags s: returns (p int32, s_new uint8) device tensors.  noalloc:
    through qh_test_flag_permute_noalloc (the library's fixed scratch)."""
    import torch
    lib = load()
    if (not isinstance(f, torch.Tensor) or not f.is_cuda or f.dtype != torch.int32 or f.dim() != 1
            or not isinstance(s, torch.Tensor) or not s.is_cuda or s.dtype != torch.uint8
            or s.shape != f.shape):
        raise TypeError("f must be int32 and s uint8 CUDA tensors of one shape (n,)")
    f = f.contiguous()
    s = s.contiguous()
    n = f.shape[0]
    p = torch.empty(max(n, 1), dtype=torch.int32, device=f.device)
    s_new = torch.empty(max(n, 1), dtype=torch.uint8, device=f.device)
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    fn = lib.qh_test_flag_permute_noalloc if noalloc else lib.qh_test_flag_permute
    rc = fn(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(s.data_ptr()), n, int(k),
            ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(s_new.data_ptr()), ctypes.c_void_p(st))
    if rc != QH_OK:
        raise QhError(rc, "qh_test_flag_permute_noalloc" if noalloc else "qh_test_flag_permute")
    return p[:n], s_new[:n]


def qh_test_compact(b, s, stream=None):
    """Segmented compact of device uint8 keep flags b and head flags s:
    returns (p int32[n], s_new uint8[m], m)."""
    import torch
    lib = load()
    if (not isinstance(b, torch.Tensor) or not b.is_cuda or b.dtype != torch.uint8 or b.dim() != 1
            or not isinstance(s, torch.Tensor) or not s.is_cuda or s.dtype != torch.uint8
            or s.shape != b.shape):
        raise TypeError("b and s must be uint8 CUDA tensors of one shape (n,)")
    b = b.contiguous()
    s = s.contiguous()
    n = b.shape[0]
    p = torch.empty(max(n, 1), dtype=torch.int32, device=b.device)
    s_new = torch.empty(max(n, 1), dtype=torch.uint8, device=b.device)
    m = ctypes.c_int64(0)
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = lib.qh_test_compact(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(s.data_ptr()), n,
                             ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(s_new.data_ptr()),
                             ctypes.byref(m), ctypes.c_void_p(st))
    if rc != QH_OK:
        raise QhError(rc, "qh_test_compact")
    return p[:n], s_new[: m.value], m.value


def qh_select(vals, offsets, ranks, stream=None):
    """The ranks[i]-th smallest value (from 0) of every segment
    [offsets[i], offsets[i+1]) of the device int32 tensor vals: an int32[k]
    device tensor."""
    import torch
    lib = load()
    if not isinstance(vals, torch.Tensor) or not vals.is_cuda or vals.dtype != torch.int32 or vals.dim() != 1:
        raise TypeError("vals must be an int32 CUDA tensor of shape (n,)")
    for t, name in ((offsets, "offsets"), (ranks, "ranks")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int64 or t.dim() != 1:
            raise TypeError(f"{name} must be an int64 CUDA tensor")
    vals = vals.contiguous()
    offsets = offsets.contiguous()
    ranks = ranks.contiguous()
    k = offsets.shape[0] - 1
    if ranks.shape[0] != k:
        raise TypeError("ranks must have one entry per segment")
    out = torch.empty(max(k, 1), dtype=torch.int32, device=vals.device)
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = lib.qh_select(ctypes.c_void_p(vals.data_ptr()), vals.shape[0], ctypes.c_void_p(offsets.data_ptr()), k,
                       ctypes.c_void_p(ranks.data_ptr()), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st))
    if rc != QH_OK:
        raise QhError(rc, "qh_select")
    return out[:k]
