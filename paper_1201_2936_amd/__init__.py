"""Segmented data-parallel Quickhull (Tzeng & Owens) on AMD Instinct MI355X.

The hull runs in the HIP library ``libqh.so`` (see ``include/qh.h``);
``qh`` is its ctypes binding.
"""
from .qh import (QH_EXACT_INT64, QH_FP32_FILTER, Context, QhError, load,  # noqa: F401
                 qh_hull2d, qh_hull2d_batched, status_str, version)
