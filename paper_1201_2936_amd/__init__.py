"""Segmented data-parallel Quickhull (Tzeng & Owens) on AMD Instinct MI355X.

The hull runs in the HIP library ``libqh.so`` (see ``include/qh.h``);
``qh`` is its ctypes binding.
"""
from .qh import (QH_EXACT_INT64, QH_FP32_FILTER, Context, QhError, load,  # noqa: F401
                 qh_hull2d, qh_hull2d_batched, qh_hull3d, qh_hull3d_batched, qh_select,
                 qh_test_compact, qh_test_flag_permute, status_str, version)
