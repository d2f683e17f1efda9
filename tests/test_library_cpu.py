"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/qh.h, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_1201_2936_amd import qh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(qh_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = qh.load()
    declared = _declared()
    assert {"qh_hull2d", "qh_hull2d_batched", "qh_ctx_create"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(qh.EXPORTED) <= declared


def test_status_strings_and_version():
    assert qh.status_str(qh.QH_OK) == "ok"
    assert "range" in qh.status_str(qh.QH_ERANGE)
    assert qh.version().startswith("qh")


def test_argument_validation_without_device():
    lib = qh.load()
    h = ctypes.c_int64(123)
    # negative n, null count pointer
    assert lib.qh_hull2d(None, -1, None, ctypes.byref(h), None) == qh.QH_EINVAL
    assert h.value == 0
    assert lib.qh_hull2d(None, 5, None, None, None) == qh.QH_EINVAL
    # n > 0 with null buffers
    assert lib.qh_hull2d(None, 5, None, ctypes.byref(h), None) == qh.QH_EINVAL
    # n = 0 is an empty hull, no device work
    assert lib.qh_hull2d(None, 0, None, ctypes.byref(h), None) == qh.QH_OK and h.value == 0
    ht = ctypes.c_int64(7)
    assert lib.qh_hull2d_batched(None, 10, None, 0, None, None, ctypes.byref(ht), None) == qh.QH_EINVAL
    assert lib.qh_hull2d_batched(None, -1, None, 1, None, None, ctypes.byref(ht), None) == qh.QH_EINVAL
    assert ht.value == 0


def test_bad_mode_rejected():
    lib = qh.load()
    o = qh.QhOpts(None, 7, 0, None, None)
    h = ctypes.c_int64(0)
    # rejected before any device call only when n == 0 is not the case; n = 0
    # returns early, so use a null pointer with n > 0 which is EINVAL as well
    assert lib.qh_hull2d(None, 3, None, ctypes.byref(h), ctypes.byref(o)) == qh.QH_EINVAL


def test_no_oracle_import_in_product():
    pkg = os.path.join(ROOT, "paper_1201_2936_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "qh_oracle" not in text and "qho_" not in text, fn


def test_graph_flag_needs_a_stream():
    lib = qh.load()
    h = ctypes.c_int64(9)
    dummy = ctypes.c_void_p(16)  # never dereferenced: the check comes first
    o = qh.QhOpts(None, qh.QH_EXACT_INT64, qh.QH_FLAG_GRAPH, None, None)
    assert lib.qh_hull2d(dummy, 5, dummy, ctypes.byref(h), ctypes.byref(o)) == qh.QH_EINVAL
    assert h.value == 0
    assert lib.qh_hull2d_batched(dummy, 5, dummy, 1, dummy, dummy, ctypes.byref(h),
                                 ctypes.byref(o)) == qh.QH_EINVAL


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of qh_stats and qh_opts, and the flag values, agree
    with include/qh.h as a C compiler lays them out."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    stats = [name for name, _ in qh.QhStats._fields_]
    opts = [name for name, _ in qh.QhOpts._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qh.h"', "int main(void) {",
             'printf("stats %zu\\n", sizeof(qh_stats));', 'printf("opts %zu\\n", sizeof(qh_opts));']
    lines += [f'printf("s.{f} %zu\\n", offsetof(qh_stats, {f}));' for f in stats]
    lines += [f'printf("o.{f} %zu\\n", offsetof(qh_opts, {f}));' for f in opts]
    flags = ["QH_FLAG_TIMING", "QH_FLAG_NO_FINISH", "QH_FLAG_GRAPH", "QH_FLAG_AUTOTUNE",
             "QH_EXACT_INT64", "QH_FP32_FILTER", "QH_FINISH_CAP"]
    lines += [f'printf("c.{f} %d\\n", (int){f});' for f in flags]
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    assert int(got["stats"]) == ctypes.sizeof(qh.QhStats)
    assert int(got["opts"]) == ctypes.sizeof(qh.QhOpts)
    for f in stats:
        assert int(got["s." + f]) == getattr(qh.QhStats, f).offset, f
    for f in opts:
        assert int(got["o." + f]) == getattr(qh.QhOpts, f).offset, f
    for f in flags:
        assert int(got["c." + f]) == getattr(qh, f), f


def test_batched3d_argument_validation_without_device():
    lib = qh.load()
    dummy = ctypes.c_void_p(16)  # never dereferenced: the checks come first
    # k out of range, negative n, missing offsets or outputs
    assert lib.qh_hull3d_batched(dummy, 10, dummy, 0, dummy, dummy, dummy, dummy, None) == qh.QH_EINVAL
    assert lib.qh_hull3d_batched(dummy, -1, dummy, 1, dummy, dummy, dummy, dummy, None) == qh.QH_EINVAL
    assert lib.qh_hull3d_batched(dummy, 10, None, 1, dummy, dummy, dummy, dummy, None) == qh.QH_EINVAL
    assert lib.qh_hull3d_batched(dummy, 10, dummy, 1, None, dummy, dummy, dummy, None) == qh.QH_EINVAL
    assert lib.qh_hull3d_batched(dummy, 10, dummy, 1, dummy, None, dummy, dummy, None) == qh.QH_EINVAL
    o = qh.QhOpts(None, 9, 0, None, None)
    assert lib.qh_hull3d_batched(dummy, 10, dummy, 1, dummy, dummy, dummy, dummy, ctypes.byref(o)) == qh.QH_EINVAL


def test_segmented_primitives_argument_validation_without_device():
    lib = qh.load()
    dummy = ctypes.c_void_p(16)  # never dereferenced: the checks come first
    m = ctypes.c_int64(5)
    assert lib.qh_test_compact(dummy, dummy, -1, dummy, dummy, ctypes.byref(m), None) == qh.QH_EINVAL
    assert m.value == 0
    assert lib.qh_test_compact(dummy, dummy, 0, dummy, dummy, ctypes.byref(m), None) == qh.QH_OK
    assert lib.qh_test_compact(dummy, dummy, 4, None, dummy, ctypes.byref(m), None) == qh.QH_EINVAL
    assert lib.qh_select(dummy, 10, dummy, 0, dummy, dummy, None) == qh.QH_EINVAL
    assert lib.qh_select(dummy, 10, None, 1, dummy, dummy, None) == qh.QH_EINVAL
    assert lib.qh_select(dummy, 10, dummy, 1, dummy, None, None) == qh.QH_EINVAL
    assert lib.qh_select(None, 10, dummy, 1, dummy, dummy, None) == qh.QH_EINVAL
