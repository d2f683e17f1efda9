"""The bench's oracle leg on the CPU: it must report parity only when every
kept GPU output equals the oracle's, and name the leg that differs.

The "GPU outputs" here are the oracle's own results (or altered copies), so
the test needs no GPU; it checks the bookkeeping of bench.oracle_leg.
"""
import numpy as np

import bench
import oracle
import workloads


def _full(inst):
    off = np.zeros(len(inst) + 1, np.int64)
    np.cumsum([q.shape[1] for q in inst], out=off[1:])
    pts = np.ascontiguousarray(np.concatenate(inst, axis=1))
    got, got_off = oracle.hull2d_batched(pts, off)
    return pts, off, got, got_off


def _checks():
    p = workloads.small_random(21, 3000, 1 << 20)
    w = oracle.hull2d(p)
    inst = [workloads.small_random(30 + i, 200, 1000) for i in range(3)]
    p3 = workloads.small_ball3(5, 300, 1000)
    f3, v3 = oracle.hull3d(p3)
    return {
        "square": (p, w.copy(), w.copy()),
        "batched": {"sample": [(q, oracle.hull2d(q)) for q in inst], "full": _full(inst)},
        "hull3d": [(p3, f3.copy(), v3.copy())],
        "hull3d_batched": [(p3, f3.copy(), v3.copy())],
        "regimes": {"disk_65k": (p, w.copy())},
    }


def _line():
    return {bench.SQUARE: {}, "hull3d": {}, "hull3d_batched": {}, "regimes": {"disk_65k": {}}}


def test_oracle_leg_all_equal():
    line = _line()
    bench.oracle_leg(line, _checks(), budget_s=0.05)
    assert line["parity_vs_oracle"] is True
    assert line["parity_vs_oracle_sample"] == {"instances": 3, "ok": True}
    assert line[bench.SQUARE]["parity_vs_oracle"] is True
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0 and cb["unit"] == "Mpoints/s"
    assert cb["thread_pool"]["cores"] >= 1 and cb["thread_pool"]["value"] > 0
    assert line["hull3d"]["parity_vs_oracle"] is True
    assert line["hull3d_batched"]["parity_vs_oracle_sample"]["ok"] is True
    assert line["regimes"]["disk_65k"]["parity_vs_oracle"] is True
    cs = line[bench.SQUARE]["cpu_baseline"]
    assert cs["kind"] == "oracle" and cs["cores"] == 1 and cs["value"] > 0


def test_oracle_leg_reports_each_mismatch():
    c = _checks()
    p, w, _ = c["square"]
    c["square"] = (p, w, w[::-1].copy())                   # the exact form differs
    q, g = c["batched"]["sample"][1]
    c["batched"]["sample"][1] = (q, g[:-1])                # one instance lost a vertex
    pts, off, got, got_off = c["batched"]["full"]
    c["batched"]["full"] = (pts, off, got[::-1].copy(), got_off)  # the whole batch reordered
    p3, f3, v3 = c["hull3d"][0]
    f3b = f3.copy()
    f3b[0] = f3b[0][::-1]                                  # one facet flipped
    c["hull3d"] = [(p3, f3b, v3)]
    line = _line()
    bench.oracle_leg(line, c, budget_s=0.05)
    assert line[bench.SQUARE]["parity_vs_oracle"] is False
    assert line["parity_vs_oracle_sample"]["ok"] is False
    assert line["parity_vs_oracle"] is False
    assert line["hull3d"]["parity_vs_oracle"] is False
    assert line["hull3d_batched"]["parity_vs_oracle_sample"]["ok"] is True
    assert line["regimes"]["disk_65k"]["parity_vs_oracle"] is True
    assert isinstance(line["parity_vs_oracle"], bool)
