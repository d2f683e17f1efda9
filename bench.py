"""Benchmark of the segmented Quickhull on one MI355X.

One step = one qh_hull2d_batched call on the batched workload: 4,096
independent 2D point sets (sizes log-uniform in [256, 2^20], 511,371,962
points in total, each uniform in a disk of radius 2^20), every instance an
initial segment of one set of rounds (extremes, first split, every round,
output), with the points already resident in device memory.  The headline
is the faster of the two forms on this GPU, the plain exact-int64 form; the
FP32 filter with exact int64 fallback (bit-exact, the same output) is timed
beside it on the same data.

Prints ONE JSON line.  ``roofline`` describes the round kernels (k_split for
the first split, k_round_ro1 for the round after it, k_round for the later
rounds, each with k_round_multi for the tiles that hold several segments; in
the last round k_finish completes the remaining small segments in LDS, one
workgroup per segment or per run of consecutive segments), which move nearly all the
bytes: algorithmic bytes per round over the round's average duration, timed
with HIP events around the pair of launches on the stream they run on.  ``traffic`` is the counter-
measured HBM traffic per round from the committed rocprofv3 summary, null when
the kernel sources changed since it was taken.
``cpu_baseline`` is the oracle (plain single-threaded C Quickhull) on the
whole batch on one host core (a thread-pool figure beside it); the same leg,
the only one that runs the oracle, checks every GPU leg's output against it.
Sub-legs: ``square_16m`` (one hull of 16,777,216 points uniform in a square,
with its own roofline), ``regimes`` (65,536 and 4,194,304 points in a disk,
4,194,304 on and near a circle), ``hull3d`` (5,242,880 ball and sphere points
through qh_hull3d), ``hull3d_batched`` and ``select``.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "batched_disks"
SQUARE = "square_16m"
METRIC = "Mpoints/s per hull + HBM GB/s; FP32-filtered/batched vs exact-int64, bit-exact"
TRAFFIC_FILES = {w: os.path.join(ROOT, "profiles", f"traffic_round_{w}.json") for w in (WORKLOAD, SQUARE)}
CSRC = os.path.join(ROOT, "paper_1201_2936_amd", "csrc")


# the sources of the 2D kernels and of their launches: the round kernel's
# traffic depends on nothing else
KERNEL_SOURCES = ("qh2d_kernels.hip", "qh2d.h", "qh_device.h", "qh_api.hip", "qh_ctx.h")


def kernel_sha() -> str:
    """Hash of the 2D kernel sources and launch code: a traffic figure taken
    from other sources is stale."""
    h = hashlib.sha256()
    for name in sorted(KERNEL_SOURCES):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per round-kernel launch on ``workload`` from the committed
    PMC summary, or None when it is missing or was taken from another kernel
    source."""
    try:
        with open(TRAFFIC_FILES[workload]) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("bytes_per_launch")


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def _oracle_batched(oracle, pts, off, got, got_off):
    """The oracle on every instance of a batch: once in one call on one core,
    once over a pool of host threads (contiguous instance ranges of about
    equal point counts, several per thread; the C oracle runs without the
    interpreter lock).  Returns (the timings, parity of the whole batch)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    n = int(off[-1])
    k = len(off) - 1
    t0 = time.perf_counter()
    want, want_off = oracle.hull2d_batched(pts, off)
    t1 = time.perf_counter() - t0
    threads = max(1, min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "0")) or 10**6))
    parts = 4 * threads
    cuts = np.searchsorted(off, np.linspace(0, n, parts + 1)[1:-1])
    bounds = np.unique(np.concatenate([[0], cuts, [k]]))
    ranges = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]

    def part(r):
        a, b = r
        sub = np.ascontiguousarray(pts[:, off[a]:off[b]])
        return oracle.hull2d_batched(sub, off[a:b + 1] - off[a])

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(part, ranges))
    t2 = time.perf_counter() - t0
    pooled = np.concatenate([r[0] for r in res]) if res else np.zeros(0, np.int32)
    ok = bool(np.array_equal(want, got) and np.array_equal(want_off, got_off) and np.array_equal(pooled, want))
    timing = {"kind": "oracle", "unit": "Mpoints/s", "sample": f"all {k} instances ({n} points)",
              "single_core": {"value": round(n / t1 / 1e6, 3), "ms": round(t1 * 1e3, 1), "cores": 1},
              "thread_pool": {"value": round(n / t2 / 1e6, 3), "ms": round(t2 * 1e3, 1), "cores": threads}}
    return timing, ok


def oracle_leg(line, checks, budget_s: float = 12.0):
    """The leg that runs the oracle (a plain single-threaded C Quickhull,
    test infrastructure that no GPU leg calls).  ``cpu_baseline`` times it
    on the whole batch of the headline (one core, and a thread pool beside
    it); the square leg times it on its points for up to ``budget_s``; every
    GPU leg's output is compared with its result, whole or on a sample of
    instances."""
    import numpy as np

    import oracle

    oracle.hull2d(np.zeros((2, 4), np.int32))  # load / build outside the timing
    if "batched" in checks:
        sample = checks["batched"]["sample"]
        line["parity_vs_oracle_sample"] = {
            "instances": len(sample), "ok": bool(all(np.array_equal(oracle.hull2d(p), got) for p, got in sample))}
        timing, ok = _oracle_batched(oracle, *checks["batched"]["full"])
        line["parity_vs_oracle"] = ok
        one = timing["single_core"]
        line["cpu_baseline"] = {"value": one["value"], "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
                                "sample": f"{WORKLOAD}: {timing['sample']}, one run on one core "
                                          f"({one['ms'] / 1e3:.1f} s)",
                                "thread_pool": timing["thread_pool"]}
    if "square" in checks:
        pts = checks["square"][0]
        n = pts.shape[1]
        runs = 0
        t0 = time.perf_counter()
        while True:
            want = oracle.hull2d(pts)
            runs += 1
            el = time.perf_counter() - t0
            if el >= budget_s or runs >= 50:
                break
        sq = line[SQUARE]
        sq["cpu_baseline"] = {
            "value": round(n * runs / el / 1e6, 3), "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"{SQUARE} full ({n} points), {runs} runs in {el:.1f} s, single thread"}
        sq["parity_vs_oracle"] = bool(all(np.array_equal(got, want) for got in checks["square"][1:]))
    if "hull3d" in checks:
        p, gf, gv = checks["hull3d"][0]
        t0 = time.perf_counter()
        wf, wv = oracle.hull3d(p)
        line["hull3d"]["oracle_s"] = round(time.perf_counter() - t0, 2)
        line["hull3d"]["parity_vs_oracle"] = bool(np.array_equal(wf, gf) and np.array_equal(wv, gv))
    if "hull3d_batched" in checks:
        ok = True
        for p, gf, gv in checks["hull3d_batched"]:
            wf, wv = oracle.hull3d(p)
            ok &= bool(np.array_equal(wf, gf) and np.array_equal(wv, gv))
        line["hull3d_batched"]["parity_vs_oracle_sample"] = {"instances": len(checks["hull3d_batched"]),
                                                             "ok": bool(ok)}
    if "regimes" in checks:
        for name, (p, got) in checks["regimes"].items():
            t0 = time.perf_counter()
            want = oracle.hull2d(p)
            line["regimes"][name]["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
            line["regimes"][name]["parity_vs_oracle"] = bool(np.array_equal(want, got))


def round_roofline(timed_stats, traffic):
    """The round kernel's roofline from the per-launch HIP-event timings of
    some calls (QH_FLAG_TIMING): algorithmic bytes per launch over the
    average launch duration."""
    bpl = sum(s["round_kernel_bytes"] for s in timed_stats) / max(1, sum(s["round_launches"] for s in timed_stats))
    avg_ms = sum(s["round_kernel_ms"] for s in timed_stats) / max(1, sum(s["round_launches"] for s in timed_stats))
    ach = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic}
    return roof, bpl, avg_ms


def tuned_graph_leg(call, key, want, steps, outs, out_names):
    """Time a call with QH_FLAG_AUTOTUNE and QH_FLAG_GRAPH on a stream of its
    own with fixed output buffers (the first call tunes and captures); check
    the output against ``want``."""
    import torch

    from paper_1201_2936_amd import qh
    ctx = qh.Context()
    st = torch.cuda.Stream()
    kw = dict(ctx=ctx, autotune=True, graph=True, stream=st.cuda_stream)
    kw.update(zip(out_names, outs))
    with torch.cuda.stream(st):
        first = call(**kw)
        st.synchronize()
        sec, last = time_steps(lambda: call(**kw), steps, 2)
        same = all(bool(torch.equal(a, b)) for a, b in zip(key(last), want))
    s0, s1 = first[-1], last[-1]
    ctx.close()
    return {"ms_per_step": round(sec * 1e3, 4), "tuned_configs": int(s0["tuned_configs"]),
            "grid_blocks": int(s1["grid_blocks"]), "multi_blocks": int(s1["multi_blocks"]),
            "finish_segments": int(s1["finish_segments"]),
            "graph_launches_per_call": int(s1["graph_launches"]), "same_output": same}


def batched_leg(steps: int, warmup: int):
    """The headline: the batched form on 4,096 disks (sizes log-uniform in
    [256, 2^20], 511,371,962 points) in one qh_hull2d_batched call per step,
    FP32 filter; the exact form, the tuned launch configuration with graph
    replay and 4,096 sequential qh_hull2d calls on the same device-resident
    instances beside it."""
    import numpy as np
    import torch

    import workloads
    from paper_1201_2936_amd import qh

    t0 = time.perf_counter()
    pts_np, off_np = workloads.batched_disks()
    gen_s = time.perf_counter() - t0
    k = len(off_np) - 1
    N = int(off_np[-1])
    pts = torch.from_numpy(pts_np).cuda()
    off = torch.from_numpy(off_np).cuda()
    ctx = qh.Context()

    def run(mode):
        return qh.qh_hull2d_batched(pts, off, mode=mode, ctx=ctx)

    # the headline form (exact int64) and the FP32 filter beside it
    sec_x, (idx_x, hoff_x, st_x) = time_steps(lambda: run(qh.QH_EXACT_INT64), steps, warmup)
    sec_f, (idx_f, hoff_f, st_f) = time_steps(lambda: run(qh.QH_FP32_FILTER), max(3, min(steps, 10)), 1)
    same = bool(torch.equal(idx_f, idx_x) and torch.equal(hoff_f, hoff_x))

    # the launch configuration picked by the autotuner, the launches replayed
    # from captured graphs (fixed output buffers, a stream of its own)
    tuned = tuned_graph_leg(lambda **kw: qh.qh_hull2d_batched(pts, off, mode=qh.QH_EXACT_INT64, **kw),
                            lambda o: (o[0], o[1]), (idx_x, hoff_x), max(3, min(steps, 10)),
                            [torch.empty(max(N, 1), dtype=torch.int32, device="cuda"),
                             torch.empty_like(hoff_x)], ["out", "hull_offsets"])

    # per-launch kernel timing (HIP events around every launch, on the
    # stream the kernels run on): a separate pass of the same call
    timed = [qh.qh_hull2d_batched(pts, off, mode=qh.QH_EXACT_INT64, ctx=ctx, timing=True)[2]
             for _ in range(3)]
    roof, bpl, avg_ms = round_roofline(timed, load_traffic(WORKLOAD))
    timed_f = [qh.qh_hull2d_batched(pts, off, mode=qh.QH_FP32_FILTER, ctx=ctx, timing=True)[2]
               for _ in range(3)]
    roof_f, _, avg_ms_f = round_roofline(timed_f, None)
    nt = len(timed)

    def tavg(key):
        return sum(s[key] for s in timed) / nt

    # 4,096 sequential single-hull calls on contiguous per-instance copies
    singles = [torch.stack([pts[0, off_np[i]:off_np[i + 1]], pts[1, off_np[i]:off_np[i + 1]]]).contiguous()
               for i in range(k)]
    sctx = qh.Context()
    for i in range(min(k, 64)):
        qh.qh_hull2d(singles[i], mode=qh.QH_EXACT_INT64, ctx=sctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_ok = True
    hoff_host = hoff_x.cpu().numpy()
    idx_host = idx_x.cpu().numpy()
    for i in range(k):
        one, _ = qh.qh_hull2d(singles[i], mode=qh.QH_EXACT_INT64, ctx=sctx)
        if i % 64 == 0:
            seq_ok &= np.array_equal(one.cpu().numpy(), idx_host[hoff_host[i]:hoff_host[i + 1]])
    torch.cuda.synchronize()
    sec_seq = time.perf_counter() - t0

    # a sample of instances, and the whole batch, for the oracle leg
    check = {"sample": [(np.ascontiguousarray(pts_np[:, off_np[i]:off_np[i + 1]]),
                         idx_host[hoff_host[i]:hoff_host[i + 1]].copy()) for i in range(0, k, 97)],
             "full": (pts_np, off_np, idx_host, hoff_host)}
    sctx.close()
    ctx.close()
    del singles, pts, off
    torch.cuda.empty_cache()
    part = {
        "value": round(N / sec_x / 1e6, 3),
        "ms_per_step": round(sec_x * 1e3, 4),
        "config": {"workload": WORKLOAD, "instances": k, "n_total": N, "dims": 2,
                   "sizes": "log-uniform in [256, 2^20] (seed 5)",
                   "coords": "int32 uniform in the disk of radius 2^20", "form": "exact_int64",
                   "call": "qh_hull2d_batched"},
        "fp32_filter": {"value": round(N / sec_f / 1e6, 3), "unit": "Mpoints/s",
                        "ms_per_step": round(sec_f * 1e3, 4), "dtype": "f32+i64",
                        "fallback_rate": (st_f["filter_fallbacks"] / st_f["filter_tests"])
                        if st_f["filter_tests"] else 0.0,
                        "argmax_candidates": int(st_f["argmax_candidates"]),
                        "round_kernel_avg_launch_us": round(avg_ms_f * 1e3, 2),
                        "roofline": roof_f},
        "autotuned_graph": tuned,
        "sequential_single_calls": {"value": round(N / sec_seq / 1e6, 3), "unit": "Mpoints/s",
                                    "ms": round(sec_seq * 1e3, 1), "calls": k,
                                    "match_batched": bool(seq_ok)},
        "modes_identical": same,
        "generate_s": round(gen_s, 1),
        "hull_vertices": int(hoff_host[-1]),
        "parity_vs_oracle_sample": None,
        "parity_vs_oracle": None,
        "rounds": int(st_x["rounds"]),
        "finish_round": int(st_x["finish_round"]),
        "finish_runs": int(st_x["finish_runs"]),
        "round_kernel": {"name": "k_split, k_round_ro1, k_round, each with k_round_multi and k_finish (the "
                                 "first split, the round after it, the later rounds; the last round "
                                 "finishing small segments)",
                         "launches_per_step": tavg("round_launches"), "avg_launch_us": round(avg_ms * 1e3, 2),
                         "bytes_per_launch": round(bpl), "grid_blocks": int(st_x["grid_blocks"]),
                         "first_split_us": round(tavg("split_ms") * 1e3, 1)},
        "device_time_us": {"all_kernels": round(tavg("kernel_ms") * 1e3, 1),
                           "rounds": round(tavg("round_kernel_ms") * 1e3, 1),
                           "extremes": round(tavg("extremes_ms") * 1e3, 1),
                           "segments": round(tavg("segment_ms") * 1e3, 1)},
        "hull_GBs_device": round(tavg("hull_bytes") / (tavg("kernel_ms") * 1e-3) / 1e9, 1)
        if tavg("kernel_ms") > 0 else None,
        "roofline": roof,
    }
    return part, check


def square_leg(steps: int):
    """One hull of 16,777,216 points uniform in [-2^20, 2^20]^2 through
    qh_hull2d, both forms, with its own round-kernel roofline."""
    import torch

    import workloads
    from paper_1201_2936_amd import qh

    pts_np = workloads.WORKLOADS[SQUARE]()
    n = pts_np.shape[1]
    pts = torch.from_numpy(pts_np).cuda()
    ctx = qh.Context()
    sec, (idx_f, st_f) = time_steps(lambda: qh.qh_hull2d(pts, mode=qh.QH_FP32_FILTER, ctx=ctx), steps, 3)
    sec_x, (idx_x, _) = time_steps(lambda: qh.qh_hull2d(pts, mode=qh.QH_EXACT_INT64, ctx=ctx), steps, 3)
    tuned = tuned_graph_leg(lambda **kw: qh.qh_hull2d(pts, mode=qh.QH_EXACT_INT64, **kw),
                            lambda o: (o[0],), (idx_x,), steps,
                            [torch.empty(max(n, 1), dtype=torch.int32, device="cuda")], ["out"])
    # the round kernels' roofline in the faster (exact) form
    timed = [qh.qh_hull2d(pts, mode=qh.QH_EXACT_INT64, ctx=ctx, timing=True)[1] for _ in range(steps)]
    roof, bpl, avg_ms = round_roofline(timed, load_traffic(SQUARE))
    nt = len(timed)
    split_ms = sum(s["split_ms"] for s in timed) / nt
    split_bytes = 8 * n  # the split reads the input and writes nothing
    check = (pts_np, idx_f.cpu().numpy(), idx_x.cpu().numpy())
    ctx.close()
    del pts
    torch.cuda.empty_cache()
    return {
        "workload": f"{SQUARE}: {n} points, int32 uniform in [-2^20, 2^20]^2, one qh_hull2d call",
        "n": n,
        "fp32_filter": {"value": round(n / sec / 1e6, 3), "unit": "Mpoints/s", "ms_per_step": round(sec * 1e3, 4)},
        "exact_int64": {"value": round(n / sec_x / 1e6, 3), "unit": "Mpoints/s",
                        "ms_per_step": round(sec_x * 1e3, 4)},
        "autotuned_graph": tuned,
        "hull_vertices": int(idx_f.numel()),
        "parity_vs_oracle": None,
        "modes_identical": bool(torch.equal(idx_f, idx_x)),
        "rounds": int(st_f["rounds"]),
        "fallback_rate": (st_f["filter_fallbacks"] / st_f["filter_tests"] if st_f["filter_tests"] else 0.0),
        "argmax_candidates": int(st_f["argmax_candidates"]),
        "round_kernel": {"launches_per_step": sum(s["round_launches"] for s in timed) / nt,
                         "avg_launch_us": round(avg_ms * 1e3, 3), "bytes_per_launch": round(bpl),
                         "first_split_us": round(split_ms * 1e3, 2),
                         "first_split_GBs": round(split_bytes / (split_ms * 1e-3) / 1e9, 1) if split_ms > 0 else None},
        "device_time_us": {"all_kernels": round(sum(s["kernel_ms"] for s in timed) / nt * 1e3, 2),
                           "extremes": round(sum(s["extremes_ms"] for s in timed) / nt * 1e3, 2),
                           "segments": round(sum(s["segment_ms"] for s in timed) / nt * 1e3, 2)},
        "roofline": roof,
    }, check


def regimes_leg(steps: int):
    """The input regimes the paper times (Section 5): points in a disk against
    points on and near a circle, at the same size (4,194,304), and the small
    disk.  Both forms on each; the circle's slowdown over the disk is the
    figure the paper reports for its own GPU (Section 6)."""
    import torch

    import workloads
    from paper_1201_2936_amd import qh

    cases = [("disk_65k", workloads.disk_65k), ("disk_4m", workloads.disk_4m),
             ("circle_mix_4m", workloads.circle_mix_4m)]
    ctx = qh.Context()
    out, check = {}, {}
    for name, gen in cases:
        p_np = gen()
        n = p_np.shape[1]
        p = torch.from_numpy(p_np).cuda()
        sec_f, (idx_f, st_f) = time_steps(lambda: qh.qh_hull2d(p, mode=qh.QH_FP32_FILTER, ctx=ctx), steps, 2)
        sec_x, (idx_x, _) = time_steps(lambda: qh.qh_hull2d(p, mode=qh.QH_EXACT_INT64, ctx=ctx), steps, 2)
        _, tt = qh.qh_hull2d(p, mode=qh.QH_FP32_FILTER, ctx=ctx, timing=True)
        out[name] = {
            "n": n, "hull_vertices": int(idx_f.numel()), "rounds": int(st_f["rounds"]),
            "finish_round": int(st_f["finish_round"]),
            "fp32_filter": {"value": round(n / sec_f / 1e6, 3), "unit": "Mpoints/s",
                            "ms_per_step": round(sec_f * 1e3, 4)},
            "exact_int64": {"value": round(n / sec_x / 1e6, 3), "unit": "Mpoints/s",
                            "ms_per_step": round(sec_x * 1e3, 4)},
            "fallback_rate": (st_f["filter_fallbacks"] / st_f["filter_tests"]) if st_f["filter_tests"] else 0.0,
            "device_time_us": {"all_kernels": round(tt["kernel_ms"] * 1e3, 1),
                               "rounds": round(tt["round_kernel_ms"] * 1e3, 1),
                               "segments": round(tt["segment_ms"] * 1e3, 1)},
            "modes_identical": bool(torch.equal(idx_f, idx_x)),
            "parity_vs_oracle": None,
        }
        check[name] = (p_np, idx_f.cpu().numpy())
        del p
    ctx.close()
    torch.cuda.empty_cache()
    out["circle_over_disk_4m"] = {
        form: round(out["circle_mix_4m"][form]["ms_per_step"] / out["disk_4m"][form]["ms_per_step"], 2)
        for form in ("fp32_filter", "exact_int64")}
    return out, check


def hull3d_leg(steps: int):
    """The 3D form on 4,194,304 points in the ball of radius 2^16 plus
    1,048,576 snapped to its sphere (5,242,880 in total), exact int64 and FP32
    filter, through qh_hull3d."""
    import numpy as np
    import torch

    import workloads
    from paper_1201_2936_amd import qh

    pts_np = workloads.ball_sphere_5m()
    n = pts_np.shape[1]
    pts = torch.from_numpy(pts_np).cuda()
    ctx = qh.Context()
    sec_x, (f_x, v_x, st_x) = time_steps(lambda: qh.qh_hull3d(pts, mode=qh.QH_EXACT_INT64, ctx=ctx),
                                         steps, 1)
    sec_f, (f_f, v_f, st_f) = time_steps(lambda: qh.qh_hull3d(pts, mode=qh.QH_FP32_FILTER, ctx=ctx),
                                         steps, 1)
    same = bool(torch.equal(f_x, f_f) and torch.equal(v_x, v_f))
    _, _, tt = qh.qh_hull3d(pts, mode=qh.QH_EXACT_INT64, ctx=ctx, timing=True)
    check = [(pts_np, f_x.cpu().numpy(), v_x.cpu().numpy())]
    ctx.close()
    return {
        "workload": "ball_sphere_5m: 4,194,304 in the ball of radius 2^16 + 1,048,576 on its sphere",
        "n": n, "vertices": int(v_x.numel()), "facets": int(f_x.shape[0]),
        "exact_int64": {"value": round(n / sec_x / 1e6, 3), "unit": "Mpoints/s",
                        "ms_per_step": round(sec_x * 1e3, 2)},
        "fp32_filter": {"value": round(n / sec_f / 1e6, 3), "unit": "Mpoints/s",
                        "ms_per_step": round(sec_f * 1e3, 2),
                        "fallback_rate": (st_f["filter_fallbacks"] / st_f["filter_tests"])
                        if st_f["filter_tests"] else 0.0},
        "modes_identical": same, "parity_vs_oracle": None,
        "rounds": int(st_x["rounds"]), "host_syncs": int(st_x["host_syncs"]),
        "max_active_facets": int(st_x["max_segments"]),
        "host_topology_ms": round(tt["host_ms"], 2),
        "device_ms": {"classify": round(tt["round_kernel_ms"], 3), "apex": round(tt["segment_ms"], 3),
                      "init": round(tt["extremes_ms"], 3), "all": round(tt["kernel_ms"], 3)},
        "classify_apex_GBs": round(tt["round_kernel_bytes"] / ((tt["round_kernel_ms"] + tt["segment_ms"]) * 1e-3) / 1e9, 1)
        if tt["round_kernel_ms"] > 0 else None,
    }, check


def hull3d_batched_leg(steps: int):
    """The batched 3D form on 512 ball-and-sphere sets (sizes log-uniform in
    [64, 16384], 1,650,780 points) in one qh_hull3d_batched call, beside
    512 sequential qh_hull3d calls on the same device-resident instances."""
    import numpy as np
    import torch

    import workloads
    from paper_1201_2936_amd import qh

    pts_np, off_np = workloads.batched_balls3d()
    k = len(off_np) - 1
    N = int(off_np[-1])
    pts = torch.from_numpy(pts_np).cuda()
    off = torch.from_numpy(off_np).cuda()
    ctx = qh.Context()
    sec_b, (fac, foff, ver, voff, st) = time_steps(
        lambda: qh.qh_hull3d_batched(pts, off, mode=qh.QH_EXACT_INT64, ctx=ctx), steps, 1)
    fac, foff, ver, voff = fac.cpu().numpy(), foff.cpu().numpy(), ver.cpu().numpy(), voff.cpu().numpy()
    singles = [pts[:, off_np[i]:off_np[i + 1]].contiguous() for i in range(k)]
    sctx = qh.Context()
    qh.qh_hull3d(singles[0], ctx=sctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same = True
    outs = [qh.qh_hull3d(s, mode=qh.QH_EXACT_INT64, ctx=sctx) for s in singles]
    torch.cuda.synchronize()
    sec_seq = time.perf_counter() - t0
    for i, (f1, v1, _) in enumerate(outs):
        same &= (np.array_equal(f1.cpu().numpy(), fac[foff[i]:foff[i + 1]]) and
                 np.array_equal(v1.cpu().numpy(), ver[voff[i]:voff[i + 1]]))
    check = [(np.ascontiguousarray(pts_np[:, off_np[i]:off_np[i + 1]]), fac[foff[i]:foff[i + 1]].copy(),
              ver[voff[i]:voff[i + 1]].copy()) for i in range(0, k, 37)]
    sctx.close()
    ctx.close()
    return {
        "workload": "batched_balls3d: 512 sets, 3/4 in the ball of radius 2^16 and 1/4 on its sphere, "
                    "sizes log-uniform in [64, 16384]",
        "n_total": N, "k": k,
        "exact_int64": {"value": round(N / sec_b / 1e6, 3), "unit": "Mpoints/s",
                        "ms_per_step": round(sec_b * 1e3, 2), "steps": steps},
        "sequential_single_calls": {"value": round(N / sec_seq / 1e6, 3), "unit": "Mpoints/s",
                                    "ms": round(sec_seq * 1e3, 1), "calls": k, "match_batched": bool(same)},
        "parity_vs_oracle_sample": None,
        "rounds": int(st["rounds"]), "facets": int(foff[-1]), "vertices": int(voff[-1]),
        "host_topology_ms": round(st["host_ms"], 2),
    }, check


def select_leg(steps: int):
    """Order statistics from flagPermute + compact (qh_select): the medians
    of 1,024 segments of 1,024 random int32 values each (1,048,576 values)."""
    import numpy as np
    import torch

    import workloads
    from paper_1201_2936_amd import qh

    rng = workloads.rng_for(9)
    k, m = 1024, 1024
    vals_np = rng.integers(-(1 << 30), 1 << 30, size=k * m).astype(np.int32)
    off_np = (np.arange(k + 1, dtype=np.int64) * m)
    rk_np = np.full(k, m // 2, np.int64)
    vals = torch.from_numpy(vals_np).cuda()
    off = torch.from_numpy(off_np).cuda()
    rk = torch.from_numpy(rk_np).cuda()
    sec, out = time_steps(lambda: qh.qh_select(vals, off, rk), steps, 1)
    want = np.sort(vals_np.reshape(k, m), axis=1)[:, m // 2]
    return {"workload": "select_medians: 1,024 segments x 1,024 int32 values (seed 9), rank 512 each",
            "value": round(k * m / sec / 1e6, 3), "unit": "Mvalues/s", "ms_per_step": round(sec * 1e3, 3),
            "steps": steps, "matches_sort": bool(np.array_equal(out.cpu().numpy(), want))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D legs")
    ap.add_argument("--no-regimes", action="store_true", help="skip the disk and circle leg")
    ap.add_argument("--no-square", action="store_true", help="skip the 16.7M-point square leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (every hull of the batch on one "
              "MI355X); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    from paper_1201_2936_amd import qh

    qh.load()
    head, check_b = batched_leg(args.steps, args.warmup)
    checks = {"batched": check_b}
    line = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i64",
        "data": "synthetic",
        "config": head.pop("config"),
        "roofline": head.pop("roofline"),
        "cpu_baseline": None,
    }
    line.update(head)
    sub = max(3, min(args.steps, 10))
    if not args.no_square:
        line[SQUARE], checks["square"] = square_leg(sub)
    if not args.no_regimes:
        line["regimes"], checks["regimes"] = regimes_leg(sub)
    if not args.no_3d:
        line["hull3d"], checks["hull3d"] = hull3d_leg(max(2, min(args.steps, 3)))
        line["hull3d_batched"], checks["hull3d_batched"] = hull3d_batched_leg(max(2, min(args.steps, 3)))
    line["select"] = select_leg(5)
    if not args.no_cpu_baseline:
        oracle_leg(line, checks)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
