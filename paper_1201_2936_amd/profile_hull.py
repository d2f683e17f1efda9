"""Driver for profiler runs, and the summary of what they measured.

Run (a few hulls of one workload; optionally first a plain device copy of
known size whose counters calibrate the HBM byte counters of the same run):

    rocprofv3 --kernel-trace --stats -d OUT -o run -- python3 -m paper_1201_2936_amd.profile_hull
    rocprofv3 --pmc FETCH_SIZE --kernel-trace -d OUT -o run -- \
        python3 -m paper_1201_2936_amd.profile_hull --copy-mb 256

Summarize (kernel statistics from a trace database, HBM traffic per launch of
one kernel from a FETCH_SIZE and a WRITE_SIZE database, both scaled by what the
counters read for the copy):

    python3 -m paper_1201_2936_amd.profile_hull summarize --trace T.db \
        --fetch F.db --write W.db --kernel k_round --copy-mb 256 --out SUMMARY.md
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _kernel_rows(db_path):
    import sqlite3
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    cur.execute("select name, start, end from kernels order by start")
    return cur.fetchall()


def _counter_rows(db_path, counter):
    import sqlite3
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    cur.execute("select dispatch_id, kernel_name, value from counters_collection "
                "where counter_name = ? order by dispatch_id", (counter,))
    per = {}
    for disp, name, val in cur.fetchall():
        k = per.setdefault(disp, [name, 0.0])
        k[1] += val
    return [tuple(v) for _, v in sorted(per.items())]


def _short(name):
    import re
    return re.sub(r"\(.*", "", name).replace("void ", "").replace("qh::", "")


def summarize(args):
    import json
    lines = []
    if args.trace:
        rows = _kernel_rows(args.trace)
        stats = {}
        for name, s, e in rows:
            st = stats.setdefault(_short(name), [0, 0.0])
            st[0] += 1
            st[1] += (e - s) / 1e3
        lines.append("| kernel | calls | total us | average us |")
        lines.append("|---|---|---|---|")
        for name, (calls, tot) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
            lines.append(f"| {name} | {calls} | {tot:.1f} | {tot / calls:.2f} |")
    if args.stats_csv:
        import csv
        with open(args.stats_csv) as fh:
            rows = list(csv.DictReader(fh))
        lines.append("| kernel | calls | total us | average us | % | min us | max us |")
        lines.append("|---|---|---|---|---|---|---|")
        for r in rows:
            lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                         f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} | "
                         f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    if args.counters:
        # every counter of the run, summed per dispatch, for the kernels named
        import sqlite3
        db = sqlite3.connect(args.counters)
        cur = db.cursor()
        cur.execute("select dispatch_id, kernel_name, counter_name, sum(value) from counters_collection "
                    "group by dispatch_id, counter_name order by dispatch_id")
        names = args.kernel.split(",")
        per = {}
        for disp, kname, cname, val in cur.fetchall():
            if any(_short(kname).startswith(k) for k in names):
                per.setdefault((disp, _short(kname)), {})[cname] = val
        ctrs = sorted({c for v in per.values() for c in v})
        lines.append("| dispatch | kernel | " + " | ".join(ctrs) + " |")
        lines.append("|---|---|" + "---|" * len(ctrs))
        for (disp, kname), v in sorted(per.items()):
            lines.append(f"| {disp} | {kname} | " + " | ".join(f"{v.get(c, 0):.4g}" for c in ctrs) + " |")
    out = {}
    if args.fetch and args.write:
        copy_kib = args.copy_mb * 1024.0
        scale = {}
        per_kernel = {}
        names = args.kernel.split(",")
        heads = args.launch_kernels.split(",") if args.launch_kernels else names[:1]
        for ctr, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
            rows = _counter_rows(path, ctr)
            copies = [v for n, v in rows if "copyBuffer" in n or "copy" in _short(n).lower()]
            big = max(copies) if copies else 0.0
            scale[ctr] = copy_kib / big if big > 0 else None
            # the launches of the kernels that start a round, each with the
            # other kernels of its round; from launch --from-launch on
            groups = []
            for n, v in rows:
                sn = _short(n)
                if any(sn.startswith(k) for k in heads):
                    groups.append(v)
                elif any(sn.startswith(k) for k in names) and groups:
                    groups[-1] += v
            groups = groups[args.from_launch:]
            per_kernel[ctr] = (sum(groups), len(groups))
        f_kib, nf = per_kernel["FETCH_SIZE"]
        w_kib, nw = per_kernel["WRITE_SIZE"]
        fetch_b = f_kib * 1024 * scale["FETCH_SIZE"] / max(nf, 1)
        write_b = w_kib * 1024 * scale["WRITE_SIZE"] / max(nw, 1)
        out = {"kernel": args.kernel, "launches": nf, "copy_mib": args.copy_mb,
               "fetch_scale": scale["FETCH_SIZE"], "write_scale": scale["WRITE_SIZE"],
               "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
               "bytes_per_launch": round(fetch_b + write_b)}
        if args.kernel_sha:
            out["kernel_sha"] = args.kernel_sha
        # per launch of the first kernel name (one per round), the kernels of
        # that round added: KiB as read, in order
        per_round = {}
        for ctr, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
            seq = []
            for n, v in _counter_rows(path, ctr):
                sn = _short(n)
                if any(sn.startswith(k) for k in heads):
                    seq.append(v)
                elif any(sn.startswith(k) for k in names) and seq:
                    seq[-1] += v
            per_round[ctr] = seq
        nr = min(len(per_round["FETCH_SIZE"]), len(per_round["WRITE_SIZE"]))
        if nr:
            lines.append("")
            lines.append("| launch | FETCH_SIZE KiB | WRITE_SIZE KiB |")
            lines.append("|---|---|---|")
            for i in range(nr):
                lines.append(f"| {i} | {per_round['FETCH_SIZE'][i]:.1f} | {per_round['WRITE_SIZE'][i]:.1f} |")
        lines.append("")
        lines.append(f"HBM traffic of {args.kernel} per launch (FETCH_SIZE x {scale['FETCH_SIZE']:.3f}, "
                     f"WRITE_SIZE x {scale['WRITE_SIZE']:.3f}, factors from a {args.copy_mb} MiB copy): "
                     f"read {fetch_b / 1e6:.2f} MB, written {write_b / 1e6:.2f} MB over {nf} launches")
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as fh:
            if args.header:
                fh.write(args.header.replace("\\n", "\n") + "\n\n")
            fh.write(text)
    else:
        print(text)
    if args.json_out and out:
        with open(args.json_out, "w") as fh:
            json.dump(out, fh, indent=1)
    return out


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        sp = argparse.ArgumentParser()
        sp.add_argument("cmd")
        sp.add_argument("--trace")
        sp.add_argument("--stats-csv", help="rocprofv3 --stats kernel summary (run_kernel_stats.csv)")
        sp.add_argument("--counters", help="a rocprofv3 --pmc results database: every counter per dispatch")
        sp.add_argument("--fetch")
        sp.add_argument("--write")
        sp.add_argument("--kernel", default="k_round",
                        help="kernel name prefixes, comma-separated; bytes are summed and "
                             "divided by the launches of the first (or of --launch-kernels)")
        sp.add_argument("--launch-kernels", default="",
                        help="kernel name prefixes whose dispatches each start a round")
        sp.add_argument("--from-launch", type=int, default=0,
                        help="count the rounds from this launch on (skip a first call)")
        sp.add_argument("--copy-mb", type=int, default=256)
        sp.add_argument("--kernel-sha", default="")
        sp.add_argument("--out")
        sp.add_argument("--json-out")
        sp.add_argument("--header", default="")
        summarize(sp.parse_args())
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="square_16m",
                    help="a single-hull workload (2D or 3D), or batched_disks (one batched call per step)")
    ap.add_argument("--mode", type=int, default=1, help="0 exact int64, 1 FP32 filter")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--copy-mb", type=int, default=0, help="also run one device copy of this size")
    args = ap.parse_args()

    import torch

    import workloads
    from paper_1201_2936_amd import qh

    qh.load()
    if args.workload == "batched_disks":
        pts_np, off_np = workloads.batched_disks()
        off = torch.from_numpy(off_np).cuda()
    else:
        pts_np, off = workloads.WORKLOADS[args.workload](), None
    pts = torch.from_numpy(pts_np).cuda()
    ctx = qh.Context()
    if args.copy_mb:
        n = args.copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy of {args.copy_mb} MiB done", flush=True)
    dims = pts.shape[0]
    for i in range(args.steps):
        if dims == 3:
            _, idx, st = qh.qh_hull3d(pts, mode=args.mode, ctx=ctx)
        elif off is None:
            idx, st = qh.qh_hull2d(pts, mode=args.mode, ctx=ctx)
        else:
            idx, _, st = qh.qh_hull2d_batched(pts, off, mode=args.mode, ctx=ctx)
        torch.cuda.synchronize()
        print(f"hull {i}: h={idx.numel()} rounds={st['rounds']} "
              f"round_kernel_bytes={st['round_kernel_bytes']} launches={st['round_launches']} "
              f"host_syncs={st['host_syncs']}", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
