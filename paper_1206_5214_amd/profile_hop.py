"""Profiling driver for the metered hop kernel (run under rocprofv3).

    python -m paper_1206_5214_amd.profile_hop run --prec f16 --reps 20
        builds the 24^3 x 64, Ls = 12 workload, tunes the hop for the given
        storage precision, runs `warm` untimed applications of each parity, a
        1 GiB device copy (the calibration kernel for the memory counters),
        then `reps` applications of each hop parity.

    python -m paper_1206_5214_amd.profile_hop summarize --prec f16 \\
            --rdreq DIR --wrreq DIR [--fetch DIR --write DIR] [--stats DIR] --out profiles/NAME
        reads the rocprofv3 outputs of two request-count passes (L2-to-memory
        read requests by size: TCC_EA0_RDREQ{,_32B,_64B,_128B}_sum; write
        requests: TCC_EA0_WRREQ{,_64B}_sum), turns them into bytes per launch
        by the request sizes, checks the rule on the calibration copy of known
        size, optionally adds the FETCH_SIZE / WRITE_SIZE passes scaled by the
        copy as a cross-check and a --kernel-trace --stats run for the
        duration, and writes NAME.json (the per-launch traffic bench.py
        reports, keyed to the kernel source it was measured on) and NAME.md
        (the figures and the commands that produced them).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PREC = {"f64": 0, "f32": 1, "f16": 2}
# the files the hop kernel is compiled from; their joint hash keys the counters
HOP_SOURCES = ("mobius_kernels.hip", "mobius_device.h", "mobius_internal.h")


def hop_sources_sha256() -> str:
    h = hashlib.sha256()
    for name in HOP_SOURCES:
        with open(os.path.join(ROOT, "paper_1206_5214_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()
COPY_BYTES = 1 << 30      # the calibration copy reads and writes 1 GiB
HOP_NAME = "hop_kernel"


def run(args):
    import numpy as np
    import torch
    from paper_1206_5214_amd import inputs, mobius
    w = inputs.WORKLOADS[args.workload]
    prec = PREC[args.prec]
    U, eta = inputs.workload_fields(w)
    brick = None if not args.brick else tuple(int(b) for b in args.brick.split(","))
    op = mobius.Operator(w.dims, w.Ls, w.M5, w.mf, w.b5, w.c5, torch.from_numpy(U).cuda(), brick=brick)
    tuned = op.tune(prec)
    even, odd = op.pack(torch.from_numpy(eta).cuda(), prec)
    oe, oo = op.new_field(prec), op.new_field(prec)
    for _ in range(args.warm):  # untimed: the clocks settle before the counted launches
        op.dslash(odd, 0, prec, out=oe)
        op.dslash(even, 1, prec, out=oo)
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)                       # calibration: reads and writes COPY_BYTES
    torch.cuda.synchronize()
    for _ in range(args.reps):
        op.dslash(odd, 0, prec, out=oe)
        op.dslash(even, 1, prec, out=oo)
    torch.cuda.synchronize()
    nbytes = 2 * op.field_bytes(prec) + 72 * (op.V // 2) * {0: 16, 1: 8, 2: 4}[prec]
    print(json.dumps({"workload": w.name, "prec": args.prec, "tuning": tuned,
                      "brick": None if brick is None else list(brick),
                      "algo_bytes_per_launch": nbytes, "reps": args.reps}), flush=True)


def _csv_rows(d, pattern):
    files = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not files:
        raise SystemExit(f"no {pattern} under {d}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _counter_per_kernel(d, counter):
    """Counter values (summed over the dimensions rocprofv3 splits a counter
    into) of the calibration copy and of the hop launches that follow it (the
    timed launches; the tuner's candidate launches come before the copy)."""
    rows = _csv_rows(d, "*counter_collection.csv")
    per = {}
    names = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        disp = int(r["Dispatch_Id"])
        per[disp] = per.get(disp, 0.0) + float(r["Counter_Value"])
        names[disp] = r["Kernel_Name"]
    copies = [k for k, n in names.items() if "copyBuffer" in n]
    if not copies:
        raise SystemExit(f"no calibration copy in {d}")
    c = max(copies)
    hops = [per[k] for k, n in sorted(names.items()) if k > c and HOP_NAME in n]
    return {"copy": [per[c]], HOP_NAME: hops}


def _requests(d, counters):
    """Average per hop launch, and the calibration copy's value, of each counter."""
    res = {}
    for c in counters:
        per = _counter_per_kernel(d, c)
        hop = per[HOP_NAME]
        res[c] = {"hop": sum(hop) / len(hop), "copy": max(per["copy"]), "launches": len(hop)}
    return res


RD = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")
WR = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum")


def _read_bytes(r, which):
    n32, n64, n128 = (r[c][which] for c in RD[1:])
    other = max(r[RD[0]][which] - n32 - n64 - n128, 0.0)  # none expected; counted as 64 B
    return 32 * n32 + 64 * (n64 + other) + 128 * n128, other


def _write_bytes(w, which):
    n, n64 = w[WR[0]][which], w[WR[1]][which]
    return 64 * n64 + 32 * (n - n64)


def summarize(args):
    sha = hop_sources_sha256()
    out = {"kernel": f"{HOP_NAME} ({args.prec}, D_{{p,1-p}} = -1/2 H B, 24^3x64 Ls=12)",
           "kernel_source_sha256": sha, "kernel_sources": list(HOP_SOURCES),
           "calibration_copy_bytes": COPY_BYTES}
    r = _requests(args.rdreq, RD)
    w = _requests(args.wrreq, WR)
    rb, other = _read_bytes(r, "hop")
    wb = _write_bytes(w, "hop")
    crb, _ = _read_bytes(r, "copy")
    cwb = _write_bytes(w, "copy")
    out["requests"] = {"read": {c: r[c]["hop"] for c in RD}, "write": {c: w[c]["hop"] for c in WR},
                       "read_bytes": rb, "write_bytes": wb, "unsized_read_requests": other,
                       "launches": r[RD[0]]["launches"],
                       "copy_check": {"read_bytes": crb, "write_bytes": cwb,
                                      "read_over_true": crb / COPY_BYTES, "write_over_true": cwb / COPY_BYTES}}
    out["traffic_bytes_per_launch"] = rb + wb
    if args.run_log:  # the launch parameters the counted launches ran with
        with open(args.run_log) as f:
            for line in f:
                if line.startswith("{") and '"tuning"' in line:
                    rec = json.loads(line)
                    out["tuning"] = {k: v for k, v in rec["tuning"].items() if k != "hop_us"}
                    # site-order brick of the run (None: the library's automatic choice)
                    out["brick"] = rec.get("brick")
    traffic = {}
    if args.fetch and args.write:  # cross-check: FETCH_SIZE / WRITE_SIZE scaled by the copy
        for counter, d in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
            per = _counter_per_kernel(d, counter)
            copy = max(per["copy"])               # KiB the counter reports for the 1 GiB copy
            scale = COPY_BYTES / (copy * 1024.0)  # true bytes per reported byte
            hop = per[HOP_NAME]
            avg_kib = sum(hop) / len(hop)
            traffic[counter] = {"raw_kib_per_launch": avg_kib, "copy_raw_kib": copy,
                                "scale": scale, "bytes_per_launch": avg_kib * 1024.0 * scale,
                                "launches": len(hop)}
        out["counters"] = traffic
        out["fetch_write_bytes_per_launch"] = (traffic["FETCH_SIZE"]["bytes_per_launch"] +
                                               traffic["WRITE_SIZE"]["bytes_per_launch"])
    if args.algo_bytes:
        out["algo_bytes_per_launch"] = args.algo_bytes
        out["traffic_over_algo"] = out["traffic_bytes_per_launch"] / args.algo_bytes
    stats = None
    if args.stats:  # durations of the timed launches (after the calibration copy)
        rows = _csv_rows(args.stats, "*kernel_trace.csv")
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        c = max(int(r["Dispatch_Id"]) for r in rows if "copyBuffer" in r["Kernel_Name"])
        durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows
                if int(r["Dispatch_Id"]) > c and HOP_NAME in r["Kernel_Name"]]
        name = next(r["Kernel_Name"] for r in rows
                    if int(r["Dispatch_Id"]) > c and HOP_NAME in r["Kernel_Name"])
        stats = {"kernel": name.split("(mobius::HopParams")[0].replace("mobius::(anonymous namespace)::", ""),
                 "launches": len(durs), "avg_us": sum(durs) / len(durs)}
        out["hop_trace"] = stats
        if args.algo_bytes:
            out["achieved_GBps"] = args.algo_bytes / (stats["avg_us"] * 1e-6) / 1e9
            out["traffic_GBps"] = out["traffic_bytes_per_launch"] / (stats["avg_us"] * 1e-6) / 1e9
    with open(args.out + ".json", "w") as f:
        json.dump(out, f, indent=1)
    lines = [f"# HBM traffic of the hop kernel, {args.prec}, 24^3x64 Ls=12", ""]
    lines += ["Commands (repository root, one MI355X, `export TMPDIR=/tmp`):", "", "```"]
    lines += args.command or []
    lines += ["```", ""]
    lines += ["L2-to-memory requests per launch, by size (bytes = 32, 64 or 128 per request;",
              "writes: 64 for the 64-byte ones, 32 for the rest; the Infinity Cache sits behind",
              "these requests, so the figure bounds the HBM bytes from above):", "",
              "| counter | requests / launch | calibration copy (1 GiB) |", "|---|---:|---:|"]
    for c in RD:
        lines.append(f"| {c} | {r[c]['hop']:.0f} | {r[c]['copy']:.0f} |")
    for c in WR:
        lines.append(f"| {c} | {w[c]['hop']:.0f} | {w[c]['copy']:.0f} |")
    lines.append("")
    lines.append(f"Read {rb / 1e6:.1f} MB + write {wb / 1e6:.1f} MB per launch; the same rule gives "
                 f"{crb / 2**30:.3f} GiB read and {cwb / 2**30:.3f} GiB written for the 1 GiB copy.")
    if traffic:
        lines += ["", "Cross-check, FETCH_SIZE / WRITE_SIZE scaled by their reading for the copy:", "",
                  "| counter | raw KiB / launch | copy raw KiB (1 GiB) | scale | bytes / launch |",
                  "|---|---:|---:|---:|---:|"]
        for c, t in traffic.items():
            lines.append(f"| {c} | {t['raw_kib_per_launch']:.0f} | {t['copy_raw_kib']:.0f} | "
                         f"{t['scale']:.3f} | {t['bytes_per_launch'] / 1e6:.1f} MB |")
    lines.append("")
    lines.append(f"Traffic per launch: {out['traffic_bytes_per_launch'] / 1e6:.1f} MB"
                 + (f" against {args.algo_bytes / 1e6:.1f} MB algorithmic "
                    f"({out['traffic_over_algo']:.2f}x)" if args.algo_bytes else ""))
    if stats:
        lines.append("")
        lines.append(f"- `{stats['kernel']}`: {stats['launches']} timed launches, average "
                     f"{stats['avg_us']:.1f} us (kernel-trace run)")
        if args.algo_bytes:
            lines.append(f"- algorithmic {out['achieved_GBps']:.0f} GB/s "
                         f"({100 * out['achieved_GBps'] / 8000:.1f}% of 8 TB/s); counted traffic "
                         f"{out['traffic_GBps']:.0f} GB/s")
    lines.append("")
    lines.append(f"Kernel sources ({', '.join(HOP_SOURCES)}) sha256: `{sha}`")
    with open(args.out + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(out, indent=1))


SQ_PASSES = (("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY",
              "SQ_ACTIVE_INST_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_VALU"),
             ("SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_SALU", "SQ_ACTIVE_INST_LDS",
              "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_VMEM_WR", "TCC_HIT_sum", "TCC_MISS_sum"))


def sq_md(args):
    """Per-launch shader-sequencer counters of the metered hop (two --pmc
    passes of `run`) as per-wave instruction counts and cycle ratios."""
    v = {}
    for d, counters in zip(args.passes, SQ_PASSES):
        for c in counters:
            hop = _counter_per_kernel(d, c)[HOP_NAME]
            v[c] = sum(hop) / len(hop)
    waves = v["SQ_WAVES"]
    lines = [f"# Shader-sequencer counters of the hop kernel, {args.prec}, 24^3x64 Ls=12", "",
             "Commands (repository root, one MI355X, `export TMPDIR=/tmp`):", "", "```"]
    lines += (args.command or []) + ["```", "",
              "| counter | per launch | per wave |", "|---|---:|---:|"]
    for c in SQ_PASSES[0] + SQ_PASSES[1]:
        lines.append(f"| {c} | {v[c]:.4g} | {v[c] / waves:.4g} |")
    hit = v["TCC_HIT_sum"] / (v["TCC_HIT_sum"] + v["TCC_MISS_sum"])
    lines += ["", "Ratios (the SQ cycle counters share one unit, so their ratios are exact):", "",
              f"- waiting on a dependency (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES): "
              f"{v['SQ_WAIT_INST_ANY'] / v['SQ_WAVE_CYCLES']:.3f} of the waves' lifetime",
              f"- waiting on anything (SQ_WAIT_ANY / SQ_WAVE_CYCLES): {v['SQ_WAIT_ANY'] / v['SQ_WAVE_CYCLES']:.3f}",
              f"- issuing VALU (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES): "
              f"{v['SQ_ACTIVE_INST_VALU'] / v['SQ_WAVE_CYCLES']:.3f}",
              f"- LDS bank conflicts per active LDS cycle: "
              f"{v['SQ_LDS_BANK_CONFLICT'] / max(v['SQ_ACTIVE_INST_LDS'], 1):.3f}",
              f"- L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)): {hit:.3f}",
              f"- {waves:.0f} waves per launch"]
    with open(args.out, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def stats_md(args):
    """Markdown table of a rocprofv3 --kernel-trace --stats run."""
    rows = _csv_rows(args.stats, "*kernel_stats.csv")
    lines = [f"# {args.title}", "", "Command (repository root, one MI355X, `export TMPDIR=/tmp`):",
             "", "```"] + (args.command or []) + ["```", "",
             "| kernel | calls | avg (us) | total (ms) | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:args.top]:
        name = r["Name"].replace("mobius::(anonymous namespace)::", "").replace("mobius::", "")
        name = name.split("(")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.1f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--prec", default="f16", choices=list(PREC))
    r.add_argument("--reps", type=int, default=20)
    r.add_argument("--warm", type=int, default=50, help="untimed launches per parity before the copy")
    r.add_argument("--workload", default="mobius_24x24x24x64_ls12")
    r.add_argument("--brick", default="", help="site-order brick bx,by,bz (default: automatic)")
    s = sub.add_parser("summarize")
    s.add_argument("--prec", default="f16", choices=list(PREC))
    s.add_argument("--rdreq", required=True)
    s.add_argument("--wrreq", required=True)
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--stats")
    s.add_argument("--run-log", help="stdout of a `run` pass (its tuning line)")
    s.add_argument("--algo-bytes", type=float)
    s.add_argument("--out", required=True)
    s.add_argument("--command", action="append")
    t = sub.add_parser("stats")
    t.add_argument("--stats", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--top", type=int, default=20)
    t.add_argument("--command", action="append")
    q = sub.add_parser("sq")
    q.add_argument("--prec", default="f16", choices=list(PREC))
    q.add_argument("--passes", nargs=2, required=True, help="the two --pmc run directories")
    q.add_argument("--out", required=True)
    q.add_argument("--command", action="append")
    args = ap.parse_args()
    {"run": run, "summarize": summarize, "stats": stats_md, "sq": sq_md}[args.cmd](args)


if __name__ == "__main__":
    main()
