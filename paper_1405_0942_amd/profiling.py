"""Summaries of rocprofv3 output for the stage sweeps: HBM bytes per launch from the
FETCH_SIZE / WRITE_SIZE counters, calibrated on a device copy of known size.

The two counters come from two separate `rocprofv3 --pmc` runs of the same program (one
counter each).  Each run also holds the 1 GiB device-to-device copy that bench.py makes
to measure copy bandwidth; its reading against the 1 GiB it moves gives the scale of each
counter on this device.

    python -m paper_1405_0942_amd.profiling traffic --fetch DIR --write DIR \\
        --workload abc_256 --precision fp64 --command "..." > profiles/<name>.txt

`read_traffic` parses such a summary; `kernel_source_hash` identifies the kernel source
the counters were taken on (a summary of other source is stale).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/stage.hip", "csrc/sweep_common.h", "csrc/relax_device.h", "csrc/relax.cpp")
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counter_csv(run_dir: str) -> str:
    hits = sorted(glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *counter_collection.csv under {run_dir}")
    return hits[0]


def read_counter(run_dir: str, counter: str):
    """[(dispatch_id, kernel_name, value in counter units)] of one --pmc run, dispatch order."""
    rows = []
    with open(_counter_csv(run_dir), newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def _stage_of(name: str):
    # stage_kernel<S, MIXED, XYP[, DIAG[, REC[, NNN]]]>; the diagnostics variant (DIAG true) is not a stage
    m = re.search(r"stage_kernel<(\d), (false|true), (false|true)(?:, false(?:, (?:false|true)){0,2})?>", name)
    if not m:
        return None
    return int(m.group(1)), m.group(2) == "true"


def traffic(fetch_dir: str, write_dir: str, mixed: bool):
    """Per-stage mean HBM bytes per launch, and the two calibration factors."""
    fetch = read_counter(fetch_dir, "FETCH_SIZE")
    write = read_counter(write_dir, "WRITE_SIZE")
    if [d for d, _, _ in fetch] != [d for d, _, _ in write]:
        raise ValueError("the two runs dispatched different kernels")
    kib = COPY_BYTES / 1024.0
    cal = [(f, w) for (_, n, f), (_, _, w) in zip(fetch, write)
           if "copyBuffer" in n and abs(w - kib) < 0.01 * kib]
    if not cal:
        raise ValueError("no 1 GiB device copy among the dispatches")
    f_scale = kib / (sum(f for f, _ in cal) / len(cal))
    w_scale = kib / (sum(w for _, w in cal) / len(cal))
    per = collections.defaultdict(list)
    for (_, n, f), (_, _, w) in zip(fetch, write):
        st = _stage_of(n)
        if st is None or st[1] != mixed:
            continue
        per[st[0]].append((f, w))
    out = {}
    for s, v in sorted(per.items()):
        fb = sum(f for f, _ in v) / len(v) * f_scale * 1024.0
        wb = sum(w for _, w in v) / len(v) * w_scale * 1024.0
        out[s] = {"launches": len(v), "fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb}
    return out, f_scale, w_scale


def sq_counters(run_dirs, mixed: bool):
    """{stage: {counter: median over the launches of that stage}} from `--pmc SQ_...` runs
    (the median keeps the stage-1 launches of retried attempts, which exit at once and are
    a minority, out of the figure)."""
    per = collections.defaultdict(lambda: collections.defaultdict(dict))  # stage -> dispatch -> counter
    for d in run_dirs:
        with open(_counter_csv(d), newline="") as f:
            for r in csv.DictReader(f):
                st = _stage_of(r["Kernel_Name"])
                if st is None or st[1] != mixed:
                    continue
                disp = per[st[0]][(d, int(r["Dispatch_Id"]))]
                disp[r["Counter_Name"]] = disp.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out = {}
    for s, disps in sorted(per.items()):
        cols = collections.defaultdict(list)
        for vals in disps.values():
            for c, v in vals.items():
                cols[c].append(v)
        out[s] = {c: sorted(v)[len(v) // 2] for c, v in cols.items()}
    return out


def read_traffic(path: str):
    """key: value lines of a traffic summary, or None if there is no such file."""
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^([A-Za-z0-9_]+):\s*(.*?)\s*$", line)
            if m:
                rec[m.group(1)] = m.group(2)
    return rec


def kernel_stats(run_dir: str):
    """Rows of a `rocprofv3 --kernel-trace --stats` run: (name, calls, average ns, min, max)."""
    hits = sorted(glob.glob(os.path.join(run_dir, "**", "*kernel_stats.csv"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *kernel_stats.csv under {run_dir}")
    rows = []
    with open(hits[0], newline="") as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"]),
                         float(r["Percentage"])))
    return rows


def _short(name: str) -> str:
    name = name.replace("relax::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    name = name.replace("(relax::SweepArgs)", "")
    name = re.sub(r"^void ", "", name)
    return re.sub(r"\(.*\)$", "", name) if "stage_kernel" not in name else name


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernel-stats")
    k.add_argument("--trace", required=True, help="rocprofv3 output directory of a --kernel-trace --stats run")
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True, help="the profiled command, recorded in the summary")
    k.add_argument("--top", type=int, default=12)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True, help="rocprofv3 output directory of the FETCH_SIZE run")
    t.add_argument("--write", required=True, help="rocprofv3 output directory of the WRITE_SIZE run")
    t.add_argument("--workload", required=True)
    t.add_argument("--precision", choices=["fp64", "fp32-mixed"], default="fp64")
    t.add_argument("--nodes", type=int, required=True, help="grid nodes (for bytes per node)")
    t.add_argument("--command", required=True, help="the profiled command, recorded in the summary")
    q = sub.add_parser("sq")
    q.add_argument("--run", action="append", required=True, help="rocprofv3 output directory of a --pmc run")
    q.add_argument("--workload", required=True)
    q.add_argument("--precision", choices=["fp64", "fp32-mixed"], default="fp64")
    q.add_argument("--nodes", type=int, required=True, help="grid nodes (counts are per 64 nodes)")
    q.add_argument("--command", required=True, help="the profiled commands, recorded in the summary")
    m = sub.add_parser("pipe")
    m.add_argument("--run", action="append", required=True, help="rocprofv3 output directory of a --pmc run")
    m.add_argument("--workload", required=True)
    m.add_argument("--precision", choices=["fp64", "fp32-mixed"], default="fp64")
    m.add_argument("--nodes", type=int, required=True, help="grid nodes (counts are per 64 nodes)")
    m.add_argument("--cus", type=int, default=256, help="compute units (one TA, TD and TCP each)")
    m.add_argument("--xcds", type=int, default=8, help="XCDs (GRBM_GUI_ACTIVE is their sum)")
    m.add_argument("--command", required=True, help="the profiled commands, recorded in the summary")
    args = ap.parse_args(argv)
    w = sys.stdout.write
    if args.cmd == "pipe":
        per = sq_counters(args.run, args.precision == "fp32-mixed")
        w(f"# Vector-memory pipe of the stage sweeps, {args.workload}, {args.precision}\n\n")
        w("Commands (from the repository root):\n\n")
        w(f"    {args.command}\n\n")
        w(f"Median over launches. Busy and stall columns: % of the launch's cycles (GRBM_GUI_ACTIVE / "
          f"{args.xcds} XCDs), per unit (summed counter / {args.cus} CUs). Count columns: per 64 grid "
          f"nodes (one wave's plane); SQ_WAIT_INST_LDS and SQ_ACTIVE_INST_LDS in units of 4 cycles.\n\n")
        w(f"source_sha256: {kernel_source_hash()}\n\n")
        busy = ["TA_TA_BUSY", "TD_TD_BUSY", "TCP_PENDING_STALL_CYCLES"]
        counts = ["TA_BUFFER_READ_WAVEFRONTS", "TA_BUFFER_WRITE_WAVEFRONTS", "TCP_TCC_READ_REQ",
                  "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_LDS"]
        cols = [c for c in busy + counts if any(c in v for v in per.values())]
        w("| stage | " + " | ".join(cols) + " |\n|---|" + "---:|" * len(cols) + "\n")
        batches = args.nodes / 64.0
        for s_, v in per.items():
            cyc = v.get("GRBM_GUI_ACTIVE", float("nan")) / args.xcds
            cells = []
            for c in cols:
                x = v.get(c, float("nan"))
                cells.append(f"{100.0 * x / args.cus / cyc:.0f} %" if c in busy else f"{x / batches:.1f}")
            w(f"| {s_} | " + " | ".join(cells) + " |\n")
        return
    if args.cmd == "sq":
        per = sq_counters(args.run, args.precision == "fp32-mixed")
        cols = sorted({c for v in per.values() for c in v})
        w(f"# SQ counters per launch of the stage sweeps, {args.workload}, {args.precision}\n\n")
        w("Commands (from the repository root):\n\n")
        w(f"    {args.command}\n\n")
        w(f"Median over launches; instruction counts are per 64 grid nodes (one wave's worth), "
          f"SQ_WAVES and cycle counts per launch.\n\n")
        w(f"source_sha256: {kernel_source_hash()}\n\n")
        w("| stage | " + " | ".join(cols) + " |\n|---|" + "---:|" * len(cols) + "\n")
        batches = args.nodes / 64.0
        for s_, v in per.items():
            cells = []
            for c in cols:
                x = v.get(c, float("nan"))
                cells.append(f"{x / batches:.1f}" if c.startswith("SQ_INSTS") else f"{x:.4g}")
            w(f"| {s_} | " + " | ".join(cells) + " |\n")
        return
    if args.cmd == "kernel-stats":
        w(f"# {args.title}\n\n")
        w("Command (from the repository root):\n\n")
        w(f"    {args.command}\n\n")
        w("| kernel | calls | avg ms | min ms | max ms | % of GPU time |\n|---|---:|---:|---:|---:|---:|\n")
        for name, calls, avg, mn, mx, pct in kernel_stats(args.trace)[: args.top]:
            w(f"| `{_short(name)}` | {calls} | {avg / 1e6:.4f} | {mn / 1e6:.4f} | {mx / 1e6:.4f} | {pct:.2f} |\n")
        return
    per, fs, ws = traffic(args.fetch, args.write, args.precision == "fp32-mixed")
    w(f"# HBM traffic per launch of the stage sweeps, {args.workload}, {args.precision}\n")
    w("# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE, one run each:\n")
    w(f"#   {args.command}\n")
    w("# counters scaled by their reading on the 1 GiB device copy of the same runs\n")
    w(f"source_sha256: {kernel_source_hash()}\n")
    w(f"fetch_scale: {fs:.4f}\n")
    w(f"write_scale: {ws:.4f}\n")
    for s, v in per.items():
        w(f"stage{s}_launches: {v['launches']}\n")
        w(f"stage{s}_fetch_bytes_per_launch: {v['fetch_bytes']:.0f}\n")
        w(f"stage{s}_write_bytes_per_launch: {v['write_bytes']:.0f}\n")
        w(f"stage{s}_bytes_per_launch: {v['bytes']:.0f}\n")
        w(f"stage{s}_bytes_per_node: {v['bytes'] / args.nodes:.1f}\n")


if __name__ == "__main__":
    main()
