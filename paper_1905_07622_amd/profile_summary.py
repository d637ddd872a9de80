"""Summarise rocprofv3 CSV output of a benchmark run into a short text file.

Two kinds of input:
  * a --kernel-trace --stats directory  -> per-kernel calls / average / share
  * --pmc FETCH_SIZE and --pmc WRITE_SIZE directories of the same workload,
    plus the same counters for a plain copy of known size (bench.py
    --copy-calibration) -> per-dispatch HBM traffic of each kernel, scaled by
    (copy bytes / copy counter bytes) for each counter.

The traffic of the dominant kernel is also written as JSON together with a
hash of the kernel sources, so that the benchmark reports it only while the
kernels are unchanged.

Usage:
  python -m paper_1905_07622_amd.profile_summary stats DIR OUT.txt --command "..."
  python -m paper_1905_07622_amd.profile_summary traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR \
        OUT.txt OUT.json --kernel-regex REGEX --command "..." [--command ...]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 32 * 1024 * 1024 * 8  # bench.py --copy-calibration copies 256 MiB


# Host-only sources: argument checking, the server and the tile cache.  They
# decide nothing about what a kernel moves (the launch shapes come from
# solver.hip and engine.hip), so editing them keeps a recorded traffic valid.
HOST_ONLY = {"capi.cpp", "server.cpp", "server.hpp", "tune_cache.cpp"}


def kernel_source_hash() -> str:
    """Hash of the sources that define the kernels and their launch shapes."""
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(PKG, "csrc", "*"))):
        if os.path.basename(path) in HOST_ONLY:
            continue
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode())
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    n = name.split("(")[0].replace("void ", "").replace("femheat::", "")
    return n


def find_csv(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def working_durations(d: str):
    """Per kernel: durations (ns) of the dispatches that did work -- at least
    half the kernel's median duration.  Iteration kernels launched after their
    solve finished exit at once; the benchmark's sampled timing skips them."""
    try:
        rows = list(csv.DictReader(open(find_csv(d, "kernel_trace.csv"))))
    except FileNotFoundError:
        return {}
    acc = defaultdict(list)
    for r in rows:
        acc[short_name(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = {}
    for k, v in acc.items():
        med = sorted(v)[len(v) // 2]
        out[k] = [x for x in v if x >= 0.5 * med]
    return out


def dispatch_gaps(d: str):
    """Idle time of the device between consecutive dispatches (any stream, in
    start order; overlapping dispatches count no gap): gaps under 50 us are
    the launch-to-launch cost inside a run, longer ones host phases (set-up,
    a host round trip, the end of the program)."""
    try:
        rows = list(csv.DictReader(open(find_csv(d, "kernel_trace.csv"))))
    except FileNotFoundError:
        return None
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows)
    gaps, end = [], None
    for s0, e0 in iv:
        if end is not None:
            gaps.append(max(0, s0 - end) / 1e3)
        end = e0 if end is None else max(end, e0)
    if not gaps:
        return None
    short = sorted(g for g in gaps if g < 50.0)
    return {"dispatches": len(iv), "short_gaps": len(short),
            "short_gap_median_us": short[len(short) // 2] if short else 0.0,
            "short_gap_mean_us": sum(short) / len(short) if short else 0.0,
            "short_gap_total_ms": sum(short) / 1e3,
            "busy_ms": sum(e0 - s0 for s0, e0 in iv) / 1e6}


def stats(d: str, out: str, commands):
    rows = list(csv.DictReader(open(find_csv(d, "kernel_stats.csv"))))
    work = working_durations(d)
    lines = ["# rocprofv3 kernel statistics", ""]
    lines += [f"command: {c}" for c in commands]
    lines += ["", "working: dispatches lasting at least half the kernel's median (iteration kernels launched",
              "after their solve finished exit at once and are left out, as the benchmark's timing does)", "",
              f"{'kernel':70s} {'calls':>7s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'share%':>7s} "
              f"{'working':>8s} {'work_avg_us':>11s}"]
    for r in rows:
        name = short_name(r["Name"])
        w = work.get(name, [])
        wa = f"{sum(w) / len(w) / 1e3:11.3f}" if w else f"{'-':>11s}"
        lines.append(f"{name[:70]:70s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.3f} "
                     f"{float(r['MinNs']) / 1e3:8.3f} {float(r['MaxNs']) / 1e3:8.3f} {float(r['Percentage']):7.2f} "
                     f"{len(w):8d} {wa}")
    g = dispatch_gaps(d)
    if g:
        lines += ["", f"dispatch gaps (device idle between consecutive dispatches, {g['dispatches']} dispatches): "
                      f"{g['short_gaps']} gaps under 50 us, median {g['short_gap_median_us']:.2f} us, "
                      f"mean {g['short_gap_mean_us']:.2f} us, total {g['short_gap_total_ms']:.2f} ms "
                      f"against {g['busy_ms']:.1f} ms of dispatches"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counter_means(d: str, working: float = 0.0):
    """Mean counter value per (kernel, counter) over its dispatches.  With
    working > 0, dispatches below that fraction of the kernel's largest value
    are left out: iteration kernels launched after their solve finished (a
    chunk runs a few iterations past the end) exit at once and move almost
    nothing, and the timing the traffic is compared with skips them too."""
    rows = list(csv.DictReader(open(find_csv(d, "counter_collection.csv"))))
    acc = defaultdict(list)
    for r in rows:
        acc[(short_name(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    out = {}
    for k, v in acc.items():
        if working > 0 and v:
            top = max(v)
            v = [x for x in v if x >= working * top] or v
        out[k] = (sum(v) / len(v), len(v))
    return out


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, out_txt, out_json, kernel_regex, commands,
            algorithmic_bytes=None):
    fetch = counter_means(fetch_dir, working=0.25)
    write = counter_means(write_dir, working=0.25)
    cf = [v for (k, c), v in counter_means(copy_fetch_dir).items() if "copy" in k.lower() and c == "FETCH_SIZE"]
    cw = [v for (k, c), v in counter_means(copy_write_dir).items() if "copy" in k.lower() and c == "WRITE_SIZE"]
    # the copy kernel with the largest count is the 256 MiB calibration copy
    fscale = COPY_BYTES / (max(x[0] for x in cf) * 1024.0)
    wscale = COPY_BYTES / (max(x[0] for x in cw) * 1024.0)
    lines = ["# HBM traffic per dispatch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB), scaled by a plain copy",
             "# (means over working dispatches: those moving at least 25% of the kernel's largest dispatch)", ""]
    lines += [f"command: {c}" for c in commands]
    lines += ["", f"copy calibration: {COPY_BYTES} bytes copied; FETCH_SIZE scale {fscale:.4f}, "
                  f"WRITE_SIZE scale {wscale:.4f}", "",
              f"{'kernel':80s} {'fetch_KiB':>11s} {'write_KiB':>11s} {'traffic_MB':>11s} {'dispatches':>10s}"]
    chosen = None
    for (k, c), (v, n) in sorted(fetch.items()):
        if c != "FETCH_SIZE":
            continue
        wv = write.get((k, "WRITE_SIZE"), (0.0, 0))[0]
        t = v * 1024 * fscale + wv * 1024 * wscale
        lines.append(f"{k[:80]:80s} {v:11.1f} {wv:11.1f} {t / 1e6:11.2f} {n:10d}")
        if re.search(kernel_regex, k) and (chosen is None or n > chosen[3]):
            chosen = (k, v, wv, n, t)
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    if chosen and out_json:
        k, v, wv, n, t = chosen
        rec = {"kernel": k, "fetch_kib": v, "write_kib": wv, "fetch_scale": fscale, "write_scale": wscale,
               "traffic_bytes": t, "dispatches": n, "source_sha256": kernel_source_hash()}
        if algorithmic_bytes:
            rec["algorithmic_bytes"] = algorithmic_bytes
        with open(out_json, "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote", out_json)


def counters(dirs, out, kernel_regex, commands):
    """Means of the SQ counters of one kernel over its working dispatches (per pass: those whose first
    present reference counter, SQ_WAVE_CYCLES or SQ_INSTS_VALU, is at least 25% of its largest value),
    with the ratios of same-unit counters: wait shares of the wave cycles, LDS bank-conflict share of the
    LDS-active cycles, and instructions per wave."""
    means = {}
    for d in dirs:
        rows = list(csv.DictReader(open(find_csv(d, "counter_collection.csv"))))
        disp = defaultdict(dict)
        for r in rows:
            k = short_name(r["Kernel_Name"])
            if re.search(kernel_regex, k):
                disp[r.get("Dispatch_Id") or r["Correlation_Id"]][r["Counter_Name"]] = float(r["Counter_Value"])
        if not disp:
            continue
        ref = next((c for c in ("SQ_WAVE_CYCLES", "SQ_INSTS_VALU") if c in next(iter(disp.values()))), None)
        vals = list(disp.values())
        if ref:
            top = max(v.get(ref, 0.0) for v in vals)
            vals = [v for v in vals if v.get(ref, 0.0) >= 0.25 * top] or vals
        for c in vals[0]:
            means[c] = (sum(v.get(c, 0.0) for v in vals) / len(vals), len(vals))
    lines = [f"# rocprofv3 SQ counters of {kernel_regex!r}: means over working dispatches", ""]
    lines += [f"command: {c}" for c in commands]
    lines += ["", f"{'counter':28s} {'mean':>16s} {'dispatches':>10s}"]
    lines += [f"{c:28s} {v:16.1f} {n:10d}" for c, (v, n) in sorted(means.items())]

    def m(c):
        return means.get(c, (None, 0))[0]

    ratios = [("wait (any) / wave cycles", "SQ_WAIT_ANY", "SQ_WAVE_CYCLES"),
              ("wait (instruction) / wave cycles", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES"),
              ("wait (LDS) / wave cycles", "SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES"),
              ("LDS bank conflict / LDS active", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS"),
              ("VALU instructions / wave", "SQ_INSTS_VALU", "SQ_WAVES"),
              ("vector-memory reads / wave", "SQ_INSTS_VMEM_RD", "SQ_WAVES"),
              ("vector-memory writes / wave", "SQ_INSTS_VMEM_WR", "SQ_WAVES"),
              ("LDS instructions / wave", "SQ_INSTS_LDS", "SQ_WAVES")]
    lines += [""]
    for label, a, b in ratios:
        if m(a) is not None and m(b):
            lines.append(f"{label:36s} {m(a) / m(b):10.3f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("out")
    a.add_argument("--command", action="append", default=[])
    b = sub.add_parser("traffic")
    for n in ("fetch_dir", "write_dir", "copy_fetch_dir", "copy_write_dir", "out_txt", "out_json"):
        b.add_argument(n)
    b.add_argument("--kernel-regex", required=True)
    b.add_argument("--command", action="append", default=[])
    b.add_argument("--algorithmic-bytes", type=float, default=None)
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel-regex", required=True)
    c.add_argument("--command", action="append", default=[])
    args = ap.parse_args()
    if args.cmd == "stats":
        stats(args.dir, args.out, args.command)
    elif args.cmd == "counters":
        counters(args.dirs, args.out, args.kernel_regex, args.command)
    else:
        traffic(args.fetch_dir, args.write_dir, args.copy_fetch_dir, args.copy_write_dir, args.out_txt,
                args.out_json, args.kernel_regex, args.command, args.algorithmic_bytes)


if __name__ == "__main__":
    main()
