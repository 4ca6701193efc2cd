#!/usr/bin/env python3
"""Summarise rocprofv3 CSV output of the fused gate kernel into the short
text files kept under profiles/ (the benchmark reads two of them back).

Usage:
  python profile_summary.py stats <kernel_stats.csv> <command> [<kernel_trace.csv> <last_n> [<kernel>]] > profiles/X.txt
  python profile_summary.py traffic <fetch_dir> <write_dir> <copy_fetch_dir> <copy_write_dir> <copy_bytes> \\
         <last_n_dispatches> <command> [<kernel>] > profiles/Y.txt
  python profile_summary.py counters <command> <kernel> <name>=<dir> [<name>=<dir> ...] > profiles/Z.txt

<kernel> picks the dispatches by name: "plain" (job_kernel<16, 2, 0, 0, true, 0, false>: one gate per pass,
the default), "entropy" (the same with the entropy stage), "run" (job_kernel<16, 2, 0, 0, true, 3, false>: a
fused run of single-chunk gates), "group" (group_kernel<16, 3>: a chunk-group run over eight chunks) or
"group4" (group_kernel<16, 2>: over four chunks).  The traffic summary scales the per-dispatch FETCH_SIZE /
WRITE_SIZE of the kernel by the bytes per counter unit that the same counters read for a plain device copy;
every summary records the hash of the device code it was taken with.
"""
from __future__ import annotations

import csv
import glob
import os
import statistics
import sys

from paper_1911_04034_amd.profile_summary import kernel_hash

KERNELS = {"plain": "job_kernel<16, 2, 0, 0, true, 0, false>", "entropy": "job_kernel<16, 2, 0, 0, true, 0, true>",
           "run": "job_kernel<16, 2, 0, 0, true, 3, false>", "group": "group_kernel<16, 3>", "group4": "group_kernel<16, 2>"}


def _counter_rows(d):
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    return rows


def per_dispatch(d, counter, name_part, last=0):
    """Mean over dispatches of `counter` (summed over its dimensions) for kernels matching name_part;
    with last > 0 only the last `last` dispatches count."""
    acc = {}
    for r in _counter_rows(d):
        if r["Counter_Name"] != counter or name_part not in r["Kernel_Name"]:
            continue
        key = int(r["Dispatch_Id"])
        acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    vals = [acc[k] for k in sorted(acc)]
    if last > 0:
        vals = vals[-last:]
    return (statistics.mean(vals) if vals else float("nan")), len(vals)


def stats(path, command, trace=None, last=0, kernel="plain"):
    rows = list(csv.DictReader(open(path)))
    if trace:
        tr = [r for r in csv.DictReader(open(trace)) if KERNELS[kernel] in r["Kernel_Name"]]
        tr.sort(key=lambda r: int(r["Start_Timestamp"]))
        d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in tr][-int(last):]
        print("# %s, last %d dispatches (the timed region): mean %.1f ns" % (KERNELS[kernel], len(d),
                                                                          statistics.mean(d)))
    print("# rocprofv3 --kernel-trace --stats summary")
    print("# command: %s" % command)
    print("# kernel source sha256[:16]: %s" % kernel_hash())
    print("%-70s %8s %14s %12s %8s" % ("kernel", "calls", "total_ns", "avg_ns", "pct"))
    for r in rows[:15]:
        print("%-70s %8s %14s %12.1f %8.2f" % (r["Name"][:70], r["Calls"], r["TotalDurationNs"],
                                              float(r["AverageNs"]), float(r["Percentage"])))


def traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, last, command, kernel="plain"):
    copy_bytes = float(copy_bytes)
    last = int(last)
    name = KERNELS[kernel]
    cf, _ = per_dispatch(cfetch_dir, "FETCH_SIZE", "copyBuffer")
    cw, _ = per_dispatch(cwrite_dir, "WRITE_SIZE", "copyBuffer")
    f, nf = per_dispatch(fetch_dir, "FETCH_SIZE", name, last)
    w, nw = per_dispatch(write_dir, "WRITE_SIZE", name, last)
    kf = copy_bytes / cf if cf else float("nan")
    kw = copy_bytes / cw if cw else float("nan")
    print("# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, fused gate kernel %s" % name)
    print("# command: %s" % command)
    print("kernel_source_sha256_16: %s" % kernel_hash())
    print("copy_bytes: %d" % copy_bytes)
    print("copy_fetch_counter: %.4f" % cf)
    print("copy_write_counter: %.4f" % cw)
    print("fetch_scale_bytes_per_unit: %.4f" % kf)
    print("write_scale_bytes_per_unit: %.4f" % kw)
    print("dispatches_fetch: %d" % nf)
    print("dispatches_write: %d" % nw)
    print("fetch_counter_per_dispatch: %.4f" % f)
    print("write_counter_per_dispatch: %.4f" % w)
    print("traffic_bytes_per_dispatch: %.1f" % (f * kf + w * kw))


SQ = ["SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VALU", "SQ_WAIT_ANY",
      "SQ_WAVES", "SQ_WAVE_CYCLES"]


WAVES_PER_SIMD = {"group": 2, "group4": 2}   # resident waves per SIMD (eight waves per CU); others three


def counters(command, kernel, *runs):
    """Mean per dispatch of the SQ counters of the fused kernel, one block per
    `name=dir` run, with the ratios derived from them."""
    name = KERNELS[kernel]
    waves_per_simd = WAVES_PER_SIMD.get(kernel, 3)
    print("# rocprofv3 SQ counters of the fused gate kernel %s (mean per dispatch)" % name)
    print("# command: %s" % command)
    print("# %d waves per SIMD: VALU busy per SIMD = %d * SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES" % (waves_per_simd,
                                                                                               waves_per_simd))
    print("# kernel source sha256[:16]: %s" % kernel_hash())
    for run in runs:
        wl, d = run.split("=", 1)
        v, n = {}, 0
        for c in SQ:
            v[c], n = per_dispatch(d, c, name)
        print()
        print("workload %s (%d dispatches)" % (wl, n))
        for c in SQ:
            print("  %-22s %.4g" % (c, v[c]))
        print("  %-22s %.3f" % ("VALU busy per SIMD", waves_per_simd * v["SQ_ACTIVE_INST_VALU"] / v["SQ_WAVE_CYCLES"]))
        print("  %-22s %.3f" % ("waiting / wave cycles", v["SQ_WAIT_ANY"] / v["SQ_WAVE_CYCLES"]))
        print("  %-22s %.0f" % ("VALU instructions/wave", v["SQ_INSTS_VALU"] / v["SQ_WAVES"]))
        print("  %-22s %.3f" % ("SALU / VALU", v["SQ_INSTS_SALU"] / v["SQ_INSTS_VALU"]))
        print("  %-22s %.3f" % ("LDS / VALU", v["SQ_INSTS_LDS"] / v["SQ_INSTS_VALU"]))


if __name__ == "__main__":
    if len(sys.argv) < 2:
        raise SystemExit(__doc__)
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], *sys.argv[4:8])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], *sys.argv[4:])
    else:
        raise SystemExit(__doc__)
