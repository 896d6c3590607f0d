"""Summarise a rocprofv3 output directory as a short markdown table.

Reads the kernel-statistics CSV (``--kernel-trace --stats --output-format
csv``) or the counter-collection CSV (``--pmc ... --output-format csv``) that
rocprofv3 wrote under a directory and prints per-kernel averages.

    python -m paper_2302_03317_amd.profile_summary <rocprof-dir> [--title T] [--command C]
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
import sys
from collections import defaultdict


def short_name(name: str) -> str:
    m = re.search(r"(k_[a-z_]+)(<[^>(]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0][:60]


def kernel_stats(d: str):
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        return None
    rows = []
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            rows.append(r)
    return rows


def counters(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        return None
    agg = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            k = short_name(r["Kernel_Name"])
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k].add(r["Dispatch_Id"])
    return agg, disp


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    print(f"# {a.title}\n")
    if a.command:
        print(f"Command: `{a.command}`\n")
    ks = kernel_stats(a.dir)
    if ks:
        print("| kernel | calls | total ms | average us | share % |")
        print("|---|---|---|---|---|")
        for r in ks:
            print(f"| {short_name(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                  f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    cc = counters(a.dir)
    if cc:
        agg, disp = cc
        names = sorted({c for v in agg.values() for c in v})
        print("| kernel | dispatches | " + " | ".join(f"{n} per dispatch" for n in names) + " |")
        print("|---|---|" + "---|" * len(names))
        for k, v in agg.items():
            nd = len(disp[k])
            print(f"| {k} | {nd} | " + " | ".join(f"{v.get(n, 0) / nd:.4g}" for n in names) + " |")
    if not ks and not cc:
        print("no rocprofv3 CSV output found", file=sys.stderr)
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
