"""Summarise a rocprofv3 output directory as a short markdown table.

Reads the kernel-statistics CSV (``--kernel-trace --stats --output-format
csv``) or the counter-collection CSV (``--pmc ... --output-format csv``) that
rocprofv3 wrote under a directory and prints per-kernel averages.

    python -m paper_2302_03317_amd.profile_summary <rocprof-dir> [--title T] [--command C]
    python -m paper_2302_03317_amd.profile_summary --traffic <fetch-dir> <write-dir> --copy-bytes B

The --traffic form reads two counter runs (FETCH_SIZE, then WRITE_SIZE, in
KiB per dispatch), takes the plain copy of B bytes in the same runs (the
copy dispatch whose WRITE_SIZE is nearest B) as the calibration, scales each
counter by bytes / counter-reading of that copy, and prints the HBM bytes
per dispatch of every kernel.
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


def per_dispatch(d: str):
    """(dispatch id, kernel short name) -> summed counter value, per counter name."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter CSV under {d}")
    out = defaultdict(lambda: defaultdict(float))
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            out[r["Counter_Name"]][(int(r["Dispatch_Id"]), short_name(r["Kernel_Name"]))] += float(r["Counter_Value"])
    return out


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int) -> int:
    fd = per_dispatch(fetch_dir)["FETCH_SIZE"]
    wd = per_dispatch(write_dir)["WRITE_SIZE"]
    copies = [k for k in wd if "copyBuffer" in k[1]]
    if not copies:
        raise SystemExit("no copy dispatch for calibration")
    target = copy_bytes / 1024.0
    cw = min(copies, key=lambda k: abs(wd[k] - target))
    # the same copy in the fetch run: the copy dispatch with the same rank by size
    cf = max((k for k in fd if "copyBuffer" in k[1]), key=lambda k: fd[k])
    f_scale = copy_bytes / (fd[cf] * 1024.0)
    w_scale = copy_bytes / (wd[cw] * 1024.0)
    print(f"Calibration: plain copy of {copy_bytes} bytes reads FETCH_SIZE {fd[cf]:.6g} KiB, "
          f"WRITE_SIZE {wd[cw]:.6g} KiB; scale factors {f_scale:.4f} (fetch), {w_scale:.4f} (write).\n")
    agg = defaultdict(lambda: [0.0, 0.0, 0, 0])
    for (did, k), v in fd.items():
        agg[k][0] += v * 1024.0 * f_scale
        agg[k][2] += 1
    for (did, k), v in wd.items():
        agg[k][1] += v * 1024.0 * w_scale
        agg[k][3] += 1
    print("| kernel | dispatches | HBM read GB per dispatch | HBM write GB per dispatch | total GB per dispatch |")
    print("|---|---|---|---|---|")
    for k, (r, w, nr, nw) in sorted(agg.items(), key=lambda x: -(x[1][0] + x[1][1])):
        n = max(nr, 1)
        if (r + w) / n < 1e6:
            continue
        print(f"| {k} | {n} | {r / n / 1e9:.3f} | {w / max(nw, 1) / 1e9:.3f} | {(r / n + w / max(nw, 1)) / 1e9:.3f} |")
    return 0


def main() -> int:
    if len(sys.argv) > 1 and sys.argv[1] == "--traffic":
        tp = argparse.ArgumentParser()
        tp.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
        tp.add_argument("--copy-bytes", type=int, required=True)
        t = tp.parse_args()
        return traffic(t.traffic[0], t.traffic[1], t.copy_bytes)
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
