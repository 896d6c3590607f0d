#!/usr/bin/env python3
"""Benchmark of the in-place ScatterShuffle on one MI355X.

One step = one complete in-place shuffle (every tiled level, the fix-ups and
the LDS leaves) of the whole array, with a fresh 64-bit seed per step.  The
default workload is 2^32 uint32 elements (16 GiB), identity-initialised and
resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config NAME]

Per-kernel times come from HIP events that the library records on the
launch stream around every kernel group inside the timed region.  The CPU
baseline times the CPU oracle on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # name: (log2 n, element bytes, description)
    "u32_2e32": (32, 4, "single in-place shuffle, uint32, n=2^32 (16 GiB), identity"),
    "u64_2e31": (31, 8, "single in-place shuffle, uint64, n=2^31 (16 GiB), identity"),
    "u32_2e28": (28, 4, "single in-place shuffle, uint32, n=2^28 (1 GiB), identity"),
    "u64_2e28": (28, 8, "single in-place shuffle, uint64, n=2^28 (2 GiB), identity"),
    "rec16_2e28": (28, 16, "single in-place shuffle, 16-byte records, n=2^28 (4 GiB), key=i, payload=splitmix64(i)"),
    "u32_2e20": (20, 4, "single in-place shuffle, uint32, n=2^20 (4 MiB), identity"),
}
HBM_PEAK_GBS = 8000.0


def fill_identity(t, n, w, torch):
    """Identity contents written on the GPU in chunks (element i holds i)."""
    chunk = 1 << 27
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        idx = torch.arange(a, b, dtype=torch.int64, device=t.device)
        if w == 4:
            t[a:b] = idx.to(torch.int32)
        elif w == 8:
            t[a:b] = idx
        else:
            t[a:b, 0] = idx
            z = idx + 0x9E3779B97F4A7C15 - (1 << 64)  # splitmix64(i), wrapping int64 arithmetic
            z = (z ^ (z >> 30).bitwise_and((1 << 34) - 1)) * (0xBF58476D1CE4E5B9 - (1 << 64))
            z = (z ^ (z >> 27).bitwise_and((1 << 37) - 1)) * (0x94D049BB133111EB - (1 << 64))
            t[a:b, 1] = z ^ (z >> 31).bitwise_and((1 << 33) - 1)


def checksum(t, torch):
    """Sum and sum of squares of the element words modulo 2^64 (unchanged by
    any permutation)."""
    v = (t.view(torch.int32) if t.dtype == torch.int32 else t.view(torch.int64)).reshape(-1)
    s1 = s2 = 0
    chunk = 1 << 27
    for a in range(0, v.numel(), chunk):
        part = v[a:a + chunk].to(torch.int64)
        s1 += int(part.sum().item())
        s2 += int((part * part).sum().item())
    return s1 % (1 << 64), s2 % (1 << 64)


def cpu_baseline(log2n: int, w: int) -> dict:
    """The CPU oracle (single thread) on a bounded sample of the workload."""
    import numpy as np

    import oracle
    import workloads

    n = 1 << log2n
    a = workloads.identity(n, w)
    t0 = time.perf_counter()
    oracle.shuffle(a, 0x5EED, oracle.default_params(n, w))
    dt = time.perf_counter() - t0
    return {
        "value": n / dt / 1e9,
        "unit": "Gelem/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one shuffle of 2^{log2n} {w}-byte identity elements, default parameters, "
                  f"{dt:.1f} s on one host core",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="u32_2e32", choices=sorted(CONFIGS))
    ap.add_argument("--cpu-sample-log2", type=int, default=26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        return 2

    import torch

    import paper_2302_03317_amd as shuf

    log2n, w, desc = CONFIGS[args.config]
    n = 1 << log2n
    dev = torch.device("cuda:0")
    if w == 4:
        t = torch.empty(n, dtype=torch.int32, device=dev)
    elif w == 8:
        t = torch.empty(n, dtype=torch.int64, device=dev)
    else:
        t = torch.empty((n, 2), dtype=torch.int64, device=dev)
    fill_identity(t, n, w, torch)
    torch.cuda.synchronize()
    before = checksum(t, torch)
    params = shuf.default_params(n, w)

    seeds = [int.from_bytes(os.urandom(8), "little") for _ in range(args.warmup + args.steps)]
    for s in seeds[: args.warmup]:
        shuf.shuffle_inplace(t, s)
    torch.cuda.synchronize()

    shuf.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in seeds[args.warmup:]:
        shuf.shuffle_inplace(t, s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = shuf.timing_read()
    shuf.timing_enable(False)
    stats = shuf.last_stats()
    after = checksum(t, torch)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gelem = n / (ms_per_step / 1e3) / 1e9
    useful_gbs = 2.0 * n * w / (ms_per_step / 1e3) / 1e9

    kernels = {}
    for k, v in kt.items():
        if v["launches"] == 0:
            continue
        kernels[k] = {
            "ms_per_step": v["ms"] / args.steps,
            "launches_per_step": v["launches"] / args.steps,
            "algorithmic_GBs": (v["bytes"] / (v["ms"] / 1e3) / 1e9) if v["bytes"] > 0 else None,
        }
    dom = max((k for k in kt if kt[k]["bytes"] > 0), key=lambda k: kt[k]["ms"])
    d = kt[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_s = d["ms"] / d["launches"] / 1e3
    achieved = per_launch_bytes / per_launch_s / 1e9
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": None,
        "bytes_per_launch": per_launch_bytes,
        "avg_launch_ms": per_launch_s * 1e3,
    }
    line = {
        "metric": "Gelem/s and achieved HBM GB/s (% of peak), single vs batched, bit-exact",
        "value": gelem,
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {4: "u32", 8: "u64", 16: "u64x2"}[w],
        "data": "synthetic",
        "config": {
            "workload": desc,
            "n": n,
            "elem_bytes": w,
            "params": {"tile": params.tile, "kmax_log2": params.kmax_log2, "n0": params.n0,
                       "lmax": params.lmax},
            "seeds": "fresh 64-bit seed per step from os.urandom",
        },
        "useful_GBs": useful_gbs,
        "useful_frac_of_peak": useful_gbs / HBM_PEAK_GBS,
        "roofline": roofline,
        "kernels": kernels,
        "levels": {"tiled_levels": stats["tiled_levels"], "movers_last_step": stats["movers"],
                   "leaves_last_step": stats["leaves"], "workspace_bytes": stats["workspace_bytes"]},
        "checksum_preserved": before == after,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(min(args.cpu_sample_log2, log2n), w)
    print(json.dumps(line), flush=True)
    return 0 if before == after else 1


if __name__ == "__main__":
    sys.exit(main())
