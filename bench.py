#!/usr/bin/env python3
"""Benchmark of the in-place ScatterShuffle on one MI355X.

One step = one complete in-place shuffle (every tiled level, the fix-ups and
the LDS leaves) of the whole array, with a fresh 64-bit seed per step.  The
default workload is 2^32 uint32 elements (16 GiB), identity-initialised and
resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--config NAME]

The default line also carries a "batched" object: 10,000 ragged u32 arrays
(sizes floor(2^(4 + 16U))) shuffled by one shuffle_batched call, against a
loop of per-array shuffle_inplace_ex calls on the same data (same bytes out).
--config serve_u64 runs the serving workload instead: a Poisson stream of
u64 requests (sizes log-uniform in [2^10, 2^26]) admitted under a 64 GiB HBM
budget into a continuous-batching session, against serving the same stream
one request at a time; p50/p99 latency and Gelem/s per arrival rate.
--config batched_u32 times the enqueue-only batched call alone on the
10,000-array workload (one call per step), for profiling it.

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

# HBM bytes per launch of a kernel, from two rocprofv3 counter runs of this
# benchmark (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
# what the same counter read for a plain 16 GiB device copy in the same run
# (see profiles/traffic_k_rough_u32_2e32.md).  Valid only for the kernel
# sources they were taken on: a different source hash reports null.
TRAFFIC = {
    ("u32_2e32", "rough"): {
        "read_bytes": 17.198e9,
        "write_bytes": 17.342e9,
        "sources": ["k_rough.hip", "common.hpp", "rng.hpp", "kernels.hpp"],
        "sha256": "c5e248c53023ab972b21fab3b64e3797d48a957ebc625263ee911ade9c4c43db",
    },
}


def measured_traffic(config: str, kernel: str):
    import hashlib

    t = TRAFFIC.get((config, kernel))
    if t is None:
        return None
    h = hashlib.sha256()
    for f in t["sources"]:
        with open(os.path.join(ROOT, "paper_2302_03317_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != t["sha256"]:
        return None
    return t["read_bytes"] + t["write_bytes"]


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
            z = idx + (0x9E3779B97F4A7C15 - (1 << 64))  # splitmix64(i), wrapping int64 arithmetic
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


# The paper's own measurements (a CPU implementation; it reports no GPU
# numbers and gives absolute rates only in its figures): hardware context,
# not a target and not a baseline of this metric.
PAPER_CONTEXT = {
    "machine": "AMD EPYC 7702P, 64 cores / 128 threads, 512 GB RAM (Sec. 6)",
    "elements": "64-bit integers",
    "parallel_speedup_over_fastest_sequential": "up to 16x at 10 GiB and more (Sec. 6.4)",
    "self_speedup_100GiB": 32.2,
    "speedup_over_fisher_yates_100GiB": 142,
    "rough_scatter_share_of_first_level": "over 90 % for n >= 2^27, 99 % for n >= 2^33 (Sec. 6.6)",
}


def host_description() -> dict:
    """CPU model, the logical CPUs this process may use, and the RAM."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as fh:
            for ln in fh:
                if ln.startswith("MemTotal:"):
                    ram = int(ln.split()[1]) * 1024
                    break
    except OSError:
        pass
    cpus = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu": model, "logical_cpus_usable": cpus, "logical_cpus_total": os.cpu_count(),
            "ram_bytes": ram}


def host_threads() -> int:
    """Threads for the multi-core CPU baselines: the CPUs this process may
    use, at most OMP_NUM_THREADS when it is set."""
    cpus = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        cpus = min(cpus, int(env))
    return max(1, cpus)


def protocol_time(work, make_buffer, n: int, runs: int = 5, min_run_s: float = 0.1) -> dict:
    """The paper's timing protocol (Sec. 6): the mean of `runs` runs, each
    averaging repetitions that total at least min_run_s, on cold data: every
    run works on its own buffer, and the buffers together exceed 512 MB (or
    the run's data is larger than that itself)."""
    import numpy as np

    first = make_buffer()
    nbuf = max(2, min(16, -(-(512 << 20) // max(1, first.nbytes)) + 1))
    bufs = [first] + [make_buffer() for _ in range(nbuf - 1)]
    per_run = []
    for r in range(runs):
        a = bufs[r % nbuf]
        reps, t0 = 0, time.perf_counter()
        while True:
            work(a, 0x5EED + 1000 * r + reps)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= min_run_s:
                break
        per_run.append(dt / reps)
    mean = float(np.mean(per_run))
    return {"value": n / mean / 1e9, "unit": "Gelem/s", "seconds_per_shuffle": mean,
            "runs": runs, "run_seconds": [round(x, 4) for x in per_run],
            "buffer_bytes": int(bufs[0].nbytes), "buffers": nbuf}


def cpu_baselines(log2n: int, w: int, pip_log2n: int) -> dict:
    """CPU baselines on the host, each by the paper's protocol: the oracle on
    one core and on all usable cores (its buckets after the first level on
    host threads), textbook Fisher-Yates with the oracle's draws on one core,
    the paper's own parallel algorithm (host PIpScShuf) on all usable cores,
    and sequential Fisher-Yates with its generator on one core."""
    import hostshuf
    import oracle
    import workloads

    n = 1 << log2n
    params = oracle.default_params(n, w)
    threads = host_threads()
    host = host_description()
    # cold data: enough buffers that they exceed 512 MB together
    mk = lambda: workloads.identity(n, w)  # noqa: E731
    out = {}
    t = protocol_time(lambda a, s: oracle.shuffle(a, s, params), mk, n)
    out["cpu_baseline"] = dict(t, cores=1, kind="oracle",
                               sample=f"shuffles of 2^{log2n} {w}-byte elements (a bounded sample of the "
                                      f"workload), default parameters, one host thread, mean of 5 runs of "
                                      f">= 0.1 s on cold buffers", host=host)
    t = protocol_time(lambda a, s: oracle.shuffle(a, s, params, threads=threads), mk, n)
    out["cpu_oracle_threads"] = dict(t, cores=threads, kind="oracle, top-level buckets on host threads",
                                     sample=f"2^{log2n} {w}-byte elements")
    t = protocol_time(lambda a, s: oracle.fisher_yates(a, s), mk, n)
    out["cpu_fisher_yates"] = dict(t, cores=1, kind="sequential Fisher-Yates, the oracle's Philox draws",
                                   sample=f"2^{log2n} {w}-byte elements")
    npip = 1 << pip_log2n
    t = protocol_time(lambda a, s: hostshuf.shuffle(a, s, threads=threads),
                      lambda: workloads.identity(npip, w), npip)
    out["cpu_pipscshuf"] = dict(t, cores=threads,
                                kind="host PIpScShuf (the paper's parallel algorithm, Sec. 3-5; its own "
                                     "generator, so not the GPU's permutation)",
                                sample=f"2^{pip_log2n} {w}-byte elements")
    t = protocol_time(lambda a, s: hostshuf.fisher_yates(a, s), mk, n)
    out["cpu_fisher_yates_pcg"] = dict(t, cores=1, kind="sequential Fisher-Yates, 128-bit MCG generator",
                                       sample=f"2^{log2n} {w}-byte elements")
    return out


def batched_async_line(torch, shuf, steps: int, warmup: int, count: int = 10000, seed: int = 2026) -> dict:
    """The enqueue-only batched call alone on the batched workload (for
    profiling it): `warmup` untimed calls, then `steps` timed ones."""
    import numpy as np

    import workloads

    from paper_2302_03317_amd import autotune

    sizes = workloads.log_uniform_sizes(count, 4, 20, seed=seed)
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    total = int(host.size)
    found = autotune.lookup(autotune.load_table(), "batched_10000_u32", 4) if count == 10000 else None
    p, table_version = found if found else (shuf.default_params(0, 4), None)
    a = torch.from_numpy(host.view(np.int32)).to("cuda:0")
    ws = torch.zeros(shuf.batched_async_workspace_bytes(count, total, 4, p), dtype=torch.uint8, device="cuda:0")
    o = torch.tensor(np.asarray(offs, dtype=np.int64), device="cuda:0")
    seeds = [int.from_bytes(os.urandom(8), "little") for _ in range(warmup + steps)]
    for s_ in seeds[:warmup]:
        shuf.shuffle_batched_async(a, o, s_, ws, total, params=p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in seeds[warmup:]:
        shuf.shuffle_batched_async(a, o, s_, ws, total, params=p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    err = int(ws[:4].view(torch.int32).item())
    return {
        "metric": "batched enqueue-only shuffle throughput", "value": total / (ms / 1e3) / 1e9,
        "unit": "Gelem/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{count} u32 arrays, sizes floor(2^(4+16U)), {total} elements, identity per "
                               f"array, sizes seed {seed}; one shuffle_batched_async call per step",
                   "params": {"tile": p.tile, "kmax_log2": p.kmax_log2, "n0": p.n0, "lmax": p.lmax},
                   "params_table_version": table_version},
        "device_error_word": err,
    }


def batched_compare(torch, shuf, count: int = 10000, seed: int = 2026) -> dict:
    """shuffle_batched on `count` ragged u32 arrays vs per-array launches."""
    import numpy as np

    import workloads

    from paper_2302_03317_amd import autotune

    sizes = workloads.log_uniform_sizes(count, 4, 20, seed=seed)
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    total = int(host.size)
    # the autotuner's parameters for this workload (every form below uses them)
    found = autotune.lookup(autotune.load_table(), "batched_10000_u32", 4) if count == 10000 else None
    p, table_version = found if found else (shuf.default_params(0, 4), None)
    a = torch.from_numpy(host.view(np.int32)).to("cuda:0")
    b = a.clone()
    views = [b[int(offs[j]):int(offs[j + 1])] for j in range(count)]
    s0 = int.from_bytes(os.urandom(8), "little")
    shuf.shuffle_batched(a, offs, s0, params=p)          # warm-up (pools, first launches)
    for j, v in enumerate(views):
        if v.shape[0] > 1:
            shuf.shuffle_inplace_ex(v, s0, j, params=p)
    torch.cuda.synchronize()
    seed_t = int.from_bytes(os.urandom(8), "little")
    reps = 5
    t0 = time.perf_counter()
    for r in range(reps):
        shuf.shuffle_batched(a, offs, seed_t + r, params=p)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for r in range(reps):
        for j, v in enumerate(views):
            if v.shape[0] > 1:
                shuf.shuffle_inplace_ex(v, seed_t + r, j, params=p)
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / reps
    same = bool(torch.equal(a, b))
    # algorithmic bytes of one blocking batched call (every element each kernel
    # moves counted once read and once written), from the library's spans
    shuf.timing_enable(True)
    shuf.shuffle_batched(a, offs, seed_t + 99, params=p)
    torch.cuda.synchronize()
    call_bytes = sum(v["bytes"] for v in shuf.timing_read().values())
    shuf.timing_enable(False)
    # the enqueue-only form: eager calls, and one call captured into a graph
    # and replayed (each replay shuffles the batch again with the captured seed)
    wsb = shuf.batched_async_workspace_bytes(count, total, 4, p)
    ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda:0")
    o = torch.tensor(np.asarray(offs, dtype=np.int64), device="cuda:0")
    shuf.shuffle_batched_async(a, o, s0, ws, total, params=p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        shuf.shuffle_batched_async(a, o, seed_t + r, ws, total, params=p)
    torch.cuda.synchronize()
    t_async = (time.perf_counter() - t0) / reps
    async_err = int(ws[:4].view(torch.int32).item())
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            shuf.shuffle_batched_async(a, o, seed_t + 1234, ws, total, stream=gs, params=p)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    graph_err = int(ws[:4].view(torch.int32).item())
    del graph, ws
    return {
        "workload": f"{count} u32 arrays, sizes floor(2^(4+16U)), {total} elements "
                    f"({total * 4 / 2**30:.2f} GiB), identity per array, sizes seed {seed}",
        "batched_ms": t_batched * 1e3,
        "batched_Gelem_s": total / t_batched / 1e9,
        "per_array_launches_ms": t_single * 1e3,
        "per_array_Gelem_s": total / t_single / 1e9,
        "speedup": t_single / t_batched,
        "identical_outputs": same,
        "batched_algorithmic_bytes": call_bytes,
        "batched_GBs": call_bytes / t_batched / 1e9,
        "batched_frac_of_hbm_peak": call_bytes / t_batched / 1e9 / HBM_PEAK_GBS,
        "params": {"tile": p.tile, "kmax_log2": p.kmax_log2, "n0": p.n0, "lmax": p.lmax},
        "params_source": (f"autotuner table paper_2302_03317_amd/pi_table.json, version {table_version}"
                          if table_version is not None else "defaults (no table entry)"),
        "form": "blocking: level by level in shared launches, stream synchronised after each tiled "
                "level (not graph-capturable)",
        "async_ms": t_async * 1e3,
        "async_Gelem_s": total / t_async / 1e9,
        "async_form": "enqueue-only: first level planned on the device, bounded grids, persistent "
                      "leaf workgroups with per-class work counters",
        "graph_replay_ms": t_graph * 1e3,
        "graph_replay_Gelem_s": total / t_graph / 1e9,
        "async_device_errors": [async_err, graph_err],
        "speedup_graph_vs_per_array": t_single / t_graph,
    }


def serving(torch, shuf, rates, count: int, budget_bytes: int, seed: int = 7) -> list:
    """Poisson stream of u64 shuffle requests; continuous batching (the
    session admits requests by the budget: data plus a workspace bound, or
    the library's exact workspace when the bound does not fit) against
    serving one request at a time."""
    import numpy as np

    import workloads

    w = 8
    sizes = workloads.log_uniform_sizes(count, 10, 26, seed=seed)
    # request data stays resident: one buffer per request
    bufs = [torch.empty(int(n), dtype=torch.int64, device="cuda:0") for n in sizes]
    # warm-up: grow the library's pools with a burst of the largest requests
    big = sorted(range(count), key=lambda j: -int(sizes[j]))[:64]
    with shuf.Session(w) as sess:
        for j in big:
            sess.submit(bufs[j], j, j)
        while sess.inflight()[0]:
            sess.step()
    for j in big[:8]:
        shuf.shuffle_inplace_ex(bufs[j], j, j)
    torch.cuda.synchronize()
    results = []
    for rate in rates:
        arrivals = workloads.poisson_arrivals(count, rate, seed + int(rate))
        seeds = np.random.default_rng(seed + 1).integers(0, 2**63, size=count)
        for mode in ("session", "one_at_a_time"):
            lat = np.zeros(count)
            steps = 0
            batch = []
            queued_max = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "session":
                sess = shuf.Session(w)
                sess.set_budget(budget_bytes)
                nxt, submitted = 0, {}
                done_n = 0
                while done_n < count:
                    now = time.perf_counter() - t0
                    while nxt < count and arrivals[nxt] <= now:
                        tk = sess.submit(bufs[nxt], int(seeds[nxt]), nxt)
                        submitted[tk] = nxt
                        nxt += 1
                    inflight = sess.inflight()[0]
                    if inflight == 0:
                        if nxt < count:
                            wait = arrivals[nxt] - (time.perf_counter() - t0)
                            if wait > 0:
                                time.sleep(min(wait, 0.001))
                        continue
                    batch.append(inflight)
                    queued_max = max(queued_max, sess.queued()[0])
                    done = sess.step()
                    steps += 1
                    tdone = time.perf_counter() - t0
                    for tk in done:
                        j = submitted.pop(tk)
                        lat[j] = tdone - arrivals[j]
                        done_n += 1
                sess.close()
            else:
                for j in range(count):
                    now = time.perf_counter() - t0
                    if arrivals[j] > now:
                        time.sleep(arrivals[j] - now)
                    shuf.shuffle_inplace_ex(bufs[j], int(seeds[j]), j)
                    lat[j] = time.perf_counter() - t0 - arrivals[j]
            elapsed = time.perf_counter() - t0
            elems = float(np.sum(sizes))
            results.append({
                "rate_per_s": rate,
                "mode": mode,
                "requests": count,
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "Gelem_s": elems / elapsed / 1e9,
                "elapsed_s": elapsed,
                "steps": steps,
                "mean_inflight_per_step": float(np.mean(batch)) if batch else None,
                "max_queued_by_budget": queued_max if mode == "session" else None,
            })
            print(f"[serve] rate {rate}/s {mode}: p50 {results[-1]['p50_ms']:.2f} ms "
                  f"p99 {results[-1]['p99_ms']:.2f} ms {results[-1]['Gelem_s']:.2f} Gelem/s",
                  file=sys.stderr, flush=True)
    del bufs
    torch.cuda.empty_cache()
    return results


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="u32_2e32", choices=sorted(CONFIGS) + ["serve_u64", "batched_u32"])
    ap.add_argument("--no-batched", action="store_true", help="skip the batched comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="before the timed region, copy the array once device-to-device (a plain "
                         "copy of known size for scaling HBM byte counters)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sweep of the default line")
    ap.add_argument("--line-serve-requests", type=int, default=300)
    ap.add_argument("--line-serve-rates", default="2000,8000,16000")
    ap.add_argument("--serve-rates", default="1000,2000,4000,8000,16000")
    ap.add_argument("--cpu-sample-log2", type=int, default=24)
    ap.add_argument("--cpu-pip-log2", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the shuffle runs on one GPU (no multi-GPU path); --gpus {args.gpus} is not supported",
              file=sys.stderr)
        return 2

    import torch

    import paper_2302_03317_amd as shuf

    if args.config == "serve_u64":
        rates = [float(r) for r in args.serve_rates.split(",")]
        res = serving(torch, shuf, rates, args.serve_requests, 64 << 30)
        top = [r for r in res if r["mode"] == "session"][-1]
        print(json.dumps({
            "metric": "serving: p50/p99 latency and Gelem/s under Poisson arrivals",
            "value": top["Gelem_s"], "unit": "Gelem/s", "n_gpus": 1,
            "steps": args.serve_requests, "warmup": 0,
            "ms_per_step": top["elapsed_s"] * 1e3 / args.serve_requests,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic",
            "config": {"workload": "Poisson stream of in-place shuffles of u64 arrays, sizes "
                                   "log-uniform in [2^10, 2^26], 64 GiB HBM budget, data resident",
                       "rates_per_s": rates, "requests_per_rate": args.serve_requests},
            "sweep": res,
        }), flush=True)
        return 0

    if args.config == "batched_u32":
        print(json.dumps(batched_async_line(torch, shuf, args.steps, args.warmup)), flush=True)
        return 0

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
    if args.copy_calibration:
        u = torch.empty_like(t)
        u.copy_(t)
        torch.cuda.synchronize()
        del u
        torch.cuda.empty_cache()
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
        "traffic": measured_traffic(args.config, dom),
        "bytes_per_launch": per_launch_bytes,
        "avg_launch_ms": per_launch_s * 1e3,
    }
    # the whole step: every kernel's algorithmic bytes (each element a kernel
    # moves counted once read and once written) over the step time
    step_bytes = sum(v["bytes"] for v in kt.values()) / args.steps
    step_gbs = step_bytes / (ms_per_step / 1e3) / 1e9
    step_roofline = {
        "bound": "hbm",
        "algorithmic_bytes_per_step": step_bytes,
        "achieved": step_gbs,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": step_gbs / HBM_PEAK_GBS,
        "target_frac": 0.6,
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
        "step_roofline": step_roofline,
        "kernels": kernels,
        "levels": {"tiled_levels": stats["tiled_levels"], "movers_last_step": stats["movers"],
                   "leaves_last_step": stats["leaves"], "workspace_bytes": stats["workspace_bytes"]},
        "checksum_preserved": before == after,
        # how the kernels took the stable ranks on this device (both ways give
        # the same permutation): 1 = LDS atomic adds, whose lane order the
        # device's probe checked at the first call; 0 = ballots
        "rank_method": {1: "lds_atomic_lane_order_probed", 0: "ballot"}.get(shuf.rank_method(), "none"),
    }
    if not args.no_batched:
        del t
        torch.cuda.empty_cache()
        line["batched"] = batched_compare(torch, shuf)
    if not args.no_serving:
        if "t" in locals():
            del t
            torch.cuda.empty_cache()
        rates = [float(r) for r in args.line_serve_rates.split(",")]
        sweep = serving(torch, shuf, rates, args.line_serve_requests, 64 << 30)
        line["serving"] = {
            "workload": "Poisson stream of in-place shuffles of u64 arrays, sizes log-uniform in "
                        "[2^10, 2^26], 64 GiB HBM budget admitted by the session (data plus a "
                        "workspace bound per request, the exact workspace when the bound does not "
                        "fit), data resident",
            "requests_per_rate": args.line_serve_requests,
            "sweep": sweep,
        }
    if not args.no_cpu_baseline:
        line.update(cpu_baselines(min(args.cpu_sample_log2, log2n), w, min(args.cpu_pip_log2, log2n)))
    line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)
    return 0 if before == after else 1


if __name__ == "__main__":
    sys.exit(main())
