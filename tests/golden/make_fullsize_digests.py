#!/usr/bin/env python3
"""Write tests/golden/fullsize_digests.json: the oracle's outputs at the
headline sizes, as SHA-256 digests (whole array and 64 equal chunks) plus
sampled elements.

Calls only the CPU oracle (oracle/) on inputs from workloads.py; nothing
here comes from the GPU library.  Each case runs in a child process so that
its memory (about 2.6 times the array) is returned before the next one.

    python tests/golden/make_fullsize_digests.py [case ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "fullsize_digests.json")

# name: (n, elem_bytes, input, seed)
CASES = {
    "u32_2e32": (1 << 32, 4, "identity", 0x2302033172026001),
    "u64_2e31": (1 << 31, 8, "identity", 0x2302033172026002),
    "u32_2e32_plus_12345": ((1 << 32) + 12345, 4, "identity_mod32", 0x2302033172026003),
}
BATCHED = {"name": "batched_10000_u32", "count": 10000, "lo_log2": 4, "hi_log2": 20,
           "sizes_seed": 2026, "seed": 0x2302033172026004}
CHUNKS = 64
SAMPLES = 1024


def digests(arr) -> dict:
    import numpy as np

    flat = arr.reshape(-1).view(np.uint8)
    total = hashlib.sha256()
    parts = []
    nbytes = flat.size
    for c in range(CHUNKS):
        a, b = nbytes * c // CHUNKS, nbytes * (c + 1) // CHUNKS
        h = hashlib.sha256(flat[a:b])
        parts.append(h.hexdigest())
        total.update(flat[a:b])
    return {"sha256": total.hexdigest(), "chunk_sha256": parts}


def samples(arr, n: int, seed: int) -> dict:
    import numpy as np

    rng = np.random.default_rng(seed)
    pos = np.unique(np.concatenate([np.arange(min(n, 64)), np.arange(max(0, n - 64), n),
                                    rng.integers(0, n, size=SAMPLES)])).astype(np.int64)
    vals = arr[pos]
    return {"positions": pos.tolist(), "values": vals.reshape(len(pos), -1).tolist()}


def run_case(name: str) -> dict:
    import numpy as np

    import oracle
    import workloads

    n, w, kind, seed = CASES[name]
    arr = workloads.identity_mod32(n) if kind == "identity_mod32" else workloads.identity(n, w)
    threads = os.cpu_count() or 1
    t0 = time.time()
    oracle.shuffle(arr, seed, oracle.default_params(n, w), stream_id=0, threads=threads)
    dt = time.time() - t0
    rec = {"n": n, "elem_bytes": w, "input": kind, "seed": seed, "stream_id": 0,
           "params": "default", "oracle_seconds": round(dt, 1), "oracle_threads": threads}
    rec.update(digests(arr))
    rec["samples"] = samples(arr, n, seed & 0xFFFF)
    return rec


def run_batched() -> dict:
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import workloads

    b = BATCHED
    sizes = workloads.log_uniform_sizes(b["count"], b["lo_log2"], b["hi_log2"], seed=b["sizes_seed"])
    offs = workloads.csr_offsets(sizes)
    arr = workloads.batched_identity(sizes)
    t0 = time.time()

    def one(j):
        a, e = int(offs[j]), int(offs[j + 1])
        if e - a > 1:
            oracle.shuffle(arr[a:e], b["seed"], oracle.default_params(e - a, 4), stream_id=j)

    with ThreadPoolExecutor(max_workers=os.cpu_count() or 1) as ex:
        list(ex.map(one, range(b["count"])))
    dt = time.time() - t0
    rec = {"count": b["count"], "sizes": f"floor(2^({b['lo_log2']} + {b['hi_log2'] - b['lo_log2']}U)), "
           f"workloads.log_uniform_sizes seed {b['sizes_seed']}", "sizes_seed": b["sizes_seed"],
           "total_elements": int(arr.size), "elem_bytes": 4, "input": "identity per array",
           "seed": b["seed"], "stream_id": "array index", "params": "default",
           "oracle_seconds": round(dt, 1)}
    rec.update(digests(arr))
    rec["samples"] = samples(arr, int(arr.size), 2026)
    return rec


def main() -> int:
    if len(sys.argv) == 3 and sys.argv[1] == "--child":
        name = sys.argv[2]
        rec = run_batched() if name == BATCHED["name"] else run_case(name)
        sys.stdout.write(json.dumps(rec))
        return 0
    names = sys.argv[1:] or [*CASES, BATCHED["name"]]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in names:
        print(f"[golden] {name} ...", flush=True)
        res = subprocess.run([sys.executable, os.path.abspath(__file__), "--child", name],
                             check=True, stdout=subprocess.PIPE)
        data[name] = json.loads(res.stdout)
        print(f"[golden] {name}: {data[name]['sha256']} ({data[name]['oracle_seconds']} s)", flush=True)
        data["_about"] = ("SHA-256 of the CPU oracle's output bytes (definition version 1) at the "
                          "headline sizes, written by tests/golden/make_fullsize_digests.py, which "
                          "calls only oracle/ on inputs from workloads.py")
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
