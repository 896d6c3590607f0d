"""The headline sizes, bit-exact against the oracle.

The oracle's outputs at these sizes (16 GiB and more) are stored as SHA-256
digests -- of the whole array and of 64 equal chunks -- plus sampled
elements, by tests/golden/make_fullsize_digests.py, which calls only the CPU
oracle.  Here the GPU library shuffles the same input through its C ABI in
the benchmark's launch configuration (shuffle_inplace: stream id 0, default
parameters; shuffle_batched for the ragged batch) and its output bytes are
hashed the same way.  Equal digests mean the two outputs are identical byte
for byte."""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "fullsize_digests.json")


def _golden(name):
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/fullsize_digests.json not written")
    with open(GOLDEN) as fh:
        g = json.load(fh)
    if name not in g:
        pytest.skip(f"no stored digest for {name}")
    return g[name]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _lib():
    import paper_2302_03317_amd as shuf

    shuf.lib()
    return shuf


def device_digests(t, chunks=64):
    """SHA-256 of a device tensor's bytes (whole and per chunk), streamed
    through a pinned host buffer."""
    flat = t.reshape(-1).view(torch.uint8)
    nbytes = flat.numel()
    piece = 1 << 28
    host = torch.empty(piece, dtype=torch.uint8, pin_memory=True)
    total = hashlib.sha256()
    parts = []
    for c in range(chunks):
        a, b = nbytes * c // chunks, nbytes * (c + 1) // chunks
        h = hashlib.sha256()
        for s in range(a, b, piece):
            e = min(b, s + piece)
            host[: e - s].copy_(flat[s:e])
            mv = host[: e - s].numpy()
            h.update(mv)
            total.update(mv)
        parts.append(h.hexdigest())
    return total.hexdigest(), parts


def check_against(t, g, what):
    digest, parts = device_digests(t)
    if digest == g["sha256"]:
        return
    bad = [i for i, (a, b) in enumerate(zip(parts, g["chunk_sha256"])) if a != b]
    pos = torch.tensor(g["samples"]["positions"], dtype=torch.int64, device=t.device)
    got = t[pos].cpu().numpy()
    got = got.view(np.uint32) if got.dtype == np.int32 else got.view(np.uint64)
    want = np.array(g["samples"]["values"], dtype=np.uint64).reshape(got.shape[0], -1)
    diff = np.nonzero((got.reshape(got.shape[0], -1).astype(np.uint64) != want).any(axis=1))[0]
    raise AssertionError(f"{what}: output differs from the oracle in chunks {bad[:16]} of 64; "
                         f"{diff.size} of {len(pos)} sampled positions differ, first at "
                         f"{[int(g['samples']['positions'][i]) for i in diff[:8]]}")


def fill_identity(t, n, mod32):
    chunk = 1 << 27
    for a in range(0, n, chunk):
        idx = torch.arange(a, min(n, a + chunk), dtype=torch.int64, device=t.device)
        t[a:a + chunk] = idx.to(t.dtype) if mod32 else idx


@pytest.mark.parametrize("name", ["u32_2e32", "u64_2e31", "u32_2e32_plus_12345"])
def test_headline_single_array_equals_oracle(name):
    """2^32 u32, 2^31 u64 (three tiled levels at full size, level 0 with
    about 264k and 526k tiles) and 2^32 + 12345 u32 (positions beyond 2^32,
    64-bit piece arithmetic), element by element through their digests."""
    g = _golden(name)
    shuf = _lib()
    dev = _dev()
    n, w = g["n"], g["elem_bytes"]
    print(f"[gpu] full-size digest {name}: n={n} w={w} seed={g['seed']:#x}", flush=True)
    t = torch.empty(n, dtype=torch.int32 if w == 4 else torch.int64, device=dev)
    fill_identity(t, n, w == 4)
    shuf.shuffle_inplace(t, g["seed"])
    torch.cuda.synchronize()
    print(f"[gpu] {name}: shuffled, hashing", flush=True)
    check_against(t, g, name)
    del t
    torch.cuda.empty_cache()


def test_batched_10000_arrays_equals_oracle():
    """The ragged batch of 10,000 u32 arrays (sizes floor(2^(4 + 16U)) from
    seed 2026, identity per array), one shuffle_batched call, against the
    oracle run per array with stream id = array index."""
    g = _golden("batched_10000_u32")
    shuf = _lib()
    dev = _dev()
    sizes = workloads.log_uniform_sizes(g["count"], 4, 20, seed=g["sizes_seed"])
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    assert host.size == g["total_elements"]
    print(f"[gpu] batched digest: arrays={len(sizes)} total={host.size} seed={g['seed']:#x}", flush=True)
    t = torch.from_numpy(host.view(np.int32)).to(dev)
    del host
    shuf.shuffle_batched(t, offs, g["seed"])
    torch.cuda.synchronize()
    check_against(t, g, "batched 10000 u32")
