"""The enqueue-only batched call (shuffle_batched_async): device-planned first
level, bounded grids, persistent leaf workgroups, no host synchronisation.
Array j must equal the single-array definition with stream id j: checked
against the oracle on ragged batches of every width, against the stored
oracle digest of the 10,000-array workload, and through a HIP graph that is
captured once and replayed."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def _lib():
    import paper_2302_03317_amd as shuf

    shuf.lib()
    return shuf


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(host):
    view = host.view(np.int32) if host.dtype == np.uint32 else host.view(np.int64)
    return torch.from_numpy(view.copy()).to(_dev())


def from_dev(t, like):
    return t.cpu().numpy().view(like.dtype).reshape(like.shape)


def run_async(shuf, t, offs, seed, total=None):
    dev = _dev()
    count = len(offs) - 1
    total = int(offs[-1]) if total is None else total
    w = t.element_size() * (t.shape[1] if t.dim() > 1 else 1)
    wsb = shuf.batched_async_workspace_bytes(count, total, w)
    ws = torch.zeros(wsb, dtype=torch.uint8, device=dev)
    o = torch.tensor(np.asarray(offs, dtype=np.int64), device=dev)
    shuf.shuffle_batched_async(t, o, seed, ws, total)
    torch.cuda.synchronize()
    return int(ws[:4].view(torch.int32).item())


@pytest.mark.parametrize("w", [4, 8, 16])
def test_async_ragged_batch_equals_oracle(w):
    shuf = _lib()
    T = 65536 // w
    mx = shuf.batched_async_max_elems(w)
    sizes = [0, 1, 2, 3, 64, 65, T - 256, T - 255, 2 * T + 7, 0, 1, 5 * T + 3, 1000, mx, 17, mx - 1]
    parts = [workloads.random_values(s, w, 900 + i) for i, s in enumerate(sizes)]
    host = np.concatenate(parts, axis=0)
    offs = workloads.csr_offsets(np.array(sizes, dtype=np.uint64))
    print(f"[gpu] async batch w={w} arrays={len(sizes)} total={host.shape[0]} max={mx}", flush=True)
    t = to_dev(host)
    assert run_async(shuf, t, offs, 4242) == 0
    got = from_dev(t, host)
    for j, s in enumerate(sizes):
        a, b = int(offs[j]), int(offs[j + 1])
        want = host[a:b].copy()
        if s > 1:
            oracle.shuffle(want, 4242, oracle.default_params(s, w), stream_id=j)
        assert np.array_equal(got[a:b], want), f"async w={w} array {j} (n={s})"


@pytest.mark.parametrize("tile_bytes,kmax_log2,n0", [(32768, 8, 32), (65536, 7, 128), (65536, 6, 16),
                                                    (16384, 8, 48)])
def test_async_nondefault_params_equal_oracle(tile_bytes, kmax_log2, n0):
    """The enqueue-only call with parameters other than the defaults (the
    autotuner's candidates and smaller tiles), u32 and u64 arrays up to the
    largest size those parameters finish in one tiled level, against the
    oracle with the same parameters; the blocking batched call with the same
    parameters must give the same bytes."""
    shuf = _lib()
    for w in (4, 8):
        p = shuf.Params(tile_bytes // w, kmax_log2, n0, 32)
        mx = shuf.batched_async_max_elems(w, p)
        assert mx == (p.tile // 2) << kmax_log2
        T = p.tile
        sizes = [mx, 0, 2, T - (1 << kmax_log2), T - (1 << kmax_log2) + 1, 3 * T + 5, 77, mx - 3, 1, 5000]
        parts = [workloads.random_values(sz, w, 7000 + i) for i, sz in enumerate(sizes)]
        host = np.concatenate(parts, axis=0)
        offs = workloads.csr_offsets(np.array(sizes, dtype=np.uint64))
        print(f"[gpu] async params tile={p.tile} kmax_log2={kmax_log2} n0={n0} w={w} total={host.shape[0]}",
              flush=True)
        dev = _dev()
        t = to_dev(host)
        total = int(offs[-1])
        wsb = shuf.batched_async_workspace_bytes(len(sizes), total, w, p)
        ws = torch.zeros(wsb, dtype=torch.uint8, device=dev)
        o = torch.tensor(np.asarray(offs, dtype=np.int64), device=dev)
        shuf.shuffle_batched_async(t, o, 31337, ws, total, params=p)
        torch.cuda.synchronize()
        assert int(ws[:4].view(torch.int32).item()) == 0
        b = to_dev(host)
        shuf.shuffle_batched(b, offs, 31337, params=p)
        torch.cuda.synchronize()
        assert torch.equal(t, b)
        got = from_dev(t, host)
        op = oracle.Params(p.tile, p.kmax_log2, p.n0, p.lmax)
        for j, sz in enumerate(sizes):
            a, e = int(offs[j]), int(offs[j + 1])
            want = host[a:e].copy()
            if sz > 1:
                oracle.shuffle(want, 31337, op, stream_id=j)
            assert np.array_equal(got[a:e], want), f"array {j} (n={sz})"


def test_async_equals_blocking_batched_on_random_sizes():
    shuf = _lib()
    sizes = workloads.log_uniform_sizes(700, 0, 20, seed=17)
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    print(f"[gpu] async vs blocking: arrays={len(sizes)} total={host.size}", flush=True)
    a = to_dev(host)
    assert run_async(shuf, a, offs, 99) == 0
    b = to_dev(host)
    shuf.shuffle_batched(b, offs, 99)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_async_10000_arrays_equals_oracle_digest():
    """The headline batched workload, against the stored oracle digest."""
    import hashlib

    path = os.path.join(HERE, "golden", "fullsize_digests.json")
    with open(path) as fh:
        g = json.load(fh)["batched_10000_u32"]
    shuf = _lib()
    sizes = workloads.log_uniform_sizes(g["count"], 4, 20, seed=g["sizes_seed"])
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    print(f"[gpu] async batched digest: arrays={len(sizes)} total={host.size}", flush=True)
    t = torch.from_numpy(host.view(np.int32)).to(_dev())
    assert run_async(shuf, t, offs, g["seed"]) == 0
    digest = hashlib.sha256(t.cpu().numpy().view(np.uint8)).hexdigest()
    assert digest == g["sha256"]


def test_async_repeated_calls_equal_oracle():
    """Persistent leaf workgroups run leaf after leaf; a level's segment count
    written by one lane must be seen by every wave after the barrier.  When
    it was not (no LDS wait before a loop-top barrier), about one run in
    three left 64 children of one leaf without their Fisher-Yates pass: six
    runs of 1025 arrays, each against the oracle."""
    shuf = _lib()
    sizes = workloads.log_uniform_sizes(10000, 4, 20, seed=2026)[:1025]
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    seed = 0x2302033172026004
    want = host.copy()
    for j in range(len(sizes)):
        a, b = int(offs[j]), int(offs[j + 1])
        if b - a > 1:
            oracle.shuffle(want[a:b], seed, oracle.default_params(b - a, 4), stream_id=j, threads=8)
    for run in range(6):
        print(f"[gpu] async repeated: run {run}, arrays={len(sizes)} total={host.size}", flush=True)
        t = to_dev(host)
        assert run_async(shuf, t, offs, seed) == 0
        got = from_dev(t, host)
        bad = [j for j in range(len(sizes))
               if not np.array_equal(got[int(offs[j]):int(offs[j + 1])], want[int(offs[j]):int(offs[j + 1])])]
        assert not bad, f"run {run}: arrays {bad[:10]} differ from the oracle"


def test_tuned_params_batched_equals_oracle():
    """The 10,000-array workload with the parameters of the autotuner's table,
    read by the library's reader for the GPU call and by the oracle's own
    reader for the expected result (arrays solved on host threads)."""
    import hashlib
    from concurrent.futures import ThreadPoolExecutor

    from paper_2302_03317_amd import autotune

    shuf = _lib()
    table_path = os.path.join(os.path.dirname(HERE), "paper_2302_03317_amd", "pi_table.json")
    p_lib, version = autotune.lookup(autotune.load_table(table_path), "batched_10000_u32", 4)
    p_or, _ = oracle.params_from_table(table_path, "batched_10000_u32", 4)
    sizes = workloads.log_uniform_sizes(10000, 4, 20, seed=2026)
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    seed = 0x2302033172026005
    print(f"[gpu] tuned parameters (table version {version}): {p_lib}, arrays={len(sizes)} total={host.size}",
          flush=True)
    t = to_dev(host)
    dev = _dev()
    total = int(offs[-1])
    wsb = shuf.batched_async_workspace_bytes(len(sizes), total, 4, p_lib)
    ws = torch.zeros(wsb, dtype=torch.uint8, device=dev)
    o = torch.tensor(np.asarray(offs, dtype=np.int64), device=dev)
    shuf.shuffle_batched_async(t, o, seed, ws, total, params=p_lib)
    torch.cuda.synchronize()
    assert int(ws[:4].view(torch.int32).item()) == 0
    got = hashlib.sha256(t.cpu().numpy().view(np.uint8)).hexdigest()
    b = to_dev(host)
    shuf.shuffle_batched(b, offs, seed, params=p_lib)
    torch.cuda.synchronize()
    assert torch.equal(b, t), "blocking and enqueue-only forms differ with the tuned parameters"
    del t, b, ws

    want = host.copy()

    def one(j):
        a, e = int(offs[j]), int(offs[j + 1])
        if e - a > 1:
            oracle.shuffle(want[a:e], seed, p_or, stream_id=j)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(one, range(len(sizes))))
    assert got == hashlib.sha256(want.view(np.uint8)).hexdigest()


def test_async_captured_graph_replays():
    """Captured once into a HIP graph and replayed three times, with other
    work and synchronisations between the replays: replay r leaves the
    batch permuted r + 1 times, as the same number of eager calls does."""
    shuf = _lib()
    dev = _dev()
    sizes = workloads.log_uniform_sizes(300, 0, 18, seed=23)
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    total = int(offs[-1])
    wsb = shuf.batched_async_workspace_bytes(len(sizes), total, 4)
    o = torch.tensor(np.asarray(offs, dtype=np.int64), device=dev)
    # eager reference: the permutation applied 1..4 times
    ref = to_dev(host)
    ws_e = torch.zeros(wsb, dtype=torch.uint8, device=dev)
    expect = []
    for _ in range(4):
        shuf.shuffle_batched_async(ref, o, 555, ws_e, total)
        torch.cuda.synchronize()
        expect.append(ref.clone())
    assert int(ws_e[:4].view(torch.int32).item()) == 0
    t = to_dev(host)
    ws = torch.zeros(wsb, dtype=torch.uint8, device=dev)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            shuf.shuffle_batched_async(t, o, 555, ws, total, stream=s)
    torch.cuda.synchronize()
    print("[gpu] captured; replaying", flush=True)
    # capture does not run the work: t is still the input
    assert torch.equal(t, to_dev(host))
    other = torch.arange(1 << 20, device=dev)
    for r in range(4):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(t, expect[r]), f"replay {r}"
        assert int(ws[:4].view(torch.int32).item()) == 0
        other = (other * 3 + 1) % 1000003  # eager work between replays
        torch.cuda.synchronize()


def test_async_device_errors_leave_data_untouched():
    shuf = _lib()
    w = 4
    mx = shuf.batched_async_max_elems(w)
    sizes = [1000, mx + 1, 50]
    host = workloads.identity(sum(sizes), w)
    offs = workloads.csr_offsets(np.array(sizes, dtype=np.uint64))
    t = to_dev(host)
    assert run_async(shuf, t, offs, 1) == 32  # an array above the limit
    assert np.array_equal(from_dev(t, host), host)
    sizes = [1000, 5000, 20000]
    host = workloads.identity(sum(sizes), w)
    offs = workloads.csr_offsets(np.array(sizes, dtype=np.uint64))
    t = to_dev(host)
    assert run_async(shuf, t, offs, 1, total=20000) == 32  # total bound too small
    assert np.array_equal(from_dev(t, host), host)
    o = torch.tensor(np.asarray(offs, dtype=np.int64), device=_dev())
    small = torch.zeros(1024, dtype=torch.uint8, device=_dev())
    with pytest.raises(shuf.ShuffleError) as ei:
        shuf.shuffle_batched_async(t, o, 1, small, int(offs[-1]))
    assert ei.value.code == shuf.SHUF_ENOMEM
