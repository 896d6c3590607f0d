"""GPU parity: the HIP library (through its C ABI) against the CPU oracle,
element by element, on the same seeded inputs.  Integer work: bit-exact."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    import paper_2302_03317_amd as shuf

    shuf.lib()
    return shuf


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(host: np.ndarray):
    view = host.view(np.int32) if host.dtype == np.uint32 else host.view(np.int64)
    return torch.from_numpy(view.copy()).to(_dev())


def from_dev(t, like: np.ndarray) -> np.ndarray:
    return t.cpu().numpy().view(like.dtype).reshape(like.shape)


def gpu_shuffle(host, seed, params=None, stream_id=0):
    shuf = _lib()
    n = host.shape[0]
    w = host.itemsize * (host.shape[1] if host.ndim > 1 else 1)
    print(f"[gpu] n={n} w={w} seed={seed} stream={stream_id} params={params}", flush=True)
    t = to_dev(host)
    p = None if params is None else shuf.Params(params.tile, params.kmax_log2, params.n0, params.lmax)
    shuf.shuffle_inplace_ex(t, seed, stream_id, p)
    torch.cuda.synchronize()
    return from_dev(t, host)


def oracle_shuffle(host, seed, params, stream_id=0):
    out = host.copy()
    oracle.shuffle(out, seed, params, stream_id=stream_id)
    return out


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.nonzero((got != want).reshape(got.shape[0], -1).any(axis=1))[0]
        raise AssertionError(f"{what}: {bad.size} rows differ, first at {bad[:8].tolist()}")


TINY = [
    oracle.Params(3, 1, 1, 4),
    oracle.Params(4, 1, 2, 5),
    oracle.Params(5, 2, 1, 3),
    oracle.Params(9, 3, 1, 2),
    oracle.Params(40, 3, 4, 32),
    oracle.Params(64, 4, 8, 6),
    oracle.Params(300, 5, 16, 32),
    oracle.Params(1000, 8, 64, 32),
    oracle.Params(4096, 8, 1, 3),
]


@pytest.mark.parametrize("p", TINY)
def test_tiny_parameters_sweep(p):
    """Tiny tiles force many tiles, movers, displaced items, in-LDS levels,
    the recursion cap and the sequential fallback at small n."""
    rng = np.random.default_rng(p.tile)
    for n in [0, 1, 2, 3, 5, 17, 64, 100, 257, 1000, 3001]:
        for w in (4, 8, 16):
            if p.tile * w > 65536:
                continue
            seed = int(rng.integers(0, 2**63))
            host = workloads.identity(n, w)
            assert_same(gpu_shuffle(host, seed, p), oracle_shuffle(host, seed, p), f"n={n} w={w} {p}")


def test_config_small_u32_seed42():
    """2^20 uint32 identity, seed 42, default parameters."""
    n, w = 1 << 20, 4
    host = workloads.identity(n, w)
    p = oracle.default_params(n, w)
    assert_same(gpu_shuffle(host, 42, p), oracle_shuffle(host, 42, p), "2^20 u32")


@pytest.mark.parametrize("n,w", [(100_003, 4), (1 << 22, 4), (3_000_017, 8), (1 << 21, 16), (777_777, 16)])
def test_default_params_widths(n, w):
    host = workloads.identity(n, w)
    p = oracle.default_params(n, w)
    seed = 0x9E3779B97F4A7C15 ^ n
    assert_same(gpu_shuffle(host, seed, p), oracle_shuffle(host, seed, p), f"n={n} w={w}")


@pytest.mark.parametrize(
    "n,w,p",
    [
        (1_000_000, 4, oracle.Params(1024, 5, 16, 32)),
        (600_000, 8, oracle.Params(777, 4, 10, 32)),
        (300_000, 16, oracle.Params(2000, 8, 64, 32)),
        (2_000_000, 4, oracle.Params(16384, 8, 64, 32)),
        (500_000, 4, oracle.Params(300, 2, 5, 32)),
    ],
)
def test_multi_level_small_tiles(n, w, p):
    """Several tiled levels with many movers per level."""
    host = workloads.identity(n, w)
    assert_same(gpu_shuffle(host, 12345, p), oracle_shuffle(host, 12345, p), f"n={n} w={w} {p}")


def test_stream_ids_and_seeds():
    n, w = 200_000, 4
    host = workloads.identity(n, w)
    p = oracle.default_params(n, w)
    for seed, sid in [(1, 0), (1, 1), (2**64 - 1, 7), (0, 2**32 - 1)]:
        assert_same(gpu_shuffle(host, seed, p, sid), oracle_shuffle(host, seed, p, sid), f"seed={seed} sid={sid}")


def test_data_independence_on_gpu():
    n, w = 300_000, 8
    ident = workloads.identity(n, w)
    vals = workloads.random_values(n, w, 5)
    p = oracle.default_params(n, w)
    perm = gpu_shuffle(ident, 99, p)
    out = gpu_shuffle(vals, 99, p)
    assert np.array_equal(out, vals[perm.astype(np.int64)])


def test_determinism_and_other_stream():
    shuf = _lib()
    n, w = 1 << 20, 4
    host = workloads.identity(n, w)
    a = gpu_shuffle(host, 5, None)
    t = to_dev(host)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        shuf.shuffle_inplace(t, 5, stream=s)
    s.synchronize()
    assert np.array_equal(from_dev(t, host), a)
    assert np.array_equal(gpu_shuffle(host, 5, None), a)


def test_batched_matches_single_arrays():
    shuf = _lib()
    sizes = workloads.log_uniform_sizes(300, 0, 15, seed=3)
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    t = to_dev(host)
    print(f"[gpu] batched arrays={len(sizes)} total={host.size}", flush=True)
    shuf.shuffle_batched(t, offs, 777)
    torch.cuda.synchronize()
    got = from_dev(t, host)
    for j in range(len(sizes)):
        a, b = int(offs[j]), int(offs[j + 1])
        want = oracle_shuffle(host[a:b], 777, oracle.default_params(b - a, 4), stream_id=j)
        assert_same(got[a:b], want, f"batched array {j} (n={b - a})")


def test_stats_report_tiled_levels():
    shuf = _lib()
    host = workloads.identity(1 << 21, 4)
    gpu_shuffle(host, 1, None)
    st = shuf.last_stats()
    assert st["tiled_levels"] == 1
    assert st["movers"] > 0 and st["leaves"] > 0


def test_argument_errors_leave_data_untouched():
    import ctypes

    shuf = _lib()
    host = workloads.identity(1000, 4)
    t = to_dev(host)
    ptr = ctypes.c_void_p(t.data_ptr())
    P = shuf._Params
    good = P(32768, 8, 64, 32)
    null = ctypes.c_void_p(0)
    cases = [
        ("shuffle_inplace", (null, 1000, 4, 1, null), shuf.SHUF_EINVAL),
        ("shuffle_inplace", (ptr, 1000, 3, 1, null), shuf.SHUF_EINVAL),
        ("shuffle_inplace", (ctypes.c_void_p(t.data_ptr() + 2), 999, 4, 1, null), shuf.SHUF_EINVAL),
        ("shuffle_inplace", (ptr, 1 << 41, 4, 1, null), shuf.SHUF_EUNSUPPORTED),
        ("shuffle_inplace_ex", (ptr, 1000, 4, 1, 0, None, null), shuf.SHUF_EINVAL),
        ("shuffle_inplace_ex", (ptr, 1000, 4, 1, 0, ctypes.byref(P(3, 2, 1, 1)), null), shuf.SHUF_EINVAL),
        ("shuffle_inplace_ex", (ptr, 1000, 4, 1, 0, ctypes.byref(P(32768, 9, 1, 1)), null), shuf.SHUF_EINVAL),
        ("shuffle_inplace_ex", (ptr, 1000, 4, 1, 0, ctypes.byref(P(32768, 8, 0, 1)), null), shuf.SHUF_EINVAL),
        ("shuffle_inplace_ex", (ptr, 1000, 4, 1, 0, ctypes.byref(P(32768, 8, 64, 256)), null), shuf.SHUF_EINVAL),
        ("shuffle_inplace_ex", (ptr, 1000, 4, 1, 0, ctypes.byref(P(40000, 8, 64, 32)), null), shuf.SHUF_EUNSUPPORTED),
        ("shuffle_inplace_ex", (ptr, 1000, 4, 1, 0, ctypes.byref(P(32768, 8, 1, 32)), null), shuf.SHUF_EUNSUPPORTED),
    ]
    for name, args, code in cases:
        print(f"[gpu] error case {name} -> {code}", flush=True)
        assert shuf.raw_call(name, *args) == code
    offs = (ctypes.c_uint64 * 3)(0, 600, 500)
    assert shuf.raw_call("shuffle_batched", ptr, offs, 2, 4, 1, null) == shuf.SHUF_EINVAL
    assert shuf.raw_call("shuffle_batched", ptr, None, 2, 4, 1, null) == shuf.SHUF_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(t, host), host)
    # n <= 1 is a successful no-op, even with a NULL pointer
    assert shuf.raw_call("shuffle_inplace", null, 1, 4, 1, null) == 0
    assert shuf.raw_call("shuffle_inplace", null, 0, 8, 1, null) == 0


def test_many_arrays_in_separate_allocations():
    """shuffle_many: arrays anywhere in device memory, each with its own seed
    and stream id, equal the single-array definition."""
    shuf = _lib()
    rng = np.random.default_rng(11)
    sizes = [0, 1, 2, 63, 64, 65, 1000, 16127, 16128, 16129, 40000, 300000]
    for w in (4, 8, 16):
        hosts = [workloads.random_values(n, w, 100 + i) for i, n in enumerate(sizes)]
        seeds = [int(rng.integers(0, 2**63)) for _ in sizes]
        sids = [int(rng.integers(0, 2**32)) for _ in sizes]
        tens = [to_dev(h) for h in hosts]
        print(f"[gpu] shuffle_many w={w} arrays={len(sizes)}", flush=True)
        shuf.shuffle_many(tens, seeds, sids)
        torch.cuda.synchronize()
        for h, t, sd, sid in zip(hosts, tens, seeds, sids):
            want = oracle_shuffle(h, sd, oracle.default_params(h.shape[0], w), stream_id=sid)
            assert_same(from_dev(t, h), want, f"many w={w} n={h.shape[0]}")


def test_batched_equals_many():
    shuf = _lib()
    sizes = workloads.log_uniform_sizes(200, 4, 18, seed=9)
    offs = workloads.csr_offsets(sizes)
    host = workloads.batched_identity(sizes)
    a = to_dev(host)
    print(f"[gpu] batched vs many: arrays={len(sizes)} total={host.size}", flush=True)
    shuf.shuffle_batched(a, offs, 4242)
    b = to_dev(host)
    views = [b[int(offs[j]):int(offs[j + 1])] for j in range(len(sizes))]
    shuf.shuffle_many(views, [4242] * len(sizes), list(range(len(sizes))))
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(a, host), from_dev(b, host))


@pytest.mark.parametrize("w", [4, 8, 16])
def test_batched_edge_sizes_all_widths(w):
    """Empty arrays, single items, the largest array that skips the tiled
    levels (T - KMAX) and the smallest that takes one (T - KMAX + 1), and
    arrays of several tiles with a ragged end, packed in one batch."""
    shuf = _lib()
    T = 65536 // w
    sizes = [0, 1, 2, 0, 3, 64, 65, T - 256, T - 255, 2 * T + 7, 1, 0, 3 * T + 1]
    parts = [workloads.identity(s, w) for s in sizes]
    host = np.concatenate(parts, axis=0)
    offs = workloads.csr_offsets(np.array(sizes, dtype=np.uint64))
    print(f"[gpu] batched edge sizes w={w} arrays={len(sizes)} total={host.shape[0]}", flush=True)
    t = to_dev(host)
    shuf.shuffle_batched(t, offs, 31337)
    torch.cuda.synchronize()
    got = from_dev(t, host)
    for j, s in enumerate(sizes):
        a, b = int(offs[j]), int(offs[j + 1])
        want = host[a:b] if s < 2 else oracle_shuffle(host[a:b], 31337, oracle.default_params(s, w), stream_id=j)
        assert_same(got[a:b], want, f"batched w={w} array {j} (n={s})")


def test_session_result_same_alone_and_in_mix():
    """Continuous batching: requests join while others are in flight; every
    result equals the same request run alone (the oracle, and the GPU
    single-array call)."""
    shuf = _lib()
    w = 8
    rng = np.random.default_rng(5)
    plan = []  # (step at which it is submitted, n)
    for step in range(6):
        for _ in range(3):
            plan.append((step, int(2 ** rng.uniform(10, 21))))
    plan.append((0, 1))
    plan.append((2, 0))
    reqs = []
    with shuf.Session(w) as sess:
        step = 0
        pending = list(plan)
        done = set()
        while pending or sess.inflight()[0]:
            for item in [p for p in pending if p[0] == step]:
                n = item[1]
                h = workloads.random_values(n, w, 1000 + len(reqs))
                t = to_dev(h)
                seed = int(rng.integers(0, 2**64, dtype=np.uint64))
                sid = int(rng.integers(0, 2**32))
                tk = sess.submit(t, seed, sid)
                reqs.append((tk, h, t, seed, sid, step))
                pending.remove(item)
            print(f"[gpu] session step {step} inflight={sess.inflight()}", flush=True)
            done.update(sess.step())
            step += 1
            assert step < 100
        torch.cuda.synchronize()
    assert done == {r[0] for r in reqs}
    for tk, h, t, seed, sid, st in reqs:
        want = oracle_shuffle(h, seed, oracle.default_params(h.shape[0], w), stream_id=sid)
        assert_same(from_dev(t, h), want, f"session request {tk} n={h.shape[0]} submitted at step {st}")
        alone = to_dev(h)
        shuf.shuffle_inplace_ex(alone, seed, sid)
        torch.cuda.synchronize()
        assert_same(from_dev(alone, h), want, f"alone {tk}")


def test_full_size_u32_2e28_equals_oracle():
    """The width-sweep size, default parameters, element by element against
    the oracle (about 20 s of single-core CPU work)."""
    n, w = 1 << 28, 4
    seed = 0xC0FFEE1234567
    host = workloads.identity(n, w)
    print(f"[gpu] full size n=2^28 u32 seed={seed}", flush=True)
    got = gpu_shuffle(host, seed, None)
    want = oracle_shuffle(host, seed, oracle.default_params(n, w))
    assert_same(got, want, "2^28 u32")


def _is_identity_permutation(t, n):
    """Every value 0..n-1 occurs exactly once in t (checked in chunks)."""
    seen = torch.zeros(n, dtype=torch.uint8, device=t.device)
    flat = t.view(-1) if t.dim() == 1 else t[:, 0]
    chunk = 1 << 27
    for a in range(0, n, chunk):
        idx = flat[a:a + chunk].to(torch.int64)
        if t.dtype == torch.int32:
            idx = idx & 0xFFFFFFFF
        if bool(((idx < 0) | (idx >= n)).any()):
            return False
        seen.index_fill_(0, idx, 1)
        del idx
    return bool(seen.all())


@pytest.mark.parametrize("log2n,w,extra", [(32, 4, 0), (31, 8, 0), (32, 8, 12345)])
def test_full_size_properties(log2n, w, extra):
    """The single-array headline sizes in the benchmark's launch
    configuration: the output is a permutation of the input, a rerun with
    the same seed gives the same bytes, another stream id does not, and the
    number of fixed points is small (Poisson(1) for a uniform permutation).
    2^32 + 12345 u64 items (32 GiB) take the 64-bit paths of the piece
    arithmetic (tile x remainder beyond 32 bits) at a ragged size."""
    shuf = _lib()
    dev = _dev()
    n = (1 << log2n) + extra
    dt = torch.int32 if w == 4 else torch.int64
    print(f"[gpu] full size properties n=2^{log2n}+{extra} w={w}", flush=True)
    a = torch.empty(n, dtype=dt, device=dev)
    chunk = 1 << 27
    for s in range(0, n, chunk):
        a[s:s + chunk] = torch.arange(s, min(n, s + chunk), device=dev, dtype=torch.int64).to(dt)
    b = a.clone()
    seed = 0x5151AB
    shuf.shuffle_inplace(a, seed)
    shuf.shuffle_inplace(b, seed)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    fixed = 0
    for s in range(0, n, chunk):
        ar = torch.arange(s, min(n, s + chunk), device=dev, dtype=torch.int64)
        v = a[s:s + chunk].to(torch.int64)
        if dt == torch.int32:
            v = v & 0xFFFFFFFF
        fixed += int((v == ar).sum())
    assert fixed < 20, fixed
    assert _is_identity_permutation(a, n)
    del b
    c = torch.empty_like(a)
    for s in range(0, n, chunk):
        c[s:s + chunk] = torch.arange(s, min(n, s + chunk), device=dev, dtype=torch.int64).to(dt)
    shuf.shuffle_inplace_ex(c, seed, 1)
    torch.cuda.synchronize()
    assert not torch.equal(a, c)


@pytest.mark.parametrize(
    "n,w,p",
    [
        (3_000_017, 4, None),
        (1_000_000, 8, None),
        (400_000, 16, None),
        (500_000, 4, oracle.Params(300, 2, 5, 32)),
        (10_000, 4, None),
    ],
)
def test_caller_workspace_is_exact_and_sufficient(n, w, p):
    """shuffle_workspace_bytes is exact: the caller-workspace shuffle succeeds
    with that many bytes (and equals the oracle), and fails with SHUF_ENOMEM
    with one byte less."""
    shuf = _lib()
    host = workloads.identity(n, w)
    params = p if p is not None else oracle.default_params(n, w)
    sp = shuf.Params(params.tile, params.kmax_log2, params.n0, params.lmax)
    seed, sid = 0xABCDEF ^ n, 3
    need = shuf.workspace_bytes(n, w, seed, sid, sp)
    print(f"[gpu] workspace n={n} w={w} params={params} bytes={need}", flush=True)
    assert need > 0
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=_dev())
    t = to_dev(host)
    shuf.shuffle_inplace_ws(t, seed, ws, sid, sp)
    torch.cuda.synchronize()
    assert_same(from_dev(t, host), oracle_shuffle(host, seed, params, stream_id=sid), f"ws n={n} w={w}")
    small = ws[: need - 1]
    t2 = to_dev(host)
    with pytest.raises(shuf.ShuffleError) as ei:
        shuf.shuffle_inplace_ws(t2, seed, small, sid, sp)
    assert ei.value.code == shuf.SHUF_ENOMEM
    torch.cuda.synchronize()


@pytest.mark.parametrize("w", [8, 16])
def test_full_size_2e28_wider_elements_equal_oracle(w):
    """The width sweep at n = 2^28: u64 and 16-byte records (key = i,
    payload = splitmix64(i)) element by element against the oracle."""
    n = 1 << 28
    seed = 0xDEC0DE ^ w
    host = workloads.identity(n, w)
    print(f"[gpu] full size n=2^28 w={w} seed={seed}", flush=True)
    got = gpu_shuffle(host, seed, None)
    want = oracle_shuffle(host, seed, oracle.default_params(n, w))
    assert_same(got, want, f"2^28 w={w}")
    if w == 16:  # no torn records: every payload still matches its key
        assert np.array_equal(got[:, 1], workloads.splitmix64(got[:, 0]))


def test_movers_fraction_matches_overflow_statistic():
    """One tiled level (n just below 2^21 u32: k = 256 buckets, c = T/k = 64
    items per piece).  The movers are the overflow items (simulated fraction
    0.40 / sqrt(c) = 5 %) plus the placed items displaced by the shift from
    equal to exact region boundaries; the shift at boundary b is a random
    walk of b steps with variance n/k each, so the displaced items number at
    most about sum_b sqrt(2 b n / (pi k)) = 0.53 k sqrt(n), 9 % here."""
    shuf = _lib()
    n = (1 << 21) - 12345
    host = workloads.identity(n, 4)
    gpu_shuffle(host, 2024, None)
    st = shuf.last_stats()
    assert st["tiled_levels"] == 1
    frac = st["movers"] / n
    assert 0.05 < frac < 0.14, frac


def test_concurrent_host_threads_and_streams():
    """Two host threads shuffle different arrays on two streams at the same
    time; each result equals the same call made alone."""
    import threading

    shuf = _lib()
    dev = _dev()
    hosts = [workloads.random_values(3_000_000, 4, 41), workloads.random_values(2_500_000, 4, 42)]
    tens = [to_dev(h) for h in hosts]
    streams = [torch.cuda.Stream(device=dev) for _ in hosts]
    errors = []

    def work(i):
        try:
            with torch.cuda.device(dev):
                for _ in range(3):
                    shuf.shuffle_inplace_ex(tens[i], 900 + i, i, stream=streams[i])
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    # three applications of the same permutation: compare with applying it thrice alone
    thr = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for x in thr:
        x.start()
    for x in thr:
        x.join()
    torch.cuda.synchronize()
    assert not errors
    for i, h in enumerate(hosts):
        t = to_dev(h)
        for _ in range(3):
            shuf.shuffle_inplace_ex(t, 900 + i, i)
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(tens[i], h), from_dev(t, h))


def test_session_budget_queues_requests_and_matches_oracle():
    """Admission by memory budget: with room for about two of the requests
    (data plus the library's workspace for each), later requests wait in the
    session's queue, the admitted charges never exceed the budget, a request
    larger than the budget is refused, and every result equals the oracle."""
    shuf = _lib()
    w = 8
    rng = np.random.default_rng(77)
    sizes = [1 << 20, 3 << 19, 1 << 20, 700_001, 1 << 20, 50_000, 1, 0, 300_000]
    reqs = []
    for i, n in enumerate(sizes):
        h = workloads.random_values(n, w, 500 + i)
        reqs.append((h, int(rng.integers(0, 2**63)), i))
    p = shuf.default_params(1 << 20, w)
    charges = [h.shape[0] * w + (shuf.workspace_bytes(h.shape[0], w, sd, sid, p) if h.shape[0] > 1 else 0)
               for h, sd, sid in reqs]
    budget = 2 * max(charges) + 4096
    print(f"[gpu] session budget {budget} charges {charges}", flush=True)
    with shuf.Session(w) as sess:
        sess.set_budget(budget)
        big = torch.empty(budget // w + 1, dtype=torch.int64, device=_dev())
        with pytest.raises(shuf.ShuffleError) as ei:
            sess.submit(big, 1, 0)
        assert ei.value.code == shuf.SHUF_ENOMEM
        del big
        tens = []
        for h, sd, sid in reqs:
            t = to_dev(h)
            tens.append(t)
            sess.submit(t, sd, sid)
        saw_queue = False
        steps = 0
        while sess.inflight()[0]:
            queued, used = sess.queued()
            assert used <= budget
            saw_queue = saw_queue or queued > 0
            sess.step()
            steps += 1
            assert steps < 200
        torch.cuda.synchronize()
        assert saw_queue
        assert sess.queued() == (0, 0)
    for (h, sd, sid), t in zip(reqs, tens):
        want = oracle_shuffle(h, sd, oracle.default_params(h.shape[0], w), stream_id=sid)
        assert_same(from_dev(t, h), want, f"budgeted session request n={h.shape[0]}")


@pytest.mark.parametrize("w", [4, 8, 16])
def test_session_cheap_workspace_bound_covers_exact(w):
    """The session's admission bound that needs no GPU work (n w + 24 n +
    16 KiB of workspace) is at least the exact workspace of a request."""
    shuf = _lib()
    T = 65536 // w
    for n in [T - 255, T + 1000, 5 * T + 17, 1 << 20, (3 << 21) + 5, (1 << 24) + 7]:
        for sd, sid in [(1, 0), (2**64 - 1, 7)]:
            exact = shuf.workspace_bytes(n, w, sd, sid)
            print(f"[gpu] workspace n={n} w={w}: exact {exact} bound {n * w + 24 * n + 16384}", flush=True)
            assert exact <= n * w + 24 * n + 16384, (n, w, exact)
