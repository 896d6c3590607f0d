"""The allocation-free entry point (shuffle_inplace_noalloc) against the
allocating one (shuffle_inplace_ex) through the C ABI: same bytes out, on two
calls in a row -- the second with a smaller input -- for every width, plus a
small case against the oracle and the size limit."""
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


def to_dev(host):
    view = host.view(np.int32) if host.dtype == np.uint32 else host.view(np.int64)
    return torch.from_numpy(view.copy()).to(_dev())


def from_dev(t, like):
    return t.cpu().numpy().view(like.dtype).reshape(like.shape)


@pytest.mark.parametrize("w", [4, 8, 16])
def test_noalloc_equals_allocating_entry_two_calls(w):
    shuf = _lib()
    # a first call with several tiled levels, then a smaller one (one tiled
    # level and a ragged end), each compared with shuffle_inplace_ex
    sizes = {4: [(6 << 20) + 13, 300_001], 8: [(3 << 20) + 7, 100_003], 16: [(1 << 20) + 5, 40_001]}[w]
    for call, n in enumerate(sizes):
        host = workloads.random_values(n, w, 70 + call)
        seed, sid = 0x5EED0000 + 17 * call + w, call + 2
        print(f"[gpu] noalloc call {call}: n={n} w={w} seed={seed:#x} sid={sid}", flush=True)
        a = to_dev(host)
        shuf.shuffle_inplace_noalloc(a, seed, sid)
        b = to_dev(host)
        shuf.shuffle_inplace_ex(b, seed, sid)
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"call {call} n={n} w={w}"


def test_noalloc_small_params_and_oracle():
    """Tiny parameters (many tiles, movers, the recursion cap) and a small
    default case, against the oracle."""
    shuf = _lib()
    cases = [(50_000, 4, oracle.Params(300, 2, 5, 32)), (20_000, 8, oracle.Params(1000, 8, 64, 32)),
             (5_000, 16, oracle.Params(9, 3, 1, 2)), (100_000, 4, None), (16_000, 4, None)]
    for n, w, p in cases:
        host = workloads.random_values(n, w, n)
        params = p if p is not None else oracle.default_params(n, w)
        sp = shuf.Params(params.tile, params.kmax_log2, params.n0, params.lmax)
        print(f"[gpu] noalloc vs oracle n={n} w={w} params={params}", flush=True)
        t = to_dev(host)
        shuf.shuffle_inplace_noalloc(t, 4321, 9, sp)
        torch.cuda.synchronize()
        want = host.copy()
        oracle.shuffle(want, 4321, params, stream_id=9)
        assert np.array_equal(from_dev(t, host), want), (n, w, params)


def test_noalloc_rejects_oversize_untouched():
    shuf = _lib()
    n = (48 << 20) // 4 + 1
    t = torch.arange(n, dtype=torch.int32, device=_dev())
    with pytest.raises(shuf.ShuffleError) as ei:
        shuf.shuffle_inplace_noalloc(t, 1)
    assert ei.value.code == shuf.SHUF_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.equal(t, torch.arange(n, dtype=torch.int32, device=t.device))
