"""Both ways of computing the stable ranks give the oracle's permutation.

The kernels rank by LDS atomic adds where the device serves one wave's
same-address atomics in lane order (a probe checks it at the device's first
call), else by ballots.  The other GPU tests run whichever the device chose;
this file reports the choice and runs the ballot path against the oracle in a
process of its own (the choice is made once per process)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rank_method_reported_after_a_call():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_03317_amd as shuf

    host = workloads.identity(50000, 4)
    t = torch.from_numpy(host.view(np.int32).copy()).to("cuda:0")
    shuf.shuffle_inplace_ex(t, 9, 0, None)
    torch.cuda.synchronize()
    got = t.cpu().numpy().view(np.uint32)
    want = host.copy()
    oracle.shuffle(want, 9, oracle.default_params(50000, 4))
    assert np.array_equal(got, want)
    method = shuf.rank_method()
    print(f"[gpu] rank method on this device: {method} (1 = LDS atomics, 0 = ballots)", flush=True)
    assert method in (0, 1)


def test_ballot_ranks_match_oracle_in_own_process():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    env = dict(os.environ, IPSCSHUF_RANK="ballot")
    print("[gpu] running tests/gpu_ballot_check.py with IPSCSHUF_RANK=ballot", flush=True)
    out = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "gpu_ballot_check.py")],
                         env=env, capture_output=True, text=True, timeout=240)
    print(out.stdout, out.stderr[-2000:], flush=True)
    assert out.returncode == 0, out.stdout + out.stderr[-2000:]


def test_slot_search_matches_oracle_in_own_process():
    """The tile kernel's slot search (taken when a tile's free slots do not
    fit its list) forced for every tile, against the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    env = dict(os.environ, IPSCSHUF_SLOTS="search")
    print("[gpu] running tests/gpu_slot_search_check.py with IPSCSHUF_SLOTS=search", flush=True)
    out = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "gpu_slot_search_check.py")],
                         env=env, capture_output=True, text=True, timeout=240)
    print(out.stdout, out.stderr[-2000:], flush=True)
    assert out.returncode == 0, out.stdout + out.stderr[-2000:]


def test_many_small_random_cases_match_oracle():
    """120 small random cases (sizes, widths, parameters, seeds) that the
    library accepts, against the oracle: the ranks of every in-tile and tiled
    level, whichever way the device computes them, must keep the oracle's
    permutation.  Parameter sets whose LDS layout exceeds a CU are refused
    before any work (counted and printed) and replaced by further draws."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_03317_amd as shuf

    rng = np.random.default_rng(2302)
    unsupported = 0
    ran = 0
    for case in range(400):
        if ran == 120:
            break
        w = int(rng.choice([4, 8, 16]))
        n = int(rng.integers(2, 30000))
        kmax_log2 = int(rng.integers(1, 9))
        tmax = 65536 // w
        tile = int(rng.integers((1 << kmax_log2) + 1, tmax + 1))
        n0 = int(rng.integers(1, 129))
        p = oracle.Params(tile, kmax_log2, n0, 32)
        seed = int(rng.integers(0, 1 << 62))
        host = workloads.random_values(n, w, case)
        view = host.view(np.int32) if host.dtype == np.uint32 else host.view(np.int64)
        print(f"[gpu] case {case}: n={n} w={w} params={p} seed={seed}", flush=True)
        t = torch.from_numpy(view.copy()).to("cuda:0")
        try:
            shuf.shuffle_inplace_ex(t, seed, case, shuf.Params(p.tile, p.kmax_log2, p.n0, p.lmax))
        except shuf.ShuffleError as e:
            # a large tile with a tiny base case needs more LDS than a CU has:
            # refused before any work, as documented
            assert e.code == -4, e
            unsupported += 1
            continue
        torch.cuda.synchronize()
        got = t.cpu().numpy().view(host.dtype).reshape(host.shape)
        want = host.copy()
        oracle.shuffle(want, seed, p, stream_id=case)
        assert np.array_equal(got, want), f"case {case}"
        ran += 1
    print(f"[gpu] {ran} random cases matched the oracle; {unsupported} parameter sets refused "
          f"(LDS layout beyond one CU) before any work", flush=True)
    assert ran == 120, (ran, unsupported)
