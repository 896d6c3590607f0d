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
