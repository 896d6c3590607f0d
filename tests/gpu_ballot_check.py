"""Run by tests/test_gpu_rank_paths.py in a process of its own with
IPSCSHUF_RANK=ballot: the ballot ranks must give the oracle's permutation
too.  Prints the rank method and one line per checked case; exits non-zero on
a mismatch."""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2302_03317_amd as shuf  # noqa: E402
import workloads  # noqa: E402


def main() -> int:
    dev = torch.device("cuda:0")
    cases = [(1000, 4, 3), (100003, 8, 5), ((1 << 20) + 77, 4, 11), (300007, 16, 13),
             ((1 << 22) + 5, 4, 17)]
    for n, w, seed in cases:
        host = workloads.random_values(n, w, seed)
        view = host.view(np.int32) if host.dtype == np.uint32 else host.view(np.int64)
        t = torch.from_numpy(view.copy()).to(dev)
        shuf.shuffle_inplace_ex(t, seed, 0, None)
        torch.cuda.synchronize()
        got = t.cpu().numpy().view(host.dtype).reshape(host.shape)
        want = host.copy()
        oracle.shuffle(want, seed, oracle.default_params(n, w))
        ok = np.array_equal(got, want)
        print(f"n={n} w={w} seed={seed} rank_method={shuf.rank_method()} same={ok}", flush=True)
        if not ok:
            return 1
    return 0 if shuf.rank_method() == 0 else 2


if __name__ == "__main__":
    sys.exit(main())
