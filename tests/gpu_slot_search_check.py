"""Run by tests/test_gpu_rank_paths.py in a process of its own with
IPSCSHUF_SLOTS=search: the tile kernel then finds the slot of every staged
item by a search over the pieces' free slots instead of its free-slot list
(the path it takes when the free slots of a tile do not fit the list, which
random labels practically never produce).  The permutation must still be the
oracle's.  Prints one line per checked case; exits non-zero on a mismatch."""
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
    # sizes with one to three tiled levels for every width, ragged tails
    cases = [(100003, 8, 5, None), ((1 << 20) + 77, 4, 11, None), (300007, 16, 13, None),
             ((1 << 22) + 5, 4, 17, None), ((1 << 21) + 3, 8, 19, None),
             # small tiles and many buckets: short pieces, many staged items per tile
             (200001, 4, 23, (1024, 8, 16, 32)), (150001, 8, 29, (700, 7, 24, 32))]
    for n, w, seed, pp in cases:
        host = workloads.random_values(n, w, seed)
        view = host.view(np.int32) if host.dtype == np.uint32 else host.view(np.int64)
        t = torch.from_numpy(view.copy()).to(dev)
        if pp is None:
            shuf.shuffle_inplace_ex(t, seed, 0, None)
            p = oracle.default_params(n, w)
        else:
            shuf.shuffle_inplace_ex(t, seed, 0, shuf.Params(*pp))
            p = oracle.Params(*pp)
        torch.cuda.synchronize()
        got = t.cpu().numpy().view(host.dtype).reshape(host.shape)
        want = host.copy()
        oracle.shuffle(want, seed, p)
        ok = np.array_equal(got, want)
        print(f"n={n} w={w} seed={seed} params={pp} same={ok}", flush=True)
        if not ok:
            return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
