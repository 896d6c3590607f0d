"""The host PIpScShuf baseline (hostshuf/): valid, scheduling-independent,
uniform permutations.  It has no oracle of its own (its draws are the
paper's randomised ones, not the definition the GPU library follows), so it
is pinned by mathematics: permutation validity, equal output for every
thread count, and chi-square uniformity over all n! permutations and over
item positions, with settings small enough that RoughScatter, its parallel
merge, TwoSweep and the staged-item shuffle all run."""
import math

import numpy as np
import pytest

import hostshuf
import workloads

TINY = dict(kappa_small=1, kappa_large=1, base_case=1, par_cutoff=2)
SMALL = dict(kappa_small=2, kappa_large=3, base_case=4, par_cutoff=8)


def _perm_rank(a):
    rank = 0
    m = len(a)
    for i in range(m):
        smaller = sum(1 for j in range(i + 1, m) if a[j] < a[i])
        rank += smaller * math.factorial(m - 1 - i)
    return rank


@pytest.mark.parametrize("n,w", [(0, 4), (1, 4), (2, 8), (3, 4), (1000, 4), (300_001, 8), (100_003, 16),
                                 ((1 << 21) + 5, 4)])
def test_valid_permutation_any_thread_count(n, w):
    h = workloads.identity(n, w)
    a = hostshuf.shuffle(h.copy(), 7, threads=1)
    b = hostshuf.shuffle(h.copy(), 7, threads=4)
    assert np.array_equal(a, b)
    key = a if w != 16 else a[:, 0]
    assert np.array_equal(np.sort(key.astype(np.uint64)), np.arange(n, dtype=np.uint64))
    if w == 16:  # records stay whole
        assert np.array_equal(a[:, 1], workloads.splitmix64(a[:, 0]))
    if n > 1000:
        assert not np.array_equal(a, h)
        assert not np.array_equal(a, hostshuf.shuffle(h.copy(), 8, threads=4))


def test_small_settings_valid_and_deterministic():
    for n in [2, 3, 5, 8, 17, 100, 1000, 4097]:
        for params in (TINY, SMALL):
            h = np.arange(n, dtype=np.uint32)
            a = hostshuf.shuffle(h.copy(), n, threads=1, **params)
            b = hostshuf.shuffle(h.copy(), n, threads=3, **params)
            assert np.array_equal(a, b)
            assert np.array_equal(np.sort(a), h)


@pytest.mark.parametrize("params", [TINY, SMALL])
def test_chi_square_all_permutations(params):
    from scipy import stats

    seeds = 60_000
    for n in range(3, 7):
        counts = np.zeros(math.factorial(n))
        for s in range(seeds):
            a = hostshuf.shuffle(np.arange(n, dtype=np.uint32), 1_000_003 * n + s, threads=1, **params)
            counts[_perm_rank(a.tolist())] += 1
        assert stats.chisquare(counts).pvalue > 1e-5, (n, params)


def test_position_frequencies():
    from scipy import stats

    n, seeds = 64, 6000
    c = np.zeros((n, n))
    for s in range(seeds):
        a = hostshuf.shuffle(np.arange(n, dtype=np.uint32), s, threads=1, **SMALL)
        c[a, np.arange(n)] += 1
    pvals = [stats.chisquare(row).pvalue for row in c]
    assert stats.kstest(pvals, "uniform").pvalue > 1e-4


def test_fisher_yates_baseline_uniform():
    from scipy import stats

    n, seeds = 5, 60_000
    counts = np.zeros(math.factorial(n))
    for s in range(seeds):
        a = hostshuf.fisher_yates(np.arange(n, dtype=np.uint32), s)
        counts[_perm_rank(a.tolist())] += 1
    assert stats.chisquare(counts).pvalue > 1e-5
