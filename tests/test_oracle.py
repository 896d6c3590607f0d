"""Pins for the CPU oracle: each test checks it against something other than
itself -- an installed third-party implementation, a closed form, a textbook
routine, exact enumeration, hand-worked examples or statistics.

Paper: arXiv 2302.03317 (Penschuck).  The oracle is test infrastructure.
"""
import ctypes
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
from oracle import spec
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
TINY = [  # (tile, kmax_log2, n0, lmax): tiny parameters that force tiles, movers and routing
    oracle.Params(3, 1, 1, 4),
    oracle.Params(4, 1, 2, 5),
    oracle.Params(5, 2, 1, 3),
    oracle.Params(3, 1, 1, 3),
]


# ---------------------------------------------------------------- Philox ---
def _rocrand_ref():
    path = os.path.join(HERE, "philox_ref", "librocrand_philox_ref.so")
    if not os.path.exists(path):
        pytest.skip("rocRAND host helper not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    lib.rocrand_philox_block.argtypes = [ctypes.c_void_p] * 3
    return lib


def test_philox_matches_rocrand():
    """Philox4x32-10 vs rocRAND's own engine (installed header, host build)."""
    lib = _rocrand_ref()
    rng = random.Random(1)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)]
    cases += [([rng.getrandbits(32) for _ in range(4)], [rng.getrandbits(32) for _ in range(2)]) for _ in range(5000)]
    for ctr, key in cases:
        c = (ctypes.c_uint32 * 4)(*ctr)
        k = (ctypes.c_uint32 * 2)(*key)
        o = (ctypes.c_uint32 * 4)()
        lib.rocrand_philox_block(c, k, o)
        assert tuple(o) == oracle.philox4x32_10(ctr, key), (ctr, key)


def test_philox_c_matches_python_spec():
    rng = random.Random(2)
    for _ in range(500):
        ctr = [rng.getrandbits(32) for _ in range(4)]
        key = [rng.getrandbits(32) for _ in range(2)]
        assert oracle.philox4x32_10(ctr, key) == spec.philox4x32_10(ctr, key)


def test_philox_bijective_on_counter_word():
    """For a fixed key the block function is a bijection on counters: no two
    of many distinct counters may collide."""
    seen = set()
    for c in range(20000):
        seen.add(oracle.philox4x32_10([c, 0, 7, 3], [11, 13]))
    assert len(seen) == 20000


# ---------------------------------------------------------------- labels ---
def test_label_layout():
    """Label = top kappa bits of byte (pos mod 16) of block pos >> 4."""
    seed, stream, level = 0x0123456789ABCDEF, 5, 3
    for pos in [0, 1, 15, 16, 17, 1 << 33, (1 << 40) + 7]:
        words = oracle.philox4x32_10(
            [(pos >> 4) & 0xFFFFFFFF, pos >> 36, level | (1 << 8), stream],
            [seed & 0xFFFFFFFF, seed >> 32])
        byte = (words[(pos & 15) >> 2] >> (8 * (pos & 3))) & 0xFF
        for kap in range(1, 9):
            assert oracle.label(seed, stream, level, pos, kap) == byte >> (8 - kap)


def test_label_counts_chi_square():
    """Labels over many positions are uniform (chi-square, 255 dof)."""
    from scipy import stats

    counts = np.zeros(256)
    for pos in range(0, 200000):
        counts[oracle.label(99, 0, 0, pos, 8)] += 1
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4


# ---------------------------------------------------------------- Lemire ---
@pytest.mark.slow
def test_lemire_exhaustive_counts():
    """Every result in [0, s) is accepted for exactly floor(2^32 / s) words
    (enumerating all 2^32 words)."""
    s = 6
    h = oracle.lemire_histogram(s)
    assert np.all(h == (1 << 32) // s)


def test_lemire16_exhaustive_counts():
    """16-bit rule: for every bound up to 2^16 tried, every result in [0, s)
    is accepted for exactly floor(2^16 / s) of the 2^16 words."""
    for s in [1, 2, 3, 5, 6, 7, 10, 21, 63, 64, 100, 1000, 4097, 32768, 40000, 65535, 65536]:
        h = oracle.lemire16_histogram(s)
        assert np.all(h == (1 << 16) // s), s


def test_lemire_threshold_closed_form():
    rng = random.Random(3)
    for s in [1, 2, 3, 7, 1000, 65537, (1 << 31) + 1, (1 << 32) - 1, 1 << 32]:
        t = (1 << 32) % s
        for _ in range(200):
            x = rng.getrandbits(32)
            r = oracle.lemire_step(x, s)
            lo, hi = (x * s) & 0xFFFFFFFF, (x * s) >> 32
            assert r == (hi if lo >= t else None)
            if r is not None:
                assert 0 <= r < s


def test_draw_in_range_and_retry_counter():
    for s in [2, 3, 5, 64, 1000]:
        for pos in range(200):
            assert 0 <= oracle.draw(5, 1, 2, pos, s) < s
    # the draw must equal the spec's attempt-by-attempt rendition, on both
    # sides of the 16-bit / 32-bit switch and for bounds with many rejections
    src = spec.PhiloxSource(77, 4)
    for pos in range(300):
        for s in [3, 40000, 65535, 65536, 65537, (1 << 31) + 1, (1 << 32) - 1]:
            assert oracle.draw(77, 4, 9, pos, s) == src.draw(9, pos, s)


def test_draw_word_layout():
    """Short draws read 16-bit half-words of block pos >> 3, low half first;
    long draws read 32-bit words of block pos >> 2."""
    seed, stream, level = 1234567, 3, 5
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for pos in [0, 1, 7, 8, 13, 1 << 35]:
        words = oracle.philox4x32_10([(pos >> 3) & 0xFFFFFFFF, pos >> 35, level | (3 << 8), stream], key)
        x = (words[(pos & 7) >> 1] >> (16 * (pos & 1))) & 0xFFFF
        for s in [2, 6, 64]:
            if ((x * s) & 0xFFFF) >= (1 << 16) % s:
                assert oracle.draw(seed, stream, level, pos, s) == (x * s) >> 16
        words = oracle.philox4x32_10([(pos >> 2) & 0xFFFFFFFF, pos >> 34, level | (2 << 8), stream], key)
        s = (1 << 20) + 3
        if ((words[pos & 3] * s) & 0xFFFFFFFF) >= (1 << 32) % s:
            assert oracle.draw(seed, stream, level, pos, s) == (words[pos & 3] * s) >> 32


# ------------------------------------------------------------ kappa rule ---
def test_kappa_schedule_examples():
    """Worked shapes: 2^32 u32 with a 32768-element tile takes three tiled
    levels of kappa 6 and leaves of about 2^14."""
    p = oracle.Params(32768)
    assert oracle.kappa(1 << 32, True, p) == 6
    assert oracle.kappa(1 << 26, True, p) == 6
    assert oracle.kappa(1 << 20, True, p) == 6
    assert oracle.kappa(1 << 14, False, p) == 5
    assert oracle.kappa(512, False, p) == 4
    for m in [2, 3, 100, 10**6, 1 << 36]:
        for hbm in (True, False):
            k = oracle.kappa(m, hbm, p)
            assert 1 <= k <= 8
            assert k == spec.kappa_for(m, hbm, p.tile, p.kmax_log2, p.n0)


# ------------------------------------------------------------- one level ---
@pytest.mark.parametrize("name", ["level_tiled_k2.json", "level_tiled_k4_empty_tiles.json"])
def test_level_hand_worked(name):
    g = json.load(open(os.path.join(HERE, "golden", name)))
    d = oracle.level_dest(g["labels"], g["kappa"], g["tile"], g["hbm_regime"])
    assert list(d) == g["dest"]


def test_level_exact_is_stable_counting_sort():
    """Untiled level = stable sort by label (numpy's stable argsort)."""
    rng = np.random.default_rng(4)
    for m in [1, 2, 17, 1000, 5000]:
        for kap in [1, 3, 8]:
            lab = rng.integers(0, 1 << kap, size=m).astype(np.uint8)
            d = oracle.level_dest(lab, kap, 1 << 20, False)
            order = np.argsort(lab, kind="stable")
            expect = np.empty(m, dtype=np.uint64)
            expect[order] = np.arange(m)
            assert np.array_equal(d, expect)


def test_level_tiled_invariants():
    """Tiled level: a permutation; every item inside its final region; the
    kept items are exactly the rank-r items placed at their piece fronts."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        kap = int(rng.integers(1, 5))
        k = 1 << kap
        tile = int(rng.integers(k + 1, 4 * k + 8))
        m = int(rng.integers(2, 400))
        lab = rng.integers(0, k, size=m).astype(np.uint8)
        d = oracle.level_dest(lab, kap, tile, True)
        assert sorted(d.tolist()) == list(range(m))
        N = np.bincount(lab, minlength=k)
        S = np.concatenate([[0], np.cumsum(N)[:-1]])
        assert np.all(d >= S[lab]) and np.all(d < S[lab] + N[lab])
        assert d.tolist() == spec.level_dest(lab.tolist(), k, tile, True)


def test_level_tiled_single_tile_without_boundary_moves():
    """With one tile and equal counts the rough pass already is exact: the
    result equals the stable counting sort."""
    lab = np.array([1, 0, 2, 3, 3, 2, 0, 1], dtype=np.uint8)  # two of each label
    d = oracle.level_dest(lab, 2, 100, True)
    e = oracle.level_dest(lab, 2, 100, False)
    assert np.array_equal(d, e)


# ---------------------------------------------------------- whole shuffle ---
def test_c_oracle_matches_python_spec():
    rng = random.Random(6)
    for trial in range(400):
        kl = rng.randint(1, 4)
        tile = rng.randint((1 << kl) + 1, 60)
        p = oracle.Params(tile, kl, rng.randint(1, 10), rng.randint(0, 9))
        n = rng.randint(0, 350)
        seed = rng.getrandbits(64)
        a = np.arange(n, dtype=np.uint32)
        oracle.shuffle(a, seed, p, stream_id=trial)
        b = spec.shuffle(list(range(n)), spec.PhiloxSource(seed, trial), p.tile, p.kmax_log2, p.n0, p.lmax)
        assert a.tolist() == b


@pytest.mark.parametrize("p", TINY + [oracle.Params(32768), oracle.Params(9, 3, 1, 2)])
def test_exact_uniformity_by_enumeration(p):
    """Over every label and draw outcome, each permutation of m <= 5 items
    has probability exactly 1/m! (up to float summation)."""
    for m in range(1, 6):
        prob, paths = oracle.enumerate_outcomes(m, p)
        assert paths >= 1
        assert np.max(np.abs(prob - 1.0 / math.factorial(m))) < 1e-12


def test_enumeration_exercises_movers():
    """The tiny parameters really route movers: many label vectors of a tiled
    level produce items that do not stay at their rough slot."""
    k, tile, m = 2, 3, 5
    moved = 0
    for code in range(1 << m):
        lab = [(code >> i) & 1 for i in range(m)]
        d = oracle.level_dest(np.array(lab, dtype=np.uint8), 1, tile, True)
        rough = oracle.level_dest(np.array(lab, dtype=np.uint8), 1, tile, False)
        moved += int(not np.array_equal(d, rough))
    assert moved > 5


def _fig1():
    with open(os.path.join(HERE, "golden", "fisher_yates_fig1.json")) as fh:
        return json.load(fh)


def test_fisher_yates_fig1_step_order_golden():
    """Fig. 1 worked by hand (tests/golden/fisher_yates_fig1.json): the draws
    are requested for i = m-1 down to 1 with bound i + 1, each keyed by the
    absolute position base + i, and the swaps give the hand-derived map."""
    g = _fig1()["single"]
    table = {int(k): v for k, v in g["draws_by_position"].items()}
    calls = []

    def draw(level, pos, bound):
        calls.append([level, pos, bound])
        return table.get(pos, 0)

    dest = oracle.fy_dest_scripted(g["m"], g["level"], g["base"], draw)
    assert calls == g["calls"]
    assert dest.tolist() == g["dest"]


def test_fisher_yates_absolute_position_keys_golden():
    """Two equal-size Fisher-Yates leaves at one level (hand-worked): every
    draw is keyed by its absolute position, so the two leaves take different
    draws; both renditions of the definition reproduce the hand result."""
    g = _fig1()["two_leaves"]
    p = oracle.Params(**g["params"])
    labels = g["labels_level0"]
    draws = {int(k): v for k, v in g["draws_level1_by_position"].items()}
    for rendition in ("c", "spec"):
        calls, bad = [], []

        def label(level, pos, kappa):
            if level != 0 or kappa != 1 or not 0 <= pos < len(labels):
                bad.append((level, pos, kappa))
                return 0
            return labels[pos]

        def draw(level, pos, bound):
            calls.append([level, pos, bound])
            return draws.get(pos, 0)

        if rendition == "c":
            arr = np.arange(g["n"], dtype=np.uint32)
            oracle.shuffle_scripted(arr, p, label, draw)
            out = arr.tolist()
        else:
            src = type("Scripted", (), {"label": staticmethod(label), "draw": staticmethod(draw)})
            out = spec.shuffle(list(range(g["n"])), src, p.tile, p.kmax_log2, p.n0, p.lmax)
        assert not bad, (rendition, bad)
        assert calls == g["calls_level1"], rendition
        assert out == g["result"], rendition


def test_threaded_oracle_equals_single_thread():
    """The top level's buckets solved on several host threads give the same
    bytes as one thread (sizes with one and two tiled levels, ragged)."""
    for n, w in [(100_003, 4), ((1 << 21) + 77, 8), (300_001, 16)]:
        h = workloads.random_values(n, w, 3)
        p = oracle.default_params(n, w)
        a = h.copy()
        oracle.shuffle(a, 1234, p, stream_id=5)
        b = h.copy()
        oracle.shuffle(b, 1234, p, stream_id=5, threads=6)
        assert np.array_equal(a, b), (n, w)


def test_enumeration_detects_bias():
    """Sanity of the enumerator itself: Fisher-Yates with the partner drawn
    from [0, m) instead of [0, i] (a classic bias) is visibly non-uniform."""
    m = 3
    counts = {}
    for draws in np.ndindex(*(m for _ in range(m - 1))):
        a = list(range(m))
        for step, i in enumerate(range(m - 1, 0, -1)):
            j = draws[step]
            a[i], a[j] = a[j], a[i]
        counts[tuple(a)] = counts.get(tuple(a), 0) + 1
    assert len(set(counts.values())) > 1


@pytest.mark.parametrize("p", [oracle.Params(32768)] + TINY)
def test_chi_square_all_permutations(p):
    """n = 3..6 over 10^6 consecutive seeds (tiny parameters: fewer seeds):
    the count of each of the n! permutations is consistent with uniform."""
    from scipy import stats

    seeds = 10**6 if p.tile > 100 else 2 * 10**5
    for n in range(3, 7):
        c = oracle.perm_histogram(n, 0, seeds, p).astype(np.float64)
        assert c.sum() == seeds
        chi2, pv = stats.chisquare(c)
        assert pv > 1e-5, (n, pv)


def test_position_frequencies():
    """Item i lands at position j with probability 1/n (chi-square per row)
    and pairs of items are not correlated (adjacent items rarely stay
    adjacent more than chance allows)."""
    from scipy import stats

    n, seeds = 256, 20000
    p = oracle.Params(40, 3, 4, 32)  # several tiled levels at n = 256
    c = oracle.position_histogram(n, 1000, seeds, p).astype(np.float64)
    assert np.all(c.sum(axis=1) == seeds) and np.all(c.sum(axis=0) == seeds)
    pvals = [stats.chisquare(row).pvalue for row in c]
    # uniform rows give uniform p-values; check their spread
    assert stats.kstest(pvals, "uniform").pvalue > 1e-4


def test_two_independence():
    """2-independence of output ranks: for items 0 and 1 the joint position
    distribution over (pos0, pos1) is uniform over ordered pairs."""
    from scipy import stats

    n, seeds = 8, 40000
    p = oracle.Params(5, 2, 1, 8)
    joint = np.zeros((n, n))
    for s in range(seeds):
        a = np.arange(n, dtype=np.uint32)
        oracle.shuffle(a, s, p)
        pos = np.argsort(a)
        joint[pos[0], pos[1]] += 1
    assert np.all(np.diag(joint) == 0)
    off = joint[~np.eye(n, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-5


def test_permutation_validity_all_widths():
    for w in (4, 8, 16):
        for n in [0, 1, 2, 3, 63, 64, 65, 1000, 70000]:
            a = workloads.identity(n, w)
            b = a.copy()
            oracle.shuffle(b, 12345, oracle.default_params(n, w))
            if w == 16:
                assert np.array_equal(np.sort(b[:, 0]), a[:, 0])
                assert np.array_equal(workloads.splitmix64(b[:, 0]), b[:, 1])
            else:
                assert np.array_equal(np.sort(b), a)


def test_data_independence():
    """shuffle(values) == values[pi] where pi = shuffle(identity)."""
    n = 50000
    p = oracle.Params(600, 5, 8, 32)
    ident = np.arange(n, dtype=np.uint64)
    oracle.shuffle(ident, 7, p)
    vals = workloads.random_values(n, 8, 8)
    out = vals.copy()
    oracle.shuffle(out, 7, p)
    assert np.array_equal(out, vals[ident])


def test_stream_id_and_seed_change_result():
    n = 1000
    p = oracle.default_params(n, 4)
    base = oracle.shuffle(np.arange(n, dtype=np.uint32), 1, p)
    assert not np.array_equal(base, oracle.shuffle(np.arange(n, dtype=np.uint32), 2, p))
    assert not np.array_equal(base, oracle.shuffle(np.arange(n, dtype=np.uint32), 1, p, stream_id=1))
    assert np.array_equal(base, oracle.shuffle(np.arange(n, dtype=np.uint32), 1, p))


def test_fisher_yates_baseline_equals_base_case():
    """The sequential FY baseline uses the oracle's base-case draws: below n0
    the oracle is exactly it."""
    p = oracle.Params(32768, 8, 64, 32)
    for n in [2, 10, 64]:
        a = oracle.shuffle(np.arange(n, dtype=np.uint32), 31, p)
        b = oracle.fisher_yates(np.arange(n, dtype=np.uint32), 31)
        assert np.array_equal(a, b)


def test_invalid_params_rejected():
    assert not oracle.check_params(oracle.Params(2, 1, 1, 1))   # tile must exceed 2^kmax
    assert not oracle.check_params(oracle.Params(100, 9, 1, 1))
    assert not oracle.check_params(oracle.Params(100, 0, 1, 1))
    assert not oracle.check_params(oracle.Params(100, 3, 0, 1))
    assert not oracle.check_params(oracle.Params(100, 3, 1, 256))
    assert oracle.check_params(oracle.Params(3, 1, 1, 0))


def _mutant_spec(old: str, new: str):
    """A copy of the Python spec oracle with one planted slip."""
    import types

    text = open(spec.__file__).read()
    assert old in text
    mod = types.ModuleType("spec_mutant")
    exec(compile(text.replace(old, new), "spec_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize(
    "old,new",
    [
        # free slots paired in descending instead of ascending order
        ("zip(movers[b], free)", "zip(movers[b], free[::-1])"),
        # piece start computed with ceil instead of floor
        ("return edge[b] + t * size // tiles", "return edge[b] - (-t * size // tiles)"),
        # read order by descending bucket
        ("        for b in range(k):\n            for x in range(lo[b], hi[b]):",
         "        for b in reversed(range(k)):\n            for x in range(lo[b], hi[b]):"),
        # tile count from T instead of T - k
        ("tiles = -(-m // (tile - k))", "tiles = -(-m // tile)"),
    ],
)
def test_planted_mistakes_are_caught(old, new):
    """Plausible slips in the tiled level still give valid, even uniform,
    shuffles; the hand-worked examples expose each of them."""
    mut = _mutant_spec(old, new)
    caught = False
    for name in ["level_tiled_k2.json", "level_tiled_k4_empty_tiles.json"]:
        g = json.load(open(os.path.join(HERE, "golden", name)))
        d = mut.level_dest(g["labels"], 1 << g["kappa"], g["tile"], True)
        assert sorted(d) == list(range(g["m"]))
        caught |= d != g["dest"]
    assert caught
