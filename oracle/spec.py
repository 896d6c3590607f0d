"""Pure-Python rendition of the ScatterShuffle definition (version 1).

TEST INFRASTRUCTURE ONLY.  A second, independent transcription of the same
definition as ``css_oracle.c``, written for readability and used on small
inputs to cross-check the C oracle.  Pure-Python loops: keep n small.

Paper: arXiv 2302.03317 (Penschuck).  Section references below are to it.
"""
from __future__ import annotations

MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64
    multiplications mixed with the key, key bumped by Weyl constants."""
    x0, x1, x2, x3 = (c & MASK32 for c in ctr)
    k0, k1 = (k & MASK32 for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & MASK32
            k1 = (k1 + 0xBB67AE85) & MASK32
        p0 = 0xD2511F53 * x0
        p1 = 0xCD9E8D57 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0) & MASK32, p1 & MASK32, ((p0 >> 32) ^ x3 ^ k1) & MASK32, p0 & MASK32
    return (x0, x1, x2, x3)


class PhiloxSource:
    """Labels and Fisher-Yates draws as pure functions of
    (seed, stream, level, position) -- Sec. 5's reproducibility requirement."""

    def __init__(self, seed: int, stream_id: int = 0):
        self.key = (seed & MASK32, (seed >> 32) & MASK32)
        self.stream = stream_id & MASK32

    def _block(self, block: int, tag: int):
        return philox4x32_10((block & MASK32, block >> 32, tag, self.stream), self.key)

    def label(self, level: int, pos: int, kappa: int) -> int:
        # 16 labels per block: byte (pos mod 16), top kappa bits (Sec. 2.3:
        # a power-of-two range is a shift of random bits)
        words = self._block(pos >> 4, level | (1 << 8))
        j = pos & 15
        byte = (words[j >> 2] >> (8 * (j & 3))) & 0xFF
        return byte >> (8 - kappa)

    def draw(self, level: int, pos: int, bound: int) -> int:
        # Lemire's multiply-and-reject (cited in Sec. 2.3); a rejected word
        # is redrawn with the next attempt number in the counter.  Bounds up
        # to 2^16 take 16-bit words (eight per block, tag purpose 3), larger
        # bounds 32-bit words (four per block, tag purpose 2).
        attempt = 0
        if bound <= 1 << 16:
            threshold = (1 << 16) % bound
            while True:
                words = self._block(pos >> 3, level | (3 << 8) | ((attempt & 0xFFFF) << 16))
                h = pos & 7
                x = (words[h >> 1] >> (16 * (h & 1))) & 0xFFFF
                prod = x * bound
                if (prod & 0xFFFF) >= threshold:
                    return prod >> 16
                attempt += 1
        threshold = (1 << 32) % bound
        while True:
            words = self._block(pos >> 2, level | (2 << 8) | ((attempt & 0xFFFF) << 16))
            prod = words[pos & 3] * bound
            if (prod & MASK32) >= threshold:
                return prod >> 32
            attempt += 1


def kappa_for(m: int, hbm: bool, tile: int, kmax_log2: int, n0: int) -> int:
    g = max(1, tile // 2 if hbm else n0 // 2)
    r = 1
    while g * (1 << r) < m:
        r += 1
    h = -(-r // kmax_log2)
    return min(kmax_log2, -(-r // h))


def level_dest(labels, k: int, tile: int, hbm: bool):
    """Destinations of one IpSc level (relative positions)."""
    m = len(labels)
    counts = [0] * k
    for a in labels:
        counts[a] += 1
    starts = [0] * k
    for b in range(1, k):
        starts[b] = starts[b - 1] + counts[b - 1]
    dest = [None] * m
    if not hbm:
        seen = [0] * k
        for i, a in enumerate(labels):
            dest[i] = starts[a] + seen[a]
            seen[a] += 1
        return dest

    # RoughScatter on k equal regions, one piece of each per tile (Sec. 3.3, 4.1)
    tiles = -(-m // (tile - k))
    edge = [b * m // k for b in range(k + 1)]

    def piece(b, t):
        size = edge[b + 1] - edge[b]
        return edge[b] + t * size // tiles

    kept = set()
    movers = [[] for _ in range(k)]
    for t in range(tiles):
        lo = [piece(b, t) for b in range(k)]
        hi = [piece(b, t + 1) for b in range(k)]
        rank = [0] * k
        for b in range(k):
            for x in range(lo[b], hi[b]):
                a = labels[x]
                r = rank[a]
                rank[a] += 1
                y = lo[a] + r
                if r < hi[a] - lo[a] and starts[a] <= y < starts[a] + counts[a]:
                    dest[x] = y
                    kept.add(y)
                else:
                    movers[a].append(x)
    # FineScatter's role: fill each final region's free slots in order
    for b in range(k):
        free = [y for y in range(starts[b], starts[b] + counts[b]) if y not in kept]
        assert len(free) == len(movers[b])
        for x, y in zip(movers[b], free):
            dest[x] = y
    return dest


def shuffle(values, source, tile: int, kmax_log2: int = 8, n0: int = 64, lmax: int = 32):
    """Return a shuffled copy of ``values`` (a list)."""
    arr = list(values)

    def solve(base: int, m: int, level: int):
        if m <= 1:
            return
        if m <= n0 or level >= lmax:
            # Fisher-Yates (Fig. 1): i from m-1 down to 1, partner in [0, i]
            for i in range(m - 1, 0, -1):
                j = source.draw(level, base + i, i + 1)
                arr[base + i], arr[base + j] = arr[base + j], arr[base + i]
            return
        hbm = m > tile - (1 << kmax_log2)
        kap = kappa_for(m, hbm, tile, kmax_log2, n0)
        k = 1 << kap
        labels = [source.label(level, base + i, kap) for i in range(m)]
        dest = level_dest(labels, k, tile, hbm)
        old = arr[base:base + m]
        for i in range(m):
            arr[base + dest[i]] = old[i]
        start = base
        for b in range(k):
            size = labels.count(b)
            solve(start, size, level + 1)
            start += size

    solve(0, len(arr), 0)
    return arr
