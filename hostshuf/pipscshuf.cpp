// Host PIpScShuf: the paper's own parallel in-place shuffle on the host's
// CPU cores, as a same-machine CPU baseline for the GPU library.
//
// M. Penschuck, "Engineering Shared-Memory Parallel Shuffling to Generate
// Random Permutations In-Place" (arXiv 2302.03317).  Written from the paper's
// description of the method (no code of its repository is used):
//   - IpScShuf (Sec. 3.2): one level scatters the items into k buckets of
//     random labels in place, then every bucket is shuffled recursively;
//     Fisher-Yates (Sec. 2.2, Fig. 1) below the base-case size (2^18 items,
//     Sec. 5);
//   - RoughScatter (Sec. 3.3): k equal buckets, each a triple (b, s, e) with
//     placed items in [b, s) and staged items in [s, e); the first staged
//     item of bucket 0 is swapped to the front of the staged part of a
//     uniformly drawn bucket j, which grows by one placed item; it stops as
//     soon as a bucket is full;
//   - FineScatter (Sec. 3.4): the final bucket sizes are the placed counts
//     plus a multinomial share of the R staged items; TwoSweep moves the
//     bucket boundaries to those sizes by swapping staged items between
//     neighbours (Sec. 3.4.1); the staged items are then compacted to the
//     front by swaps, shuffled, and the swaps undone, which puts a random
//     permutation of them into the staged slots (Sec. 3.4.2);
//   - parallel RoughScatter (Sec. 4.1): binary fork-join; each bucket is
//     split in two halves, one per subtask; after both subtasks join the
//     halves are merged by swapping the first half's staged items behind the
//     second half's placed items, and RoughScatter continues on the merged
//     buckets; the k buckets of a level are then independent subproblems,
//     run as parallel tasks;
//   - k = 64 below 128 MiB of data and 256 above; subtasks' generators are
//     derived from the parent's in a fixed order, so the permutation does
//     not depend on scheduling (Sec. 5).
// The generator is a 128-bit multiplicative congruential generator with the
// XSL-RR output of the PCG family (O'Neill 2014; the paper measures with
// this generator); bounded integers use Lemire's multiply-and-reject
// (Sec. 2.3).
//
// This library is a CPU baseline only: the GPU library never calls it.
#include <omp.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace {

using u128 = unsigned __int128;

// 128-bit MCG, XSL-RR 64-bit output.
struct Rng {
    u128 s;
    explicit Rng(u128 seed) : s(seed | 1) {}
    uint64_t next()
    {
        const u128 mult = (static_cast<u128>(0x2360ED051FC65DA4ull) << 64) | 0x4385DF649FCCF645ull;
        s *= mult;
        const unsigned rot = static_cast<unsigned>(s >> 122);
        const uint64_t x = static_cast<uint64_t>(s >> 64) ^ static_cast<uint64_t>(s);
        return (x >> rot) | (x << ((64 - rot) & 63));
    }
    // uniform in [0, bound), Lemire's method
    uint64_t below(uint64_t bound)
    {
        u128 m = static_cast<u128>(next()) * bound;
        uint64_t lo = static_cast<uint64_t>(m);
        if (lo < bound) {
            const uint64_t t = (0 - bound) % bound;
            while (lo < t) {
                m = static_cast<u128>(next()) * bound;
                lo = static_cast<uint64_t>(m);
            }
        }
        return static_cast<uint64_t>(m >> 64);
    }
    // a generator for a subtask, derived from this one
    Rng child() { return Rng((static_cast<u128>(next()) << 64) | next()); }
};

// Labels in [0, 2^kappa): floor(64 / kappa) of them per random word.
struct Labels {
    Rng& rng;
    unsigned kappa, per, left = 0;
    uint64_t word = 0;
    Labels(Rng& r, unsigned k) : rng(r), kappa(k), per(64 / k) {}
    unsigned next()
    {
        if (left == 0) {
            word = rng.next();
            left = per;
        }
        const unsigned l = static_cast<unsigned>(word >> (64 - kappa));
        word <<= kappa;
        --left;
        return l;
    }
};

struct Bucket {
    uint64_t b, s, e;  // placed [b, s), staged [s, e)
};

struct Config {
    unsigned kappa_small = 6, kappa_large = 8;  // k = 64 / 256
    uint64_t large_bytes = 128ull << 20;        // data size from which k = 256
    uint64_t base_case = 1ull << 18;            // Fisher-Yates at or below this many items
    uint64_t par_cutoff = 1ull << 16;           // sequential RoughScatter at or below this many items
    uint64_t task_min = 1ull << 16;             // subproblems below this run inside their parent's task
};

template <typename E>
struct Shuffler {
    E* X;
    Config cfg;

    void swap(uint64_t a, uint64_t b)
    {
        const E t = X[a];
        X[a] = X[b];
        X[b] = t;
    }

    void fisher_yates(uint64_t base, uint64_t m, Rng& rng)
    {
        for (uint64_t i = m; i-- > 1;) swap(base + i, base + rng.below(i + 1));
    }

    static bool any_full(const Bucket* B, unsigned k)
    {
        for (unsigned i = 0; i < k; ++i)
            if (B[i].s == B[i].e) return true;
        return false;
    }

    // Sequential RoughScatter on the buckets as they are.
    void rough(Bucket* B, unsigned k, unsigned kappa, Rng& rng)
    {
        if (any_full(B, k)) return;
        Labels lab(rng, kappa);
        for (;;) {
            const unsigned j = lab.next();
            if (j != 0) swap(B[0].s, B[j].s);
            if (++B[j].s == B[j].e) return;
        }
    }

    // Parallel RoughScatter on the buckets (all items staged on entry).
    void par_rough(Bucket* B, unsigned k, unsigned kappa, uint64_t items, Rng& rng)
    {
        if (items <= cfg.par_cutoff) {
            rough(B, k, kappa, rng);
            return;
        }
        std::vector<Bucket> L(k), R(k);
        for (unsigned i = 0; i < k; ++i) {
            const uint64_t mid = B[i].b + (B[i].e - B[i].b) / 2;
            L[i] = {B[i].b, B[i].b, mid};
            R[i] = {mid, mid, B[i].e};
        }
        Rng rl = rng.child(), rr = rng.child();
        const uint64_t half = items / 2;
#pragma omp task default(shared) firstprivate(half)
        par_rough(L.data(), k, kappa, half, rl);
        par_rough(R.data(), k, kappa, items - half, rr);
#pragma omp taskwait
        // merge the halves: the first half's staged items behind the second
        // half's placed items
        for (unsigned i = 0; i < k; ++i) {
            const uint64_t mid = L[i].e;
            const uint64_t a = mid - L[i].s, p = R[i].s - mid;
            const uint64_t c = std::min(a, p);
            for (uint64_t x = 0; x < c; ++x) swap(L[i].s + x, R[i].s - c + x);
            B[i].s = L[i].s + p;
        }
        rough(B, k, kappa, rng);
    }

    // Bucket i gives the last d slots of its staged part to bucket i + 1.
    void give_right(Bucket* B, unsigned i, uint64_t d)
    {
        Bucket& n = B[i + 1];
        const uint64_t nb = B[i].e - d, p = n.s - n.b;
        const uint64_t c = std::min(d, p);
        for (uint64_t x = 0; x < c; ++x) swap(nb + x, n.s - c + x);
        B[i].e = nb;
        n.b = nb;
        n.s = nb + p;
    }

    // Bucket i + 1 gives the first d slots of its region to bucket i (as
    // staged slots), after moving d staged items to its front.
    void give_left(Bucket* B, unsigned i, uint64_t d)
    {
        Bucket& n = B[i + 1];
        const uint64_t p = n.s - n.b;
        const uint64_t c = std::min(d, p);
        for (uint64_t x = 0; x < c; ++x) swap(n.b + x, n.s + d - c + x);
        n.b += d;
        n.s = n.b + p;
        B[i].e += d;
    }

    // FineScatter: final sizes, TwoSweep, shuffle of the staged items.
    void fine(Bucket* B, unsigned k, unsigned kappa, Rng& rng)
    {
        uint64_t R = 0;
        for (unsigned i = 0; i < k; ++i) R += B[i].e - B[i].s;
        if (R == 0) return;
        // multinomial share of the staged items: R uniform labels counted
        std::vector<uint64_t> extra(k, 0);
        {
            Labels lab(rng, kappa);
            for (uint64_t r = 0; r < R; ++r) extra[lab.next()]++;
        }
        std::vector<uint64_t> fend(k);  // final end of every bucket
        uint64_t run = B[0].b;
        for (unsigned i = 0; i < k; ++i) {
            run += (B[i].s - B[i].b) + extra[i];
            fend[i] = run;
        }
        // TwoSweep: boundaries that move left, from the left; then those
        // that move right, from the right
        for (unsigned i = 0; i + 1 < k; ++i)
            if (B[i].e > fend[i]) give_right(B, i, B[i].e - fend[i]);
        for (unsigned i = k - 1; i-- > 0;)
            if (B[i].e < fend[i]) give_left(B, i, fend[i] - B[i].e);
        // compact the staged items to the front of the level by swaps,
        // shuffle them there, undo the swaps
        const uint64_t base = B[0].b;
        uint64_t r = 0;
        for (unsigned i = 0; i < k; ++i)
            for (uint64_t p = B[i].s; p < B[i].e; ++p) swap(base + r++, p);
        fisher_yates(base, R, rng);
        for (unsigned i = k; i-- > 0;)
            for (uint64_t p = B[i].e; p-- > B[i].s;) swap(base + --r, p);
    }

    void solve(uint64_t base, uint64_t m, Rng rng)
    {
        if (m <= 1) return;
        if (m <= cfg.base_case) {
            fisher_yates(base, m, rng);
            return;
        }
        const unsigned kappa = m * sizeof(E) >= cfg.large_bytes ? cfg.kappa_large : cfg.kappa_small;
        const unsigned k = 1u << kappa;
        std::vector<Bucket> B(k);
        for (unsigned i = 0; i < k; ++i) {
            const uint64_t b = base + static_cast<uint64_t>((static_cast<u128>(i) * m) >> kappa);
            const uint64_t e = base + static_cast<uint64_t>((static_cast<u128>(i + 1) * m) >> kappa);
            B[i] = {b, b, e};
        }
        Rng rr = rng.child(), rf = rng.child();
        par_rough(B.data(), k, kappa, m, rr);
        fine(B.data(), k, kappa, rf);
        // the buckets are independent subproblems
        for (unsigned i = 0; i < k; ++i) {
            const uint64_t b = B[i].b, len = B[i].e - B[i].b;
            Rng rc = rng.child();
            if (len >= cfg.task_min) {
#pragma omp task default(shared) firstprivate(b, len, rc)
                solve(b, len, rc);
            } else {
                solve(b, len, rc);
            }
        }
#pragma omp taskwait
    }
};

template <typename E>
int run(void* data, uint64_t n, uint64_t seed, int threads, const Config& cfg)
{
    Shuffler<E> S{static_cast<E*>(data), cfg};
    const Rng root(static_cast<u128>(seed) * 0x9E3779B97F4A7C15ull + 0x2302033172026ull);
    if (threads < 1) threads = omp_get_max_threads();
#pragma omp parallel num_threads(threads)
#pragma omp single
    S.solve(0, n, root);
    return 0;
}

struct Rec16 {
    uint64_t a, b;
};

template <typename E>
int fy_run(void* data, uint64_t n, uint64_t seed)
{
    Shuffler<E> S{static_cast<E*>(data), Config{}};
    Rng rng(static_cast<u128>(seed) * 0x9E3779B97F4A7C15ull + 0x2302033172026ull);
    S.fisher_yates(0, n, rng);
    return 0;
}

}  // namespace

extern "C" {

// Shuffle n elements of elem_bytes (4, 8 or 16) at `data` in place on
// `threads` host threads (<= 0: all).  kappa_small / kappa_large (1..8, 0 =
// the paper's 6 / 8), base_case (0 = 2^18) and par_cutoff (0 = 2^16) allow
// small settings for tests.  Returns 0, or -1 for bad arguments.
int pipscshuf_shuffle_ex(void* data, uint64_t n, uint32_t elem_bytes, uint64_t seed, int threads,
                         uint32_t kappa_small, uint32_t kappa_large, uint64_t base_case,
                         uint64_t par_cutoff)
{
    if ((!data && n > 1) || kappa_small > 8 || kappa_large > 8) return -1;
    Config cfg;
    if (kappa_small) cfg.kappa_small = kappa_small;
    if (kappa_large) cfg.kappa_large = kappa_large;
    if (base_case) cfg.base_case = base_case;
    if (par_cutoff) {
        cfg.par_cutoff = par_cutoff;
        cfg.task_min = par_cutoff;
    }
    switch (elem_bytes) {
    case 4: return run<uint32_t>(data, n, seed, threads, cfg);
    case 8: return run<uint64_t>(data, n, seed, threads, cfg);
    case 16: return run<Rec16>(data, n, seed, threads, cfg);
    default: return -1;
    }
}

int pipscshuf_shuffle(void* data, uint64_t n, uint32_t elem_bytes, uint64_t seed, int threads)
{
    return pipscshuf_shuffle_ex(data, n, elem_bytes, seed, threads, 0, 0, 0, 0);
}

// Sequential Fisher-Yates (Fig. 1) with the same generator, one thread.
int pipscshuf_fisher_yates(void* data, uint64_t n, uint32_t elem_bytes, uint64_t seed)
{
    if (!data && n > 1) return -1;
    switch (elem_bytes) {
    case 4: return fy_run<uint32_t>(data, n, seed);
    case 8: return fy_run<uint64_t>(data, n, seed);
    case 16: return fy_run<Rec16>(data, n, seed);
    default: return -1;
    }
}

}  // extern "C"
