// Subproblems that fit one tile, finished in LDS: the remaining recursion
// levels of ScatterShuffle (arXiv 2302.03317, Sec. 3.1 / Fig. 2) and the
// Fisher-Yates base case (Fig. 1).
//
// One workgroup at a time per subproblem ("leaf"); persistent workgroups take
// the leaves of a size class one after another.  Only 16-bit indices move
// while the levels run: idx[x] is the original
// leaf index of the item at position x.  Each in-tile level is a stable
// counting sort of every splitting segment by its label; segments larger
// than one wave can hold are split by the whole workgroup, the others by one
// wave each.  Segments at the base case run Fisher-Yates, one lane per
// segment.  Finally the elements are read once from HBM into an LDS staging
// copy and written once, every position gathering its item by the index array.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

namespace ipss {

namespace {

// ROUNDS (a template parameter) bounds the index rounds a thread holds in
// registers: a leaf has at most kThreads * ROUNDS items, and one wave splits
// segments of up to 64 * ROUNDS items.

__device__ __forceinline__ uint32_t seg_start(uint32_t e) { return e & 0xFFFFu; }
__device__ __forceinline__ uint32_t seg_len(uint32_t e) { return e >> 16; }
__device__ __forceinline__ uint32_t seg_pack(uint32_t s, uint32_t l) { return s | (l << 16); }

// Bucket-count exponent of an in-tile segment: target size max(1, n0/2).
__device__ __forceinline__ uint32_t kappa_in_tile(uint32_t m, const Params& prm)
{
    uint32_t g = prm.n0 / 2;
    if (g < 1) g = 1;
    uint32_t r = 1;
    uint64_t reach = 2ull * g;
    while (reach < m) {
        reach <<= 1;
        ++r;
    }
    const uint32_t h = (r + prm.kmax_log2 - 1) / prm.kmax_log2;
    const uint32_t kap = (r + h - 1) / h;
    return kap < prm.kmax_log2 ? kap : prm.kmax_log2;
}

// Fisher-Yates on idx[s0, s0 + len) (2 <= len <= 2^16): i from len-1 down
// to 1, the partner drawn from [0, i] at position pbase + s0 + i with a short
// draw.  One Philox block serves the eight positions 8B..8B+7.  The lanes of
// a wave run different segments, so each lane starts after o idle steps, o
// chosen so that every lane enters a new block on the same step: the block
// is then computed once per eight steps for the whole wave, and the 16-bit
// word a step uses is known at compile time.  (Batching steps into one LDS
// round trip with the swaps resolved in registers measured slower: the
// chains of different lanes and waves already overlap.)
__device__ __forceinline__ void fy_segment(uint16_t* idx, uint32_t s0, uint32_t len, uint64_t pbase,
                                           uint32_t level, const Key& key)
{
    const uint64_t top = pbase + s0 + len - 1;  // position of the first step
    const uint32_t o = (7u - static_cast<uint32_t>(top & 7)) & 7u;
    const uint32_t steps = o + len - 1;
    for (uint32_t s8 = 0; s8 < steps; s8 += 8) {
        // virtual position of step s is top + o - s; (top + o) mod 8 = 7
        const uint64_t vb = (top + o - s8) >> 3;
        const Word4 v = fy_short_block(key, level, vb, 0);
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) {
            const uint32_t s = s8 + u;
            if (s >= o && s < steps) {
                const uint32_t i = len - 1 - (s - o);
                const uint32_t x = half_of(v, 7 - u);
                const uint32_t j = fy_short_draw(key, level, top + o - s, i + 1, x);
                const uint16_t a = idx[s0 + i];
                idx[s0 + i] = idx[s0 + j];
                idx[s0 + j] = a;
            }
        }
    }
}

// Whole-workgroup stable split of segment [s0, s0 + len) by KAPPA-bit labels;
// children (start, length) go to out[0..k).  On a leaf's first split
// (`first`) the segment is the whole leaf in its initial order, so the item
// at position x is leaf item x and the index array is not read (nor need it
// have been written).  Labels stay in registers between the ranking and the
// placement; the bucket offsets are folded into the per-wave offsets so that
// the placement reads one counter per item.
template <int KAPPA, int ROUNDS, bool ATOMIC>
__device__ __forceinline__ void split_workgroup(uint16_t* idx, const uint8_t* lab, uint32_t* H,
                                                uint32_t hs, uint32_t* out, uint32_t s0,
                                                uint32_t len, uint32_t tid, uint32_t wv,
                                                uint32_t lane, bool first)
{
    constexpr uint32_t k = 1u << KAPPA, sh = 8 - KAPPA;
    uint32_t* Htot = H + kWaves * hs;
    const uint32_t end = s0 + len;
    const uint32_t per_wave = ((len + kWaves * 64 - 1) / (kWaves * 64)) * 64;
    const uint32_t rounds = per_wave / 64;
    const uint32_t first_x = s0 + wv * per_wave + lane;
    for (uint32_t j = tid; j < (kWaves + 1) * hs; j += kThreads) H[j] = 0;
    block_sync();
    uint32_t pk[ROUNDS];
    uint32_t lb[(ROUNDS + 3) / 4];
#pragma unroll
    for (uint32_t r = 0; r < static_cast<uint32_t>(ROUNDS); ++r) {
        const uint32_t x = first_x + 64u * r;
        uint32_t v = 0, l = 0;
        if (r < rounds && x < end) {
            l = lab[x] >> sh;
            uint32_t rank;
            if (ATOMIC) {
                rank = atomicAdd(&H[wv * hs + l], 1u);  // lane-ordered: the stable rank
            } else {
                const uint64_t peers = match_label_bits<KAPPA>(l);
                const uint32_t below = bits_below(peers);
                const uint32_t old = H[wv * hs + l];
                if (below == 0) H[wv * hs + l] = old + static_cast<uint32_t>(__popcll(peers));
                rank = old + below;
            }
            v = (first ? x : static_cast<uint32_t>(idx[x])) | (rank << 16);
        }
        pk[r] = v;
        if (r % 4 == 0) lb[r / 4] = l;
        else lb[r / 4] |= l << (8 * (r % 4));
    }
    block_sync();
    for (uint32_t l = tid; l < k; l += kThreads) {
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t v = H[w * hs + l];
            H[w * hs + l] = run;
            run += v;
        }
        Htot[l] = run;
    }
    block_sync();
    if (wv == 0) wave_exclusive_scan(Htot, k);
    block_sync();
    for (uint32_t l = tid; l < k; l += kThreads) {
        const uint32_t base = s0 + Htot[l];
        out[l] = seg_pack(base, Htot[l + 1] - Htot[l]);
        for (int w = 0; w < kWaves; ++w) H[w * hs + l] += base;
    }
    block_sync();
#pragma unroll
    for (uint32_t r = 0; r < static_cast<uint32_t>(ROUNDS); ++r) {
        const uint32_t x = first_x + 64u * r;
        if (r < rounds && x < end) {
            const uint32_t l = (lb[r / 4] >> (8 * (r % 4))) & 0xFFu;
            idx[H[wv * hs + l] + (pk[r] >> 16)] = static_cast<uint16_t>(pk[r]);
        }
    }
    block_sync();
}

// One wave's stable split of segment [s0, s0 + len), len <= 64 * ROUNDS
// (`first` as for split_workgroup).
template <int KAPPA, int ROUNDS, bool ATOMIC>
__device__ __forceinline__ void split_wave(uint16_t* idx, const uint8_t* lab, uint32_t* Hw,
                                           uint32_t* out, uint32_t s0, uint32_t len,
                                           uint32_t lane, bool first)
{
    constexpr uint32_t k = 1u << KAPPA, sh = 8 - KAPPA;
    const uint32_t end = s0 + len;
    for (uint32_t j = lane; j <= k; j += 64) Hw[j] = 0;
    const uint32_t rounds = (len + 63) / 64;
    uint32_t pk[ROUNDS];
    uint32_t lb[(ROUNDS + 3) / 4];
#pragma unroll
    for (uint32_t r = 0; r < static_cast<uint32_t>(ROUNDS); ++r) {
        const uint32_t x = s0 + 64u * r + lane;
        uint32_t v = 0, l = 0;
        if (r < rounds && x < end) {
            l = lab[x] >> sh;
            uint32_t rank;
            if (ATOMIC) {
                rank = atomicAdd(&Hw[l], 1u);  // lane-ordered: the stable rank
            } else {
                const uint64_t peers = match_label_bits<KAPPA>(l);
                const uint32_t below = bits_below(peers);
                const uint32_t old = Hw[l];
                if (below == 0) Hw[l] = old + static_cast<uint32_t>(__popcll(peers));
                rank = old + below;
            }
            v = (first ? x : static_cast<uint32_t>(idx[x])) | (rank << 16);
        }
        pk[r] = v;
        if (r % 4 == 0) lb[r / 4] = l;
        else lb[r / 4] |= l << (8 * (r % 4));
    }
    wave_exclusive_scan(Hw, k);
    for (uint32_t l = lane; l < k; l += 64) out[l] = seg_pack(s0 + Hw[l], Hw[l + 1] - Hw[l]);
#pragma unroll
    for (uint32_t r = 0; r < static_cast<uint32_t>(ROUNDS); ++r) {
        const uint32_t x = s0 + 64u * r + lane;
        if (r < rounds && x < end) {
            const uint32_t l = (lb[r / 4] >> (8 * (r % 4))) & 0xFFu;
            idx[s0 + Hw[l] + (pk[r] >> 16)] = static_cast<uint16_t>(pk[r]);
        }
    }
}

// One leaf of a size class: at most kThreads * ROUNDS items, LDS laid out
// for the class capacity `cap` at smem.  Called by the whole workgroup.
template <typename E, int ROUNDS, bool ATOMIC>
__device__ __forceinline__ void leaf_body(const LeafDesc ld, const Params& prm, uint32_t cap, uint8_t* smem)
{
    constexpr int EMAX = ROUNDS;
    constexpr uint32_t kWaveSegMax = 64u * ROUNDS;  // largest segment split by one wave
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wv = uniform(tid >> 6);  // the same in all lanes of a wave
    const uint32_t m = static_cast<uint32_t>(ld.m);
    const uint32_t kmax = 1u << prm.kmax_log2;
    const uint32_t hs = kmax + 1;  // row stride of the counters
    const LeafLayout LL = leaf_layout(cap, sizeof(E), kmax, prm.n0);
    uint16_t* idx = reinterpret_cast<uint16_t*>(smem + LL.idx);
    uint8_t* labraw = smem + LL.lab;
    uint32_t* H = reinterpret_cast<uint32_t*>(smem + LL.hist);
    uint32_t* cur = reinterpret_cast<uint32_t*>(smem + LL.segs);
    uint32_t* nxt = cur + LL.seg_cap;
    uint32_t* tmpk = reinterpret_cast<uint32_t*>(smem + LL.tmpk);
    uint32_t* wl = reinterpret_cast<uint32_t*>(smem + LL.wl);
    // misc: [0] segments of the level, [1] large splitting segments,
    // [2] segments split by one wave, [3] base-case segments, [4..) large list
    uint32_t* misc = reinterpret_cast<uint32_t*>(smem + LL.misc);
    E* stage = reinterpret_cast<E*>(smem);

    global_t<E>* X = elem_gptr<E>(ld.elem_off) + ld.base;
    const uint64_t pbase = ld.base;
    const Key key = make_key(ld.seed, ld.stream_id);
    // labraw holds whole label blocks; lab[x] is the label byte of position pbase + x
    const uint8_t* lab = labraw + (pbase & 15);

    // The first level has the single segment [0, m), classified right here.
    // When it splits, the split writes the whole index array (the item at x
    // is leaf item x until then); otherwise the identity is written here.
    uint32_t level = ld.level;
    const bool first_split = m >= 2 && !(m <= prm.n0 || level >= prm.lmax);
    if (!first_split)
        for (uint32_t x = tid; x < m; x += kThreads) idx[x] = static_cast<uint16_t>(x);
    if (tid == 0) {
        const bool base = m <= prm.n0 || level >= prm.lmax;
        const bool split = m >= 2 && !base;
        cur[0] = seg_pack(0, m);
        nxt[0] = cur[0];
        tmpk[0] = split ? (1u << kappa_in_tile(m, prm)) : 0u;
        wl[0] = 0;
        misc[0] = 1;
        misc[1] = (split && m > kWaveSegMax) ? 1u : 0u;
        misc[2] = (split && m <= kWaveSegMax) ? 1u : 0u;
        misc[3] = (m >= 2 && base) ? 1u : 0u;
        misc[4] = 0;
    }
    bool classified = true;
    for (;;) {
        block_sync();
        const uint32_t nseg = misc[0];
        if (nseg == 0) break;
        const bool first = level == ld.level;  // the single segment [0, m) in its initial order
        if (!classified) {
            // Base-case segments are listed longest first (counting sort on
            // the length, kept in the next-level list, which only the splits
            // below write) so that the lanes of one wave run Fisher-Yates on
            // segments of similar length.  Splitting segments go to the large
            // list or to the one-wave list.
            for (uint32_t j = tid; j < 257; j += kThreads) H[j] = 0;
            if (tid == 0) {
                misc[1] = 0;
                misc[2] = 0;
            }
            block_sync();
            for (uint32_t i = tid; i < nseg; i += kThreads) {
                const uint32_t len = seg_len(cur[i]);
                uint32_t kk = 0;
                if (len >= 2) {
                    if (len <= prm.n0 || level >= prm.lmax) {
                        atomicAdd(&H[255 - (len < 255 ? len : 255)], 1u);
                    } else {
                        kk = 1u << kappa_in_tile(len, prm);
                        if (len > kWaveSegMax) misc[4 + atomicAdd(&misc[1], 1u)] = i;
                        else wl[atomicAdd(&misc[2], 1u)] = i;
                    }
                }
                tmpk[i] = kk;
            }
            block_sync();
            if (wv == 0) wave_exclusive_scan(H, 256);
            block_sync();
            for (uint32_t i = tid; i < nseg; i += kThreads) {
                const uint32_t e = cur[i];
                const uint32_t len = seg_len(e);
                if (len >= 2 && (len <= prm.n0 || level >= prm.lmax))
                    nxt[atomicAdd(&H[255 - (len < 255 ? len : 255)], 1u)] = e;
            }
            if (tid == 0) misc[3] = H[256];
            block_sync();
        }
        classified = false;
        const uint32_t nbig = misc[1], nwave = misc[2], nfy = misc[3];
        for (uint32_t i = tid; i < nfy; i += kThreads) {
            const uint32_t e = nxt[i];
            fy_segment(idx, seg_start(e), seg_len(e), pbase, level, key);
        }
        if (nbig + nwave == 0) break;
        // Label bytes of this level: whole 16-byte blocks, aligned.
        {
            const uint64_t b0 = pbase >> 4;
            const uint64_t nb = ((pbase + m - 1) >> 4) - b0 + 1;
            for (uint64_t i = tid; i < nb; i += kThreads) {
                const Word4 v = label_block(key, level, b0 + i);
                *reinterpret_cast<uint4*>(labraw + 16 * i) = make_uint4(v.x, v.y, v.z, v.w);
            }
        }
        block_sync();
        if (wv == 0) wave_exclusive_scan(tmpk, nseg);  // child offsets; tmpk[nseg] = total
        block_sync();

        // Large segments: the whole workgroup, one segment at a time.
        for (uint32_t bi = 0; bi < nbig; ++bi) {
            const uint32_t i = uniform(misc[4 + bi]);
            const uint32_t e = uniform(cur[i]);
            const uint32_t s0 = seg_start(e), len = seg_len(e);
            uint32_t* out = nxt + tmpk[i];
            if constexpr (ATOMIC) {
                switch (kappa_in_tile(len, prm)) {
                case 1: split_workgroup<1, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 2: split_workgroup<2, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 3: split_workgroup<3, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 4: split_workgroup<4, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 5: split_workgroup<5, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 6: split_workgroup<6, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 7: split_workgroup<7, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                default: split_workgroup<8, ROUNDS, true>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                }
            } else {
                switch (kappa_in_tile(len, prm)) {
                case 1: split_workgroup<1, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 2: split_workgroup<2, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 3: split_workgroup<3, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 4: split_workgroup<4, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 5: split_workgroup<5, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 6: split_workgroup<6, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                case 7: split_workgroup<7, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                default: split_workgroup<8, ROUNDS, false>(idx, lab, H, hs, out, s0, len, tid, wv, lane, first); break;
                }
            }
        }

        // Other splitting segments: one wave each.
        for (uint32_t j = wv; j < nwave; j += kWaves) {
            const uint32_t i = uniform(wl[j]);
            const uint32_t e = uniform(cur[i]);
            const uint32_t s0 = seg_start(e), len = seg_len(e);
            uint32_t* Hw = H + wv * hs;
            uint32_t* out = nxt + tmpk[i];
            if constexpr (ATOMIC) {
                switch (kappa_in_tile(len, prm)) {
                case 1: split_wave<1, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 2: split_wave<2, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 3: split_wave<3, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 4: split_wave<4, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 5: split_wave<5, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 6: split_wave<6, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 7: split_wave<7, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                default: split_wave<8, ROUNDS, true>(idx, lab, Hw, out, s0, len, lane, first); break;
                }
            } else {
                switch (kappa_in_tile(len, prm)) {
                case 1: split_wave<1, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 2: split_wave<2, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 3: split_wave<3, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 4: split_wave<4, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 5: split_wave<5, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 6: split_wave<6, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                case 7: split_wave<7, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                default: split_wave<8, ROUNDS, false>(idx, lab, Hw, out, s0, len, lane, first); break;
                }
            }
        }
        block_sync();
        if (tid == 0) misc[0] = tmpk[nseg];
        uint32_t* sw = cur;
        cur = nxt;
        nxt = sw;
        ++level;
    }
    block_sync();

    // idx[x] is the leaf index of the item that ends at x.  The elements come
    // from HBM straight into the staging copy (over the dead index arrays),
    // and every position gathers its item from there.
    uint32_t src[EMAX];
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
        const uint32_t x = r * kThreads + tid;
        if (x < m) src[r] = idx[x];
    }
    block_sync();
    {
        const uint32_t nw = m * static_cast<uint32_t>(sizeof(E) / 4);
        const global_t<uint32_t>* from = reinterpret_cast<const global_t<uint32_t>*>(X);
        uint32_t* to = reinterpret_cast<uint32_t*>(stage);
        copy_run_to_lds(from, to, nw, wv * 256u, kWaves * 256u, lane);
        __builtin_amdgcn_s_waitcnt(0);
    }
    block_sync();
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
        const uint32_t x = r * kThreads + tid;
        if (x < m) X[x] = stage[src[r]];
    }
}

// One size class of leaves, MINW waves per SIMD, in persistent workgroups:
// each takes the next leaf of the class from the work counter *qctr until
// *count leaves are taken.
template <typename E, int ROUNDS, int MINW, bool ATOMIC>
__global__ __launch_bounds__(kThreads, MINW) void k_leaf_persistent(const LeafDesc* __restrict__ leaves,
                                                                    const unsigned long long* __restrict__ count,
                                                                    unsigned long long* __restrict__ qctr,
                                                                    Params prm, uint32_t cap)
{
    extern __shared__ __align__(16) uint8_t smem[];
    // take[it & 1] holds the leaf of iteration it; thread 0 takes the next
    // leaf while the current one runs, so the atomic's latency is hidden.
    // Slot (it + 1) & 1 is written after every thread read it in iteration
    // it - 1 and read after the barriers that end iteration it.
    __shared__ unsigned long long take[2];
    const unsigned long long total = *count;
    if (threadIdx.x == 0) take[0] = atomicAdd(qctr, 1ull);
    block_sync();
    for (uint32_t it = 0;; ++it) {
        const unsigned long long i = take[it & 1u];
        if (i >= total) break;
        if (threadIdx.x == 0) take[(it + 1) & 1u] = atomicAdd(qctr, 1ull);
        leaf_body<E, ROUNDS, ATOMIC>(leaves[i], prm, cap, smem);
        block_sync();  // the next leaf reuses the LDS
    }
}

template <typename E>
__global__ void k_fy_global(const LeafDesc* __restrict__ items)
{
    if (threadIdx.x != 0) return;
    const LeafDesc ld = items[blockIdx.x];
    global_t<E>* X = elem_gptr<E>(ld.elem_off) + ld.base;
    const Key key = make_key(ld.seed, ld.stream_id);
    for (uint64_t i = ld.m - 1; i >= 1; --i) {
        const uint64_t p = ld.base + i;
        const uint32_t bound = static_cast<uint32_t>(i + 1);
        uint64_t j;
        if (bound <= 0x10000u) {
            const Word4 v = fy_short_block(key, ld.level, p >> 3, 0);
            j = fy_short_draw(key, ld.level, p, bound, half_of(v, static_cast<uint32_t>(p & 7)));
        } else {
            j = fy_long_draw(key, ld.level, p, bound);
        }
        const E a = X[i];
        X[i] = X[j];
        X[j] = a;
    }
}

// Leaf size classes of an element type: capacities (items) of the small and
// medium classes for the largest tile, and their register rounds.
template <typename E>
struct LeafClasses {
    static constexpr uint32_t kTmax = kTileBytesMax / sizeof(E);
    static constexpr int kRoundsL = static_cast<int>(kTmax / kThreads);
    static constexpr int kRoundsM = static_cast<int>((kTmax / 2 + kTmax / 32 + kThreads - 1) / kThreads);
    static constexpr int kRoundsS = static_cast<int>((kTmax / 4 + kTmax / 32 + kThreads - 1) / kThreads);
};

template <typename E, int ROUNDS, int MINW>
hipError_t leaf_class_persistent_t(const LeafDesc* leaves, const unsigned long long* count,
                                   unsigned long long* qctr, const Params& prm, uint32_t cap,
                                   hipStream_t stream)
{
    if (cap > static_cast<uint32_t>(ROUNDS) * kThreads) return hipErrorInvalidValue;
    const LeafLayout LL = leaf_layout(cap, sizeof(E), 1u << prm.kmax_log2, prm.n0);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // one kernel per rank method (the other method's split code would only
    // add registers)
    auto* kern = prm.rank_atomic ? &k_leaf_persistent<E, ROUNDS, MINW, true> : &k_leaf_persistent<E, ROUNDS, MINW, false>;
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kThreads,
                                                         LL.total);
    if (e != hipSuccess) return e;
    const uint32_t grid = static_cast<uint32_t>(std::max(1, cus) * std::max(1, per_cu));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), LL.total, stream, leaves, count, qctr, prm, cap);
    return hipGetLastError();
}

template <typename E>
hipError_t leaf_persistent_t(const LeafDesc* leaves, const unsigned long long* count, uint64_t stride,
                             const Params& prm, const uint32_t* caps, unsigned long long* qctr,
                             hipStream_t stream)
{
    using LC = LeafClasses<E>;
    hipError_t e;
    e = leaf_class_persistent_t<E, LC::kRoundsS, 8>(leaves, count, qctr, prm, caps[0], stream);
    if (e != hipSuccess) return e;
    e = leaf_class_persistent_t<E, LC::kRoundsM, 6>(leaves + stride, count + 1, qctr + 1, prm, caps[1], stream);
    if (e != hipSuccess) return e;
    return leaf_class_persistent_t<E, LC::kRoundsL, 4>(leaves + 2 * stride, count + 2, qctr + 2, prm, caps[2],
                                                       stream);
}

// Sort leaves into the three classes (order inside a class is immaterial:
// every leaf is finished independently).
constexpr int kClassThreads = 1024;

__global__ __launch_bounds__(kClassThreads) void k_leaf_classes(const LeafDesc* __restrict__ in,
                                                                uint64_t n, LeafDesc* __restrict__ out,
                                                                uint64_t stride, uint32_t cap_s,
                                                                uint32_t cap_m,
                                                                unsigned long long* __restrict__ count,
                                                                const unsigned long long* __restrict__ dn)
{
    if (dn) n = *dn;  // the device's leaf count (the grid covers an upper bound)
    // Slots are reserved with one atomic per class and workgroup: the waves'
    // counts are added up in LDS.  No early exit: every thread takes part in
    // the barriers.
    constexpr uint32_t kW = kClassThreads / 64;
    __shared__ uint32_t wcnt[3][kW];
    __shared__ unsigned long long wbase[3][kW];
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kClassThreads + threadIdx.x;
    LeafDesc d{};
    uint32_t c = 3;
    if (i < n) {
        d = in[i];
        c = d.m <= cap_s ? 0u : (d.m <= cap_m ? 1u : 2u);
    }
    uint64_t mask[3];
#pragma unroll
    for (uint32_t k = 0; k < 3; ++k) {
        mask[k] = __ballot(c == k);
        if (lane == 0) wcnt[k][wv] = static_cast<uint32_t>(__popcll(mask[k]));
    }
    block_sync();
    if (threadIdx.x < 3) {
        const uint32_t k = threadIdx.x;
        unsigned long long run = 0;
        for (uint32_t w = 0; w < kW; ++w) {
            wbase[k][w] = run;
            run += wcnt[k][w];
        }
        const unsigned long long b = run ? atomicAdd(&count[k], run) : 0ull;
        for (uint32_t w = 0; w < kW; ++w) wbase[k][w] += b;
    }
    block_sync();
    if (c < 3) out[c * stride + wbase[c][wv] + bits_below(mask[c])] = d;
}

template <typename E>
hipError_t fy_t(const LeafDesc* items, uint64_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fy_global<E>, dim3(static_cast<uint32_t>(n)), dim3(64), 0, stream, items);
    return hipGetLastError();
}

}  // namespace

void leaf_class_caps(uint32_t w, const Params& prm, uint32_t* caps)
{
    uint32_t rs = 0, rm = 0;
    switch (w) {
    case 4: rs = LeafClasses<uint32_t>::kRoundsS; rm = LeafClasses<uint32_t>::kRoundsM; break;
    case 8: rs = LeafClasses<uint64_t>::kRoundsS; rm = LeafClasses<uint64_t>::kRoundsM; break;
    default: rs = LeafClasses<Elem16>::kRoundsS; rm = LeafClasses<Elem16>::kRoundsM; break;
    }
    const uint32_t T = prm.tile, big = T - (1u << prm.kmax_log2);
    uint32_t cm = T / 2 + T / 32, cs = T / 4 + T / 32;
    if (cm > rm * kThreads) cm = rm * kThreads;
    if (cs > rs * kThreads) cs = rs * kThreads;
    if (cm > big) cm = big;
    if (cs > cm) cs = cm;
    caps[0] = cs;
    caps[1] = cm;
    caps[2] = big;
}

hipError_t launch_leaf_classes(const LeafDesc* in, uint64_t n, LeafDesc* out, uint64_t stride,
                               const uint32_t* caps, unsigned long long* count, hipStream_t stream,
                               const unsigned long long* dn)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_leaf_classes, dim3(static_cast<uint32_t>((n + kClassThreads - 1) / kClassThreads)),
                       dim3(kClassThreads), 0, stream, in, n, out, stride, caps[0], caps[1], count, dn);
    return hipGetLastError();
}

hipError_t launch_leaf_persistent(uint32_t w, const LeafDesc* leaves, const unsigned long long* dcount,
                                  uint64_t stride, const Params& prm, const uint32_t* caps,
                                  unsigned long long* qctr, hipStream_t stream)
{
    switch (w) {
    case 4: return leaf_persistent_t<uint32_t>(leaves, dcount, stride, prm, caps, qctr, stream);
    case 8: return leaf_persistent_t<uint64_t>(leaves, dcount, stride, prm, caps, qctr, stream);
    case 16: return leaf_persistent_t<Elem16>(leaves, dcount, stride, prm, caps, qctr, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename E, bool ATOMIC>
static hipError_t leaf_limits_method_t()
{
    using LC = LeafClasses<E>;
    hipError_t e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_leaf_persistent<E, LC::kRoundsS, 8, ATOMIC>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax - 64);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_leaf_persistent<E, LC::kRoundsM, 6, ATOMIC>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax - 64);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_leaf_persistent<E, LC::kRoundsL, 4, ATOMIC>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax - 64);
}

template <typename E>
static hipError_t leaf_limits_t()
{
    const hipError_t e = leaf_limits_method_t<E, true>();
    return e != hipSuccess ? e : leaf_limits_method_t<E, false>();
}

hipError_t set_leaf_lds_limits()
{
    hipError_t e = leaf_limits_t<uint32_t>();
    if (e != hipSuccess) return e;
    e = leaf_limits_t<uint64_t>();
    if (e != hipSuccess) return e;
    return leaf_limits_t<Elem16>();
}

hipError_t launch_fy_global(uint32_t w, const LeafDesc* items, uint64_t count, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    switch (w) {
    case 4: return fy_t<uint32_t>(items, count, stream);
    case 8: return fy_t<uint64_t>(items, count, stream);
    case 16: return fy_t<Elem16>(items, count, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ipss
