// Rough pass of a tiled level (RoughScatter, arXiv 2302.03317 Sec. 3.3 and
// Sec. 4.1): one workgroup per tile.  Tile t of a subproblem owns piece t of
// every one of the k equal regions.  It reads its pieces in order (piece of
// bucket 0 first, ascending positions inside a piece), gives every item its
// label and its stable rank among equal labels, and writes the tile back in
// place: an item of label l and rank r goes to slot r of the tile's piece of
// region l while that piece has room ("placed"); the remaining items of the
// tile ("staged") fill the tile's free slots, ordered by (label, rank).  The
// tile's per-bucket counts go to the level's count table; the fix-up kernels
// use them to route staged and displaced items.
//
// Memory path: every piece is one contiguous run in HBM, copied whole into an
// LDS staging array (direct global-to-LDS loads) and, after the permutation,
// copied back whole; the ranking works on the staging order.  HBM traffic per
// tile is one read and one write of its elements.  A tile needs
// T * w + ~8 KiB of LDS, so two workgroups share a CU and one's memory phase
// overlaps the other's ranking.
#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

namespace ipss {

namespace {

// A thread's R elements in registers.  16-byte elements are held as four
// arrays of words: an array of vectors would be left in scratch memory.
template <typename E, int R>
struct ElemRegs {
    E v[R];
    __device__ __forceinline__ E get(int r) const { return v[r]; }
    __device__ __forceinline__ void set(int r, const E& e) { v[r] = e; }
};

template <int R>
struct ElemRegs<uint4, R> {
    uint32_t x[R], y[R], z[R], w[R];
    __device__ __forceinline__ uint4 get(int r) const { return make_uint4(x[r], y[r], z[r], w[r]); }
    __device__ __forceinline__ void set(int r, const uint4& e)
    {
        x[r] = e.x;
        y[r] = e.y;
        z[r] = e.z;
        w[r] = e.w;
    }
};

// Stable ranks of one wave's rounds for KAPPA-bit labels.  Round r gives lane
// l the staging slot first + 64r; pk[r] receives label | rank << 8 where rank
// counts earlier items of the wave with the same label.
template <int KAPPA, int R>
__device__ __forceinline__ void rank_rounds(const uint8_t* lab, uint32_t* Hw, uint32_t first,
                                            uint32_t ts, uint32_t (&pk)[R])
{
    // labels of eight rounds are read ahead (slots past the tile read slot 0)
    constexpr int kAhead = R < 8 ? R : 8;
#pragma unroll
    for (int r0 = 0; r0 < R; r0 += kAhead) {
        uint32_t lb[kAhead];
#pragma unroll
        for (int i = 0; i < kAhead; ++i) {
            const uint32_t q = first + 64u * (r0 + i);
            lb[i] = lab[q < ts ? q : 0u];
        }
#pragma unroll
        for (int i = 0; i < kAhead; ++i) {
            const int r = r0 + i;
            const uint32_t q = first + 64u * r;
            uint32_t v = 0;
            if (q < ts) {
                const uint32_t l = lb[i];
                const uint64_t peers = match_label_bits<KAPPA>(l);
                const uint32_t below = bits_below(peers);
                const uint32_t old = Hw[l];
                if (below == 0) Hw[l] = old + static_cast<uint32_t>(__popcll(peers));
                v = l | ((old + below) << 8);
            }
            pk[r] = v;
        }
    }
}

// The same ranks from one LDS atomic add per item: the adds of one wave
// instruction that hit the same label's counter return the old counts in lane
// order (checked on the device before this path is chosen), which is the
// stable order.
template <int R>
__device__ __forceinline__ void rank_rounds_atomic(const uint8_t* lab, uint32_t* Hw, uint32_t first,
                                                   uint32_t ts, uint32_t (&pk)[R])
{
    constexpr int kAhead = R < 8 ? R : 8;
#pragma unroll
    for (int r0 = 0; r0 < R; r0 += kAhead) {
        uint32_t lb[kAhead];
#pragma unroll
        for (int i = 0; i < kAhead; ++i) {
            const uint32_t q = first + 64u * (r0 + i);
            lb[i] = lab[q < ts ? q : 0u];
        }
#pragma unroll
        for (int i = 0; i < kAhead; ++i) {
            const int r = r0 + i;
            const uint32_t q = first + 64u * r;
            uint32_t v = 0;
            if (q < ts) {
                const uint32_t l = lb[i];
                v = l | (atomicAdd(&Hw[l], 1u) << 8);
            }
            pk[r] = v;
        }
    }
}

// Byte j (0 .. 15) of a 16-byte block held as two 64-bit halves.
__device__ __forceinline__ uint8_t block_byte(uint64_t lo, uint64_t hi, int32_t j)
{
    const uint64_t h = (j & 8) ? hi : lo;
    return static_cast<uint8_t>(h >> (8 * (j & 7)));
}

// Checks on the device that LDS atomic adds of one wave instruction that hit
// the same address return their old values in lane order, for random label
// patterns (1 to 256 labels, all or some lanes active); out[0] counts lanes
// that saw any other value.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(256) void k_lane_order_probe(uint32_t trials,
                                                          unsigned long long* __restrict__ out)
{
    __shared__ uint32_t H[4 * 257];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t* Hw = H + wv * 257;
    unsigned long long bad = 0;
    for (uint32_t t = 0; t < trials; ++t) {
        const uint32_t h = probe_hash(0x51ED270Bu ^ probe_hash(blockIdx.x * 1000003u + t * 4u + wv));
        const uint32_t nl = 1u << (h % 9u);
        const uint32_t l = probe_hash(h + lane * 0x9E3779B9u) & (nl - 1u);
        const bool active = ((h >> 8) & 3u) != 0u || (probe_hash(h ^ lane) & 1u) != 0u;
        for (uint32_t j = lane; j < 257; j += 64) Hw[j] = 0;
        uint32_t o = 0;
        if (active) o = atomicAdd(&Hw[l], 1u);
        const uint64_t act = __ballot(active);
        uint32_t expect = 0;  // active lanes below with the same label
        for (uint32_t j = 0; j < 64; ++j) {  // every lane takes part in the shuffles
            const uint32_t lj = static_cast<uint32_t>(__shfl(static_cast<int>(l), static_cast<int>(j), 64));
            if (j < lane && ((act >> j) & 1u) && lj == l) ++expect;
        }
        if (active && o != expect) ++bad;
    }
    if (bad) atomicAdd(&out[0], bad);
}

template <typename E, int R, bool ATOMIC>
__global__ __launch_bounds__(kRoughThreads, 8) void k_rough(const SubDesc* __restrict__ subs,
                                                    const uint32_t* __restrict__ tile_sub,
                                                    const uint64_t* __restrict__ tile_pofs,
                                                    uint32_t* __restrict__ cnt_tab, Params prm,
                                                    const uint64_t* __restrict__ dsz)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wv = uniform(tid >> 6);  // the same in all lanes of a wave
    // tiles of the level: the grid, or the device's count for a level planned
    // on the device (the grid then covers an upper bound)
    const uint32_t ntl = dsz ? static_cast<uint32_t>(dsz[1]) : gridDim.x;
    if (blockIdx.x >= ntl) return;
    const uint64_t g = xcd_order(blockIdx.x, ntl);
    const SubDesc sd = subs[tile_sub[g]];
    const uint64_t t = g - sd.tile_off;
    const uint32_t kappa = sd.kappa, k = 1u << kappa;
    const uint32_t kmax = 1u << prm.kmax_log2;
    const uint32_t hs = k + 1;  // row stride of the per-wave counters
    const RoughLayout L = rough_layout(prm.tile, sizeof(E), kmax);
    constexpr uint32_t kWordsPerElem = sizeof(E) / 4;

    E* stage = reinterpret_cast<E*>(smem);
    uint8_t* lab = smem;                                                  // overlays stage
    uint16_t* fs = reinterpret_cast<uint16_t*>(smem);                    // overlays lab
    uint32_t* H = reinterpret_cast<uint32_t*>(smem + L.counts);          // overlays stage
    uint2* WT = reinterpret_cast<uint2*>(smem + L.slot_tab);              // overlays stage
    uint64_t* lo = reinterpret_cast<uint64_t*>(smem + L.tables);
    uint32_t* qoff = reinterpret_cast<uint32_t*>(lo + kmax + 1);
    uint32_t* cap = qoff + kmax + 1;
    uint32_t* fill = cap + kmax + 1;
    uint32_t* ovt = fill + kmax + 1;
    uint32_t* hot = ovt + kmax + 1;
    uint32_t* nblk = hot + kmax + 1;

    global_t<E>* X = elem_gptr<E>(sd.elem_off) + sd.base;
    const uint64_t pbase = sd.base;
    const Key key = make_key(sd.seed, sd.stream_id);

    // Pieces -> staging, one contiguous run each, straight into LDS.  A
    // piece's bounds and staging offset have closed forms (TilePieces), so
    // every wave sends its pieces' loads before any table is built.  Wave wv
    // takes the consecutive pieces [wv k / 16, (wv + 1) k / 16): a piece's
    // region end and staging end are the next one's starts, so the closed
    // forms (64-bit products on the scalar unit) are evaluated once per piece.
    const TilePieces tp(sd.m, kappa, sd.tiles, t, tile_pofs + 2 * g);
    const uint32_t ts = tp.start(k);  // items of the tile
    {
        static_assert(kRoughWaves == 16, "pieces per wave: k / 16");
        const global_t<uint32_t>* src = reinterpret_cast<const global_t<uint32_t>*>(X);
        uint32_t* dst = reinterpret_cast<uint32_t*>(stage);
        const uint32_t b0 = (wv * k) >> 4, b1 = ((wv + 1) * k) >> 4;
        uint64_t e0 = tp.region_start(b0);
        uint32_t st = tp.start(b0);
        for (uint32_t b = b0; b < b1; ++b) {
            const uint64_t e1 = tp.region_start(b + 1);
            const Piece pc = tp.of_region(e0, e1);
            const uint32_t nw = static_cast<uint32_t>(pc.cap) * kWordsPerElem;
            const uint64_t s0 = pc.lo * kWordsPerElem;
            const uint32_t d0 = st * kWordsPerElem;
            // 4-byte loads: for these short runs they measured faster than
            // the 16-byte form the leaves use
            for (uint32_t j = 0; j < nw; j += 64) {
                if (j + lane < nw)
                    __builtin_amdgcn_global_load_lds(src + s0 + j + lane, dst + d0 + j, 4, 0, 0);
            }
            st += static_cast<uint32_t>(pc.cap);
            e0 = e1;
        }
    }

    // While the loads are in flight: the piece tables (waves 1..) and, in
    // wave 0, the label blocks (16 positions per Philox call) each piece
    // touches, scanned in registers (lane l takes pieces 4l .. 4l + 3).  The
    // barrier here waits for LDS operations only, not for the loads.
    static_assert(kKmax <= 4 * 64, "wave 0 takes four pieces per lane");
    if (wv == 0) {
        uint32_t nb[4];
        uint32_t own = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t b = 4 * lane + q;
            nb[q] = 0;
            if (b < k) {
                const Piece pc = tp.of(b);
                if (pc.cap) {
                    const uint64_t p0 = pbase + pc.lo, p1 = p0 + pc.cap - 1;
                    nb[q] = static_cast<uint32_t>((p1 >> 4) - (p0 >> 4) + 1);
                }
            }
            own += nb[q];
        }
        const uint32_t incl = wave_inclusive_sum(own);
        uint32_t run = incl - own;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t b = 4 * lane + q;
            if (b < k) nblk[b] = run;
            run += nb[q];
        }
        if (lane == 63) nblk[k] = incl;
    } else {
        for (uint32_t b = tid - 64; b < k; b += kRoughThreads - 64) {
            const Piece pc = tp.of(b);
            lo[b] = pc.lo;
            cap[b] = static_cast<uint32_t>(pc.cap);
            qoff[b] = tp.start(b);
        }
    }
    lds_barrier();
    const uint32_t nblocks = nblk[k];

    // While the loads are in flight: the Philox blocks of this thread's label
    // blocks (a tile touches at most T/16 + 2k <= 2 * kRoughThreads blocks).
    constexpr int kBlk = 2;
    static_assert((kTileBytesMax / 4) / 16 + 2 * kKmax <= kBlk * kRoughThreads, "label blocks per thread");
    // The piece of label block i: the last piece whose blocks start at or
    // before i (pieces without blocks share their start with the next one).
    Word4 lw[kBlk];
    uint32_t bb[kBlk];
#pragma unroll
    for (int u = 0; u < kBlk; ++u) {
        const uint32_t i = tid + u * kRoughThreads;
        bb[u] = 0;
        if (i < nblocks) {
            const uint32_t b = upper_index(nblk, k, i);
            bb[u] = b;
            lw[u] = label_block(key, sd.level, ((pbase + lo[b]) >> 4) + (i - nblk[b]));
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    block_sync();

    // Wave wv owns read-order slots [wv * 64R, (wv + 1) * 64R); round r gives
    // lane l the slot wv * 64R + 64r + l.
    const uint32_t first = wv * 64u * R + lane;
    // Slots past the tile's end are read too (the staging area spans all
    // kRoughThreads * R slots) and ignored: one base address, no branches,
    // every read at a constant offset.
    ElemRegs<E, R> data;
#pragma unroll
    for (int r = 0; r < R; ++r) data.set(r, stage[first + 64u * r]);
    block_sync();  // staging is free: labels and per-wave counters overlay it

    // Labels in staging order: block i of the tile belongs to piece bb[u];
    // d is the offset of its first position from the piece start.
    const uint32_t sh = 8 - kappa;
#pragma unroll
    for (int u = 0; u < kBlk; ++u) {
        const uint32_t i = tid + u * kRoughThreads;
        if (i >= nblocks) continue;
        const uint32_t b = bb[u];
        const uint64_t p0 = pbase + lo[b];
        const uint64_t B = (p0 >> 4) + (i - nblk[b]);
        const Word4 v = lw[u];
        const int32_t d = static_cast<int32_t>(static_cast<uint32_t>(B << 4) - static_cast<uint32_t>(p0));
        const int32_t c = static_cast<int32_t>(cap[b]);
        const int32_t q0 = static_cast<int32_t>(qoff[b]) + d;
        // The block's 16 label bytes (top kappa bits of every byte) sit at
        // staging bytes q0 .. q0 + 15, of which [s0, s1) lie in the piece.
        // One code path for every block: the aligned words fully inside
        // [s0, s1) as words, the at most three bytes before the first and
        // after the last such word one by one (neighbouring blocks and
        // pieces write the other bytes of those words).
        const uint32_t msk = 0x01010101u * (0xFFu >> sh);
        const uint32_t L0 = (v.x >> sh) & msk, L1 = (v.y >> sh) & msk;
        const uint32_t L2 = (v.z >> sh) & msk, L3 = (v.w >> sh) & msk;
        const int32_t s0 = q0 + (d < 0 ? -d : 0);
        const int32_t s1 = q0 + (c - d < 16 ? c - d : 16);
        const int32_t wb = q0 >> 2;  // the word holding byte q0 (floor)
        const uint32_t a = static_cast<uint32_t>(q0) & 3u;
        const int32_t up0 = (s0 + 3) & ~3;  // first word boundary at or after s0
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const uint32_t lo_w = m == 1 ? L0 : m == 2 ? L1 : m == 3 ? L2 : m == 4 ? L3 : 0u;
            const uint32_t hi_w = m == 0 ? L0 : m == 1 ? L1 : m == 2 ? L2 : m == 3 ? L3 : 0u;
            const uint32_t W = a ? __builtin_amdgcn_alignbyte(hi_w, lo_w, 4u - a) : hi_w;
            const int32_t p = 4 * (wb + m);
            if (p >= s0 && p + 4 <= s1) reinterpret_cast<uint32_t*>(lab)[wb + m] = W;
        }
        const int32_t lead_end = up0 < s1 ? up0 : s1;
        const int32_t tail_beg = (s1 & ~3) > up0 ? (s1 & ~3) : up0;
        const uint64_t Llo = (static_cast<uint64_t>(L1) << 32) | L0;
        const uint64_t Lhi = (static_cast<uint64_t>(L3) << 32) | L2;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int32_t p = s0 + e;
            if (p < lead_end) lab[p] = block_byte(Llo, Lhi, p - q0);
            const int32_t p2 = tail_beg + e;
            if (p2 < s1) lab[p2] = block_byte(Llo, Lhi, p2 - q0);
        }
    }
    for (uint32_t i = tid; i < kRoughWaves * hs; i += kRoughThreads) H[i] = 0;
    block_sync();

    uint32_t pk[R];
    uint32_t* Hw = H + wv * hs;
    if constexpr (ATOMIC) {
        rank_rounds_atomic<R>(lab, Hw, first, ts, pk);
    } else {
        switch (kappa) {
        case 1: rank_rounds<1, R>(lab, Hw, first, ts, pk); break;
        case 2: rank_rounds<2, R>(lab, Hw, first, ts, pk); break;
        case 3: rank_rounds<3, R>(lab, Hw, first, ts, pk); break;
        case 4: rank_rounds<4, R>(lab, Hw, first, ts, pk); break;
        case 5: rank_rounds<5, R>(lab, Hw, first, ts, pk); break;
        case 6: rank_rounds<6, R>(lab, Hw, first, ts, pk); break;
        case 7: rank_rounds<7, R>(lab, Hw, first, ts, pk); break;
        default: rank_rounds<8, R>(lab, Hw, first, ts, pk); break;
        }
    }
    block_sync();

    // Per label: offsets of the waves, the tile's count, fill, overflow, holes.
    for (uint32_t l = tid; l < k; l += kRoughThreads) {
        uint32_t run = 0;
        for (int w = 0; w < kRoughWaves; ++w) {
            const uint32_t v = H[w * hs + l];
            H[w * hs + l] = run;
            run += v;
        }
        cnt_tab[sd.tab_off + t * k + l] = run;
        const uint32_t f = run < cap[l] ? run : cap[l];
        fill[l] = f;
        ovt[l] = run - f;
        hot[l] = cap[l] - f;
    }
    block_sync();
    if (wv == 0) wave_exclusive_scan(ovt, k);
    if (wv == 1) wave_exclusive_scan(hot, k);
    block_sync();

    // Free slots of the pieces, in order, as a list (the label area is dead),
    // and the slot table of every (wave, label): an item of rank rr within
    // its wave is placed at A + rr if rr < B, else it is staged item C + rr
    // of the tile (A = piece start + earlier waves' count, B = capacity left
    // to the wave, C = staged items of smaller labels - B).
    const uint32_t nfree = hot[k];
    const bool use_list = !prm.slot_search && nfree <= prm.tile / 2;
    if (use_list) {
        // kRoughThreads / k threads per piece, each writing every
        // (kRoughThreads / k)-th of its holes
        static_assert(kRoughThreads == 1024 && kKmax <= 1024, "threads per piece: 2^(10 - kappa)");
        const uint32_t tsh = 10u - kappa;
        const uint32_t b = tid >> tsh;
        const uint32_t base = hot[b], f0 = qoff[b] + fill[b], nh = cap[b] - fill[b];
        for (uint32_t j = tid & ((1u << tsh) - 1u); j < nh; j += 1u << tsh)
            fs[base + j] = static_cast<uint16_t>(f0 + j);
    }
    for (uint32_t i = tid; i < kRoughWaves * k; i += kRoughThreads) {
        const uint32_t w = i >> kappa, l = i & (k - 1);
        const uint32_t h = H[w * hs + l];
        const int32_t B = static_cast<int32_t>(cap[l]) - static_cast<int32_t>(h);
        const uint32_t A = qoff[l] + h;
        WT[w * k + l] = make_uint2((A & 0xFFFFu) | (static_cast<uint32_t>(B) << 16),
                                   ovt[l] - static_cast<uint32_t>(B));
    }
    block_sync();

    // Destination slot in staging order.
    if (use_list) {
        // every round, also those past the tile (pk = 0 there: label 0,
        // rank 0), so that the reads of all rounds overlap; every read stays
        // inside the table and the free list
        const uint32_t fmax = nfree ? nfree - 1 : 0u;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t l = pk[r] & 0xFFu, rr = pk[r] >> 8;
            const uint2 e = WT[wv * k + (l & (k - 1))];
            const bool placed = static_cast<int32_t>(rr) < (static_cast<int32_t>(e.x) >> 16);
            const uint32_t fi = e.y + rr;
            const uint32_t f = fs[placed ? 0u : (fi < fmax ? fi : fmax)];
            pk[r] = placed ? (e.x & 0xFFFFu) + rr : f;
        }
    } else {
        // every round again, without branches: the piece of a staged item
        // is the last one whose holes start at or before it (kappa halving
        // steps over the hole offsets, k being a power of two)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t l = pk[r] & 0xFFu, rr = pk[r] >> 8;
            const uint2 e = WT[wv * k + (l & (k - 1))];
            const bool placed = static_cast<int32_t>(rr) < (static_cast<int32_t>(e.x) >> 16);
            const uint32_t s = e.y + rr;
            uint32_t bb = 0;
            for (uint32_t step = k >> 1; step; step >>= 1) bb = hot[bb + step] <= s ? bb + step : bb;
            pk[r] = placed ? (e.x & 0xFFFFu) + rr : qoff[bb] + fill[bb] + (s - hot[bb]);
        }
    }
    block_sync();  // labels, free list and counters are dead from here on
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t q = first + 64u * r;
        if (q < ts) stage[pk[r]] = data.get(r);
    }
    block_sync();

    // Staging -> pieces, one contiguous run each.
    {
        global_t<uint32_t>* dst = reinterpret_cast<global_t<uint32_t>*>(X);
        const uint32_t* src = reinterpret_cast<const uint32_t*>(stage);
        for (uint32_t b = wv; b < k; b += kRoughWaves) {
            const uint32_t nw = cap[b] * kWordsPerElem;
            const uint64_t d0 = lo[b] * kWordsPerElem;
            const uint32_t s0 = qoff[b] * kWordsPerElem;
            for (uint32_t j = lane; j < nw; j += 64) dst[d0 + j] = src[s0 + j];
        }
    }
}

template <typename E>
hipError_t launch_rough_t(const SubDesc* subs, const uint32_t* tile_sub, const uint64_t* tile_pofs,
                          uint32_t* cnt_tab, uint64_t ntiles, const Params& prm, hipStream_t stream,
                          const uint64_t* dsz)
{
    constexpr int R = static_cast<int>(kTileBytesMax / (sizeof(E) * kRoughThreads));
    const RoughLayout L = rough_layout(prm.tile, sizeof(E), 1u << prm.kmax_log2);
    if (ntiles == 0) return hipSuccess;
    // one kernel per rank method (the other method's code would only add
    // registers)
    auto* kern = prm.rank_atomic ? &k_rough<E, R, true> : &k_rough<E, R, false>;
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(ntiles)), dim3(kRoughThreads), L.total, stream, subs,
                       tile_sub, tile_pofs, cnt_tab, prm, dsz);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_rough(uint32_t w, const SubDesc* subs, const uint32_t* tile_sub,
                        const uint64_t* tile_pofs, uint32_t* cnt_tab, uint64_t ntiles,
                        const Params& prm, hipStream_t stream, const uint64_t* dsz)
{
    switch (w) {
    case 4: return launch_rough_t<uint32_t>(subs, tile_sub, tile_pofs, cnt_tab, ntiles, prm, stream, dsz);
    case 8: return launch_rough_t<uint64_t>(subs, tile_sub, tile_pofs, cnt_tab, ntiles, prm, stream, dsz);
    case 16: return launch_rough_t<Elem16>(subs, tile_sub, tile_pofs, cnt_tab, ntiles, prm, stream, dsz);
    default: return hipErrorInvalidValue;
    }
}

hipError_t probe_lds_lane_order(hipStream_t stream, unsigned long long* d, bool* lane_ordered)
{
    *lane_ordered = false;
    unsigned long long h = 1;
    hipError_t e = hipMemsetAsync(d, 0, sizeof(unsigned long long), stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_lane_order_probe, dim3(1024), dim3(256), 0, stream, 64u, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    *lane_ordered = h == 0;
    return hipSuccess;
}

template <typename E, bool ATOMIC>
static hipError_t rough_limit_t()
{
    constexpr int R = static_cast<int>(kTileBytesMax / (sizeof(E) * kRoughThreads));
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rough<E, R, ATOMIC>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
}

hipError_t set_rough_lds_limits()
{
    hipError_t e = rough_limit_t<uint32_t, true>();
    if (e == hipSuccess) e = rough_limit_t<uint32_t, false>();
    if (e == hipSuccess) e = rough_limit_t<uint64_t, true>();
    if (e == hipSuccess) e = rough_limit_t<uint64_t, false>();
    if (e == hipSuccess) e = rough_limit_t<Elem16, true>();
    if (e == hipSuccess) e = rough_limit_t<Elem16, false>();
    return e;
}

}  // namespace ipss
