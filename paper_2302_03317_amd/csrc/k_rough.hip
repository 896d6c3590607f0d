// Rough pass of a tiled level (RoughScatter, arXiv 2302.03317 Sec. 3.2 and
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
// HBM traffic per tile: one read and one write of its elements, both streamed
// through a staging copy in LDS so that global accesses stay contiguous.
#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

namespace ipss {

template <typename E, int EMAX>
__global__ __launch_bounds__(kThreads) void k_rough(uint8_t* __restrict__ buf,
                                                    const SubDesc* __restrict__ subs,
                                                    const uint32_t* __restrict__ tile_sub,
                                                    uint32_t* __restrict__ cnt_tab, uint64_t seed,
                                                    Params prm)
{
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    const uint64_t g = blockIdx.x;
    const SubDesc sd = subs[tile_sub[g]];
    const uint64_t t = g - sd.tile_off;
    const uint32_t kappa = sd.kappa, k = 1u << kappa;
    const uint32_t kmax = 1u << prm.kmax_log2;
    const RoughLayout L = rough_layout(prm.tile, sizeof(E), kmax);

    E* stage = reinterpret_cast<E*>(smem);
    uint8_t* lab = smem;                                                    // overlays stage
    uint32_t* H = reinterpret_cast<uint32_t*>(smem + align16(prm.tile));   // overlays stage
    uint64_t* lo = reinterpret_cast<uint64_t*>(smem + L.tables);
    uint32_t* qoff = reinterpret_cast<uint32_t*>(lo + kmax + 1);
    uint32_t* cap = qoff + kmax + 1;
    uint32_t* fill = cap + kmax + 1;
    uint32_t* ovt = fill + kmax + 1;
    uint32_t* hot = ovt + kmax + 1;
    uint32_t* nblk = hot + kmax + 1;

    E* X = reinterpret_cast<E*>(buf) + sd.elem_off + sd.base;
    const uint64_t pbase = sd.base;
    const Key key = make_key(seed, sd.stream_id);

    // Pieces of this tile, their offsets in read order, and the label blocks
    // (16 positions per Philox call) each piece touches.
    for (uint32_t b = tid; b < k; b += kThreads) {
        const Piece pc = piece_of(sd.m, kappa, sd.tiles, t, b);
        lo[b] = pc.lo;
        cap[b] = static_cast<uint32_t>(pc.cap);
        qoff[b] = static_cast<uint32_t>(pc.cap);
        uint32_t nb = 0;
        if (pc.cap) {
            const uint64_t p0 = pbase + pc.lo, p1 = p0 + pc.cap - 1;
            nb = static_cast<uint32_t>((p1 >> 4) - (p0 >> 4) + 1);
        }
        nblk[b] = nb;
    }
    __syncthreads();
    if (wv == 0) wave_exclusive_scan(qoff, k);
    if (wv == 1) wave_exclusive_scan(nblk, k);
    __syncthreads();
    const uint32_t ts = qoff[k];
    const uint32_t nblocks = nblk[k];

    for (uint32_t i = tid; i < nblocks; i += kThreads) {
        const uint32_t b = upper_index(nblk, k, i);
        const uint64_t p0 = pbase + lo[b];
        const uint64_t p1 = p0 + cap[b];
        const uint64_t B = (p0 >> 4) + (i - nblk[b]);
        const Word4 v = label_block(key, sd.level, B);
        const uint32_t qb = qoff[b];
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) {
            const uint64_t p = B * 16 + j;
            if (p >= p0 && p < p1)
                lab[qb + static_cast<uint32_t>(p - p0)] =
                    static_cast<uint8_t>(block_byte(v, j) >> (8 - kappa));
        }
    }
    for (uint32_t i = tid; i < kWaves * k; i += kThreads) H[i] = 0;
    __syncthreads();

    // Wave wv owns read-order slots [wv*per_wave, (wv+1)*per_wave); round r
    // gives lane l the slot wv*per_wave + 64r + l.
    const uint32_t per_wave = ((ts + kWaves * 64 - 1) / (kWaves * 64)) * 64;
    const uint32_t rounds = per_wave / 64;  // <= EMAX: the host keeps T <= EMAX * kThreads
    const uint32_t first = wv * per_wave + lane;

    E data[EMAX];
    uint32_t pk[EMAX];
    uint32_t pb = 0;
    if (first < ts) pb = upper_index(qoff, k, first);
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
        if (static_cast<uint32_t>(r) < rounds) {
            const uint32_t q = first + 64u * r;
            if (q < ts) {
                while (qoff[pb + 1] <= q) ++pb;
                data[r] = X[lo[pb] + (q - qoff[pb])];
            }
        }
    }

    // Stable ranks: labels of one round are matched with kappa ballots; the
    // wave keeps a running count per label.
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
        if (static_cast<uint32_t>(r) < rounds) {
            const uint32_t q = first + 64u * r;
            const bool valid = q < ts;
            const uint32_t l = valid ? lab[q] : 0u;
            uint64_t peers = __ballot(valid);
            for (uint32_t i = 0; i < kappa; ++i) {
                const bool bit = (l >> i) & 1u;
                const uint64_t mb = __ballot(bit);
                peers &= bit ? mb : ~mb;
            }
            const uint32_t below = bits_below(peers);
            const uint32_t total = static_cast<uint32_t>(__popcll(peers));
            uint32_t old = 0;
            if (valid) old = H[wv * k + l];
            if (valid && below == 0) H[wv * k + l] = old + total;
            pk[r] = l | ((old + below) << 8);
        }
    }
    __syncthreads();

    // Per label: offsets of the waves, the tile's count, fill, overflow, holes.
    for (uint32_t l = tid; l < k; l += kThreads) {
        uint32_t run = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t v = H[w * k + l];
            H[w * k + l] = run;
            run += v;
        }
        cnt_tab[sd.tab_off + t * k + l] = run;
        const uint32_t f = run < cap[l] ? run : cap[l];
        fill[l] = f;
        ovt[l] = run - f;
        hot[l] = cap[l] - f;
    }
    __syncthreads();
    if (wv == 0) wave_exclusive_scan(ovt, k);
    if (wv == 1) wave_exclusive_scan(hot, k);
    __syncthreads();

    // Destination slot in read order: placed items at the front of their
    // label's piece; staged items, ordered by (label, rank), into the free
    // slots of the pieces taken in order.
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
        if (static_cast<uint32_t>(r) < rounds) {
            const uint32_t q = first + 64u * r;
            if (q < ts) {
                const uint32_t l = pk[r] & 0xFFu;
                const uint32_t rr = H[wv * k + l] + (pk[r] >> 8);
                uint32_t slot;
                if (rr < cap[l]) {
                    slot = qoff[l] + rr;
                } else {
                    const uint32_t s = ovt[l] + (rr - cap[l]);
                    const uint32_t bb = upper_index(hot, k, s);
                    slot = qoff[bb] + fill[bb] + (s - hot[bb]);
                }
                pk[r] = slot;
            }
        }
    }
    __syncthreads();  // labels and per-wave counts are dead from here on
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
        if (static_cast<uint32_t>(r) < rounds) {
            const uint32_t q = first + 64u * r;
            if (q < ts) stage[pk[r]] = data[r];
        }
    }
    __syncthreads();
    if (first < ts) pb = upper_index(qoff, k, first);
#pragma unroll
    for (int r = 0; r < EMAX; ++r) {
        if (static_cast<uint32_t>(r) < rounds) {
            const uint32_t q = first + 64u * r;
            if (q < ts) {
                while (qoff[pb + 1] <= q) ++pb;
                X[lo[pb] + (q - qoff[pb])] = stage[q];
            }
        }
    }
}

template <typename E>
hipError_t launch_rough_t(uint8_t* buf, const SubDesc* subs, const uint32_t* tile_sub,
                          uint32_t* cnt_tab, uint64_t ntiles, uint64_t seed, const Params& prm,
                          hipStream_t stream)
{
    constexpr int EMAX = static_cast<int>(kTileBytesMax / (sizeof(E) * kThreads));
    const RoughLayout L = rough_layout(prm.tile, sizeof(E), 1u << prm.kmax_log2);
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_rough<E, EMAX>), dim3(static_cast<uint32_t>(ntiles)), dim3(kThreads),
                       L.total, stream, buf, subs, tile_sub, cnt_tab, seed, prm);
    return hipGetLastError();
}

hipError_t launch_rough(uint32_t w, uint8_t* buf, const SubDesc* subs, const uint32_t* tile_sub,
                        uint32_t* cnt_tab, uint64_t ntiles, uint64_t seed, const Params& prm,
                        hipStream_t stream)
{
    switch (w) {
    case 4: return launch_rough_t<uint32_t>(buf, subs, tile_sub, cnt_tab, ntiles, seed, prm, stream);
    case 8: return launch_rough_t<uint64_t>(buf, subs, tile_sub, cnt_tab, ntiles, seed, prm, stream);
    case 16: return launch_rough_t<Elem16>(buf, subs, tile_sub, cnt_tab, ntiles, seed, prm, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t set_rough_lds_limits()
{
    hipError_t e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rough<uint32_t, 32>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rough<uint64_t, 16>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rough<Elem16, 8>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytesMax);
}

}  // namespace ipss
