// Planning pass of a tiled level: the per-(tile, bucket) label counts that
// the rough pass (RoughScatter, arXiv 2302.03317 Sec. 3.3 and 4.1) would
// write, without moving any element.  With the level tables built from them
// it gives the exact sizes of every level, hence a call's exact workspace.
#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

namespace ipss {

namespace {

// Labels counted per (tile, bucket) without moving any element: the count
// table the rough pass would write, for planning a call's memory ahead of
// time.  The order of the counting does not matter, so LDS atomics do it.
constexpr int kCountThreads = 256;

__global__ __launch_bounds__(kCountThreads) void k_count(const SubDesc* __restrict__ subs,
                                                         const uint32_t* __restrict__ tile_sub,
                                                         const uint64_t* __restrict__ tile_pofs,
                                                         uint32_t* __restrict__ cnt_tab)
{
    __shared__ uint32_t hist[kKmax];
    __shared__ uint64_t plo[kKmax];
    __shared__ uint32_t pcap[kKmax];
    __shared__ uint32_t nblk[kKmax + 1];
    const uint32_t tid = threadIdx.x, wv = tid >> 6;
    const uint64_t g = blockIdx.x;
    const SubDesc sd = subs[tile_sub[g]];
    const uint64_t t = g - sd.tile_off;
    const uint32_t kappa = sd.kappa, k = 1u << kappa;
    const Key key = make_key(sd.seed, sd.stream_id);
    const TilePieces tp(sd.m, kappa, sd.tiles, t, tile_pofs + 2 * g);
    for (uint32_t b = tid; b < k; b += kCountThreads) {
        const Piece pc = tp.of(b);
        const uint64_t p0 = sd.base + pc.lo;
        plo[b] = p0;
        pcap[b] = static_cast<uint32_t>(pc.cap);
        nblk[b] = pc.cap ? static_cast<uint32_t>(((p0 + pc.cap - 1) >> 4) - (p0 >> 4) + 1) : 0u;
        hist[b] = 0;
    }
    block_sync();
    if (wv == 0) wave_exclusive_scan(nblk, k);
    block_sync();
    const uint32_t nblocks = nblk[k];
    for (uint32_t i = tid; i < nblocks; i += kCountThreads) {
        const uint32_t b = upper_index(nblk, k, i);
        const uint64_t p0 = plo[b];
        const uint64_t B = (p0 >> 4) + (i - nblk[b]);
        const Word4 v = label_block(key, sd.level, B);
        for (uint32_t j = 0; j < 16; ++j) {
            const uint64_t p = B * 16 + j;
            if (p >= p0 && p < p0 + pcap[b]) atomicAdd(&hist[block_byte(v, j) >> (8 - kappa)], 1u);
        }
    }
    block_sync();
    for (uint32_t b = tid; b < k; b += kCountThreads) cnt_tab[sd.tab_off + t * k + b] = hist[b];
}

}  // namespace

hipError_t launch_count(const SubDesc* subs, const uint32_t* tile_sub, const uint64_t* tile_pofs,
                        uint32_t* cnt_tab, uint64_t ntiles, hipStream_t stream)
{
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count, dim3(static_cast<uint32_t>(ntiles)), dim3(kCountThreads), 0, stream,
                       subs, tile_sub, tile_pofs, cnt_tab);
    return hipGetLastError();
}

}  // namespace ipss
