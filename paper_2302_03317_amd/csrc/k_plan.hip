// Planning of a batched call's first level on the device, for the batched
// call that is only enqueued (no host synchronisation, so a caller can
// capture it into a HIP graph): from the arrays' offsets in device memory,
// which arrays take a tiled level (their tiles, table rows and buckets, laid
// out in array order) and which are finished in LDS right away.  The same
// plan the host makes for the blocking calls (arXiv 2302.03317 Sec. 3.5:
// every array is its own ScatterShuffle; Sec. 4.1: a tiled level is cut into
// subtasks that own a piece of every bucket).
#include "common.hpp"
#include "kernels.hpp"

namespace ipss {

namespace {

constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;
constexpr int kPlanSums = 7;  // tiles, table rows, chunks, chunk rows, buckets, tiled arrays, leaves

// Bucket-count exponent of a subproblem of m items (the κ schedule).
__device__ __forceinline__ uint32_t kappa_dev(uint64_t m, bool tiled, const Params& p)
{
    uint64_t g = tiled ? p.tile / 2 : p.n0 / 2;
    if (g < 1) g = 1;
    uint32_t r = 1;
    uint64_t reach = 2 * g;
    while (reach < m) {
        reach *= 2;
        ++r;
    }
    const uint32_t h = (r + p.kmax_log2 - 1) / p.kmax_log2;
    const uint32_t kap = (r + h - 1) / h;
    return kap < p.kmax_log2 ? kap : p.kmax_log2;
}

struct ArrayPlan {
    uint64_t n;
    uint32_t kind;  // 0 nothing to do, 1 leaf, 2 tiled
    uint32_t kappa;
    uint64_t tiles, chunks;
};

__device__ __forceinline__ ArrayPlan plan_array(const uint64_t* off, uint64_t j, const Params& p)
{
    ArrayPlan a{};
    a.n = off[j + 1] - off[j];
    const uint64_t tile_limit = p.tile - (1u << p.kmax_log2);
    if (a.n < 2) return a;
    if (a.n <= tile_limit) {
        a.kind = 1;
        return a;
    }
    a.kind = 2;
    a.kappa = kappa_dev(a.n, true, p);
    const uint64_t k = 1ull << a.kappa;
    a.tiles = (a.n + (p.tile - k) - 1) / (p.tile - k);
    a.chunks = (a.tiles + kChunk - 1) / kChunk;
    return a;
}

__device__ __forceinline__ uint64_t wave_incl64(uint64_t v, uint32_t lane)
{
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// One workgroup.  Thread t plans arrays [t * per, (t + 1) * per); the
// per-thread sums are scanned across the workgroup; every tiled array gets
// the next subproblem slot and its ranges, every small array a leaf slot.
// dsz receives {subproblems, tiles, chunks, buckets}; counters[0] the number
// of leaves (children are appended after them), counters[2] their items.
// When a size exceeds its bound (or an array exceeds max_elems), err is set
// and nothing is planned, so that no later kernel of the call does anything.
__global__ __launch_bounds__(kPlanThreads) void k_plan_batched(
    const uint64_t* __restrict__ off, uint64_t count, uint64_t elem_base, uint64_t seed, Params prm,
    uint64_t max_elems, uint64_t max_tiles, uint64_t max_chunks, uint64_t max_buckets, uint64_t total_elems,
    SubDesc* __restrict__ subs, LeafDesc* __restrict__ leaves, unsigned long long* __restrict__ counters,
    uint64_t* __restrict__ dsz, uint32_t* __restrict__ err)
{
    __shared__ uint64_t wsum[kPlanSums + 1][kPlanWaves];
    __shared__ uint64_t wtot[kPlanSums + 1];
    __shared__ uint32_t bad;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    // the arrays must lie inside the first total_elems elements
    if (tid == 0) bad = off[count] > total_elems ? 1u : 0u;
    block_sync();
    const uint64_t per = (count + kPlanThreads - 1) / kPlanThreads;
    const uint64_t j0 = tid * per < count ? tid * per : count;
    const uint64_t j1 = j0 + per < count ? j0 + per : count;
    uint64_t v[kPlanSums] = {0, 0, 0, 0, 0, 0, 0};
    uint64_t elems = 0;
    for (uint64_t j = j0; j < j1; ++j) {
        if (off[j + 1] < off[j]) {
            bad = 1;
            continue;
        }
        const ArrayPlan a = plan_array(off, j, prm);
        elems += a.n;
        if (a.n > max_elems) bad = 1;
        if (a.kind == 2) {
            const uint64_t k = 1ull << a.kappa;
            v[0] += a.tiles;
            v[1] += a.tiles * k;
            v[2] += a.chunks;
            v[3] += a.chunks * k;
            v[4] += k;
            v[5] += 1;
        } else if (a.kind == 1) {
            v[6] += 1;
        }
    }
    // exclusive prefix of every sum over the threads: within each wave, then
    // over the waves (wave 0 scans the per-wave sums in place; the last row
    // holds the items of the arrays)
    uint64_t pre[kPlanSums];
#pragma unroll
    for (int q = 0; q < kPlanSums; ++q) {
        const uint64_t incl = wave_incl64(v[q], lane);
        pre[q] = incl - v[q];
        if (lane == 63) wsum[q][wv] = incl;
    }
    {
        const uint64_t incl = wave_incl64(elems, lane);
        if (lane == 63) wsum[kPlanSums][wv] = incl;
    }
    block_sync();
    if (wv == 0) {
#pragma unroll 1
        for (int q = 0; q <= kPlanSums; ++q) {
            const uint64_t x = lane < kPlanWaves ? wsum[q][lane] : 0;
            const uint64_t incl = wave_incl64(x, lane);
            if (lane < kPlanWaves) wsum[q][lane] = incl - x;
            if (lane == kPlanWaves - 1) wtot[q] = incl;
        }
    }
    block_sync();
#pragma unroll
    for (int q = 0; q < kPlanSums; ++q) pre[q] += wsum[q][wv];
    const bool over = wtot[0] > max_tiles || wtot[2] > max_chunks || wtot[4] > max_buckets ||
                      wtot[5] > count || wtot[kPlanSums] > total_elems;
    if (over || bad) {
        if (tid == 0) {
            *err = 32u;
            dsz[0] = dsz[1] = dsz[2] = dsz[3] = 0;
            counters[0] = 0;
        }
        return;
    }
    uint64_t leaf_items = 0;
    for (uint64_t j = j0; j < j1; ++j) {
        const ArrayPlan a = plan_array(off, j, prm);
        if (a.kind == 2) {
            const uint64_t k = 1ull << a.kappa;
            SubDesc d{};
            d.elem_off = elem_base + off[j];
            d.base = 0;
            d.m = a.n;
            d.seed = seed;
            d.kappa = a.kappa;
            d.tiles = a.tiles;
            d.tile_off = pre[0];
            d.tab_off = pre[1];
            d.chunk_off = pre[2];
            d.chtab_off = pre[3];
            d.bk_off = static_cast<uint32_t>(pre[4]);
            d.level = 0;
            d.stream_id = static_cast<uint32_t>(j);
            d.owner = 0;
            subs[pre[5]] = d;
            pre[0] += a.tiles;
            pre[1] += a.tiles * k;
            pre[2] += a.chunks;
            pre[3] += a.chunks * k;
            pre[4] += k;
            pre[5] += 1;
        } else if (a.kind == 1) {
            leaves[pre[6]] = LeafDesc{elem_base + off[j], 0, a.n, seed, 0, static_cast<uint32_t>(j), 0, 0};
            pre[6] += 1;
            leaf_items += a.n;
        }
    }
    if (leaf_items) atomicAdd(&counters[2], static_cast<unsigned long long>(leaf_items));
    if (tid == 0) {
        dsz[0] = wtot[5];
        dsz[1] = wtot[0];
        dsz[2] = wtot[2];
        dsz[3] = wtot[4];
        counters[0] = wtot[6];
    }
}

// Zero `words` 32-bit words (a kernel rather than a memset node, for callers
// that capture the call into a graph).
__global__ void k_zero_words(uint32_t* __restrict__ p, uint32_t words)
{
    for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
}

// A child too large for one tile would need a second tiled level, which the
// enqueue-only call does not run: report it.
__global__ void k_check_one_level(const unsigned long long* __restrict__ counters, uint32_t* __restrict__ err)
{
    if (threadIdx.x == 0 && counters[1] != 0) atomicOr(err, 16u);
}

}  // namespace

hipError_t launch_plan_batched(const uint64_t* offsets, uint64_t count, uint64_t elem_base, uint64_t seed,
                               const Params& prm, uint64_t max_elems, uint64_t max_tiles, uint64_t max_chunks,
                               uint64_t max_buckets, uint64_t total_elems, SubDesc* subs, LeafDesc* leaves,
                               unsigned long long* counters, uint64_t* dsz, uint32_t* err, hipStream_t stream)
{
    hipLaunchKernelGGL(k_plan_batched, dim3(1), dim3(kPlanThreads), 0, stream, offsets, count, elem_base, seed,
                       prm, max_elems, max_tiles, max_chunks, max_buckets, total_elems, subs, leaves, counters,
                       dsz, err);
    return hipGetLastError();
}

hipError_t launch_zero_words(uint32_t* p, uint32_t words, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, stream, p, words);
    return hipGetLastError();
}

hipError_t launch_check_one_level(const unsigned long long* counters, uint32_t* err, hipStream_t stream)
{
    hipLaunchKernelGGL(k_check_one_level, dim3(1), dim3(64), 0, stream, counters, err);
    return hipGetLastError();
}

}  // namespace ipss
