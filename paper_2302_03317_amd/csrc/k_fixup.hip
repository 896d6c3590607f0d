// Fix-up of a tiled level (the role of FineScatter, arXiv 2302.03317 Sec. 3.4).
//
// After the rough pass every tile has written its per-bucket counts.  From
// them the final bucket sizes N_b and starts S_b follow, so the bucket
// boundaries move from the equal split to the exact split.  An item is kept
// where the rough pass put it when that slot lies inside its final region;
// every other item is a mover.  Movers of bucket b are taken in (tile, read
// order) order and fill the free slots of the final region F_b in ascending
// order.  The tables below give every (tile, bucket) pair its share of that
// order; the gather kernel copies movers to a workspace and the scatter
// kernel copies them into the free slots.
//
// All table kernels work on the level's subproblems at once.  Per-(tile,
// bucket) columns are summed in chunks of kChunk tiles, chunk sums are
// scanned per bucket, and the in-chunk prefixes are materialised last.
#include "common.hpp"
#include "kernels.hpp"

namespace ipss {

namespace {

constexpr int kTabThreads = 256;
// Threads of a gather or scatter workgroup (one tile each); 128, 512 and
// 1024 measured slower.
constexpr int kFixThreads = 256;
// Subproblems of more chunks than this get one wave per bucket in the
// per-bucket reductions over chunks.
constexpr uint64_t kWaveChunks = 16;

// Per (tile, bucket): the rough piece, how much of it was filled, the part of
// the placed front that lies inside the final region (kept), the displaced
// and the staged (overflow) counts.
struct Stats {
    uint64_t lo;       // piece start (relative to the subproblem)
    uint64_t cap;
    uint64_t fill;
    uint64_t kept_lo;  // kept range [kept_lo, kept_lo + kept)
    uint64_t kept;
    uint64_t disp;     // placed but outside the final region
    uint64_t ov;       // did not fit the piece
};

__device__ __forceinline__ Stats piece_stats(const Piece& pc, uint32_t cnt, uint64_t S, uint64_t N)
{
    Stats st;
    st.lo = pc.lo;
    st.cap = pc.cap;
    st.fill = cnt < pc.cap ? cnt : pc.cap;
    st.ov = cnt - st.fill;
    const uint64_t a = pc.lo > S ? pc.lo : S;
    const uint64_t e = (pc.lo + st.fill) < (S + N) ? (pc.lo + st.fill) : (S + N);
    st.kept = e > a ? e - a : 0;
    st.kept_lo = e > a ? a : pc.lo;
    st.disp = st.fill - st.kept;
    return st;
}


// The pieces of region b in tiles t0, t0 + 1, ...: piece t of a region of len
// items starts at t*q + floor(t*r / P) (len = q*P + r, P tiles), so from one
// tile to the next the start advances by q, plus one where the remainder
// t*r mod P wraps.  Divisions at the first tile only.
struct PieceWalk {
    uint64_t e0, q, r, P, off, rem;

    __device__ __forceinline__ PieceWalk(const SubDesc& sd, uint64_t t0, uint32_t b)
    {
        e0 = (static_cast<uint64_t>(b) * sd.m) >> sd.kappa;
        const uint64_t len = ((static_cast<uint64_t>(b + 1) * sd.m) >> sd.kappa) - e0;
        P = sd.tiles;
        q = len / P;
        r = len - q * P;
        off = piece_offset(t0, len, P);
        const uint64_t tr = t0 * r;  // t0 < P and r < P, P <= 2^32
        rem = ((tr | P) >> 32) == 0 ? static_cast<uint32_t>(tr) % static_cast<uint32_t>(P) : tr % P;
    }
    // the piece of the current tile; moves on to the next tile
    __device__ __forceinline__ Piece next()
    {
        uint64_t nrem = rem + r, step = q;
        if (nrem >= P) {
            nrem -= P;
            ++step;
        }
        const Piece pc{e0 + off, step};
        off += step;
        rem = nrem;
        return pc;
    }
};

// Inclusive prefix sum of 64-bit values across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_inclusive_sum64(uint64_t v, uint32_t lane)
{
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Sizes of the level: the host's, or the device's for a level planned on
// the device (the launches then cover upper bounds).
__device__ __forceinline__ uint64_t n_subs(const LevelTables& T) { return T.dsz ? T.dsz[0] : T.nsubs; }
__device__ __forceinline__ uint64_t n_tiles(const LevelTables& T) { return T.dsz ? T.dsz[1] : T.ntiles; }
__device__ __forceinline__ uint64_t n_chunks(const LevelTables& T) { return T.dsz ? T.dsz[2] : T.nchunks; }
__device__ __forceinline__ uint64_t n_buckets(const LevelTables& T) { return T.dsz ? T.dsz[3] : T.nbuckets; }

__device__ __forceinline__ uint64_t chunk_tiles(const SubDesc& sd, uint64_t c, uint64_t* t0)
{
    *t0 = c * kChunk;
    const uint64_t t1 = (*t0 + kChunk) < sd.tiles ? (*t0 + kChunk) : sd.tiles;
    return t1 - *t0;
}

__device__ __forceinline__ uint64_t num_chunks(const SubDesc& sd)
{
    return (sd.tiles + kChunk - 1) / kChunk;
}

// ---- maps of a level: global tile / chunk / bucket -> subproblem ----
// The last subproblem whose range starts at or before x (ranges start in
// increasing order and none is empty).
template <int F>
__device__ __forceinline__ uint32_t sub_of(const SubDesc* subs, uint32_t nsub, uint64_t x)
{
    uint32_t lo = 0, hi = nsub;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        const uint64_t off = F == 0 ? subs[mid].tile_off : (F == 1 ? subs[mid].chunk_off : subs[mid].bk_off);
        if (off <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kTabThreads) void k_level_maps(const SubDesc* __restrict__ subs,
                                                            uint32_t nsub, uint64_t ntiles,
                                                            uint64_t nchunks, uint64_t nbuckets,
                                                            uint32_t* __restrict__ tile_sub,
                                                            uint64_t* __restrict__ tile_pofs,
                                                            uint32_t* __restrict__ chunk_sub,
                                                            uint32_t* __restrict__ bk_sub,
                                                            const uint64_t* __restrict__ dsz)
{
    // the index space is [tiles | chunks | buckets] with the host's (upper
    // bound) sizes; entries beyond the device's sizes are skipped
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * kTabThreads + threadIdx.x;
    if (dsz) nsub = static_cast<uint32_t>(dsz[0]);
    if (i < ntiles) {
        if (dsz && i >= dsz[1]) return;
        const uint32_t j = sub_of<0>(subs, nsub, i);
        tile_sub[i] = j;
        // the tile's piece offsets for the two region lengths
        const SubDesc& sd = subs[j];
        const uint64_t t = i - sd.tile_off, len0 = sd.m >> sd.kappa;
        tile_pofs[2 * i] = piece_offset(t, len0, sd.tiles);
        tile_pofs[2 * i + 1] = piece_offset(t, len0 + 1, sd.tiles);
        return;
    }
    i -= ntiles;
    if (i < nchunks) {
        if (dsz && i >= dsz[2]) return;
        chunk_sub[i] = sub_of<1>(subs, nsub, i);
        return;
    }
    i -= nchunks;
    if (i < nbuckets && !(dsz && i >= dsz[3])) bk_sub[i] = sub_of<2>(subs, nsub, i);
}

// chA[chunk][b] = sum of the chunk's counts of bucket b
__global__ __launch_bounds__(kTabThreads) void k_chunk_count_sum(LevelTables T)
{
    const uint64_t g = blockIdx.x;
    if (g >= n_chunks(T)) return;
    const SubDesc sd = T.subs[T.chunk_sub[g]];
    const uint32_t k = 1u << sd.kappa;
    const uint64_t c = g - sd.chunk_off;
    uint64_t t0;
    const uint64_t nt = chunk_tiles(sd, c, &t0);
    for (uint32_t b = threadIdx.x; b < k; b += kTabThreads) {
        uint64_t s = 0;
        for (uint64_t i = 0; i < nt; ++i) s += T.cnt[sd.tab_off + (t0 + i) * k + b];
        T.chA[sd.chtab_off + c * k + b] = s;
    }
}

// N[b] = sum over chunks
__global__ __launch_bounds__(kTabThreads) void k_bucket_count_total(LevelTables T)
{
    const uint64_t gb = static_cast<uint64_t>(blockIdx.x) * kTabThreads + threadIdx.x;
    if (gb >= n_buckets(T)) return;
    const SubDesc sd = T.subs[T.bk_sub[gb]];
    const uint32_t k = 1u << sd.kappa;
    const uint32_t b = static_cast<uint32_t>(gb - sd.bk_off);
    const uint64_t nc = num_chunks(sd);
    uint64_t run = 0;
    for (uint64_t c = 0; c < nc; ++c) run += T.chA[sd.chtab_off + c * k + b];
    T.N[gb] = run;
}

// The same with one wave per bucket, for levels whose subproblems span many
// chunks (a thread per bucket would walk them one by one).
__global__ __launch_bounds__(kTabThreads) void k_bucket_count_total_wave(LevelTables T)
{
    const uint64_t gb = static_cast<uint64_t>(blockIdx.x) * (kTabThreads / 64) + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (gb >= n_buckets(T)) return;  // the whole wave
    const SubDesc sd = T.subs[T.bk_sub[gb]];
    const uint32_t k = 1u << sd.kappa;
    const uint32_t b = static_cast<uint32_t>(gb - sd.bk_off);
    const uint64_t nc = num_chunks(sd);
    uint64_t run = 0;
    for (uint64_t c = lane; c < nc; c += 64) run += T.chA[sd.chtab_off + c * k + b];
    run = wave_inclusive_sum64(run, lane);
    if (lane == 63) T.N[gb] = run;
}

// S[b] = exclusive prefix of N over the subproblem's buckets; one wave per
// subproblem, each lane a run of consecutive buckets.
__global__ __launch_bounds__(64) void k_bucket_starts(LevelTables T)
{
    if (blockIdx.x >= n_subs(T)) return;
    const SubDesc sd = T.subs[blockIdx.x];
    const uint32_t lane = threadIdx.x;
    const uint32_t k = 1u << sd.kappa;
    const uint32_t per = (k + 63) / 64, b0 = lane * per;
    uint64_t own = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (b0 + j < k) own += T.N[sd.bk_off + b0 + j];
    uint64_t run = wave_inclusive_sum64(own, lane) - own;
    for (uint32_t j = 0; j < per; ++j) {
        if (b0 + j < k) {
            T.S[sd.bk_off + b0 + j] = run;
            run += T.N[sd.bk_off + b0 + j];
        }
    }
}

// chA[chunk][b] = movers, chB[chunk][b] = kept items of the chunk's tiles
__global__ __launch_bounds__(kTabThreads) void k_chunk_route_sum(LevelTables T)
{
    const uint64_t g = blockIdx.x;
    if (g >= n_chunks(T)) return;
    const SubDesc sd = T.subs[T.chunk_sub[g]];
    const uint32_t k = 1u << sd.kappa;
    const uint64_t c = g - sd.chunk_off;
    uint64_t t0;
    const uint64_t nt = chunk_tiles(sd, c, &t0);
    for (uint32_t b = threadIdx.x; b < k; b += kTabThreads) {
        const uint64_t S = T.S[sd.bk_off + b], N = T.N[sd.bk_off + b];
        uint64_t mv = 0, kp = 0;
        PieceWalk pw(sd, t0, b);
        for (uint64_t i = 0; i < nt; ++i) {
            const uint64_t t = t0 + i;
            const Stats st = piece_stats(pw.next(), T.cnt[sd.tab_off + t * k + b], S, N);
            mv += st.disp + st.ov;
            kp += st.kept;
        }
        T.chA[sd.chtab_off + c * k + b] = mv;
        T.chB[sd.chtab_off + c * k + b] = kp;
    }
}

// chunk sums -> exclusive chunk prefixes; M[b], K[b] totals
__global__ __launch_bounds__(kTabThreads) void k_bucket_route_scan(LevelTables T)
{
    const uint64_t gb = static_cast<uint64_t>(blockIdx.x) * kTabThreads + threadIdx.x;
    if (gb >= n_buckets(T)) return;
    const SubDesc sd = T.subs[T.bk_sub[gb]];
    const uint32_t k = 1u << sd.kappa;
    const uint32_t b = static_cast<uint32_t>(gb - sd.bk_off);
    const uint64_t nc = num_chunks(sd);
    uint64_t rm = 0, rk = 0;
    for (uint64_t c = 0; c < nc; ++c) {
        const uint64_t i = sd.chtab_off + c * k + b;
        const uint64_t vm = T.chA[i], vk = T.chB[i];
        T.chA[i] = rm;
        T.chB[i] = rk;
        rm += vm;
        rk += vk;
    }
    T.M[gb] = rm;
    T.K[gb] = rk;
}

// The same with one wave per bucket (subproblems of many chunks).
__global__ __launch_bounds__(kTabThreads) void k_bucket_route_scan_wave(LevelTables T)
{
    const uint64_t gb = static_cast<uint64_t>(blockIdx.x) * (kTabThreads / 64) + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (gb >= n_buckets(T)) return;  // the whole wave
    const SubDesc sd = T.subs[T.bk_sub[gb]];
    const uint32_t k = 1u << sd.kappa;
    const uint32_t b = static_cast<uint32_t>(gb - sd.bk_off);
    const uint64_t nc = num_chunks(sd);
    uint64_t rm = 0, rk = 0;
    for (uint64_t c0 = 0; c0 < nc; c0 += 64) {
        const uint64_t c = c0 + lane;
        const uint64_t i = sd.chtab_off + c * k + b;
        uint64_t vm = 0, vk = 0;
        if (c < nc) {
            vm = T.chA[i];
            vk = T.chB[i];
        }
        const uint64_t sm = wave_inclusive_sum64(vm, lane), sk = wave_inclusive_sum64(vk, lane);
        if (c < nc) {
            T.chA[i] = rm + sm - vm;
            T.chB[i] = rk + sk - vk;
        }
        rm += __shfl(sm, 63, 64);
        rk += __shfl(sk, 63, 64);
    }
    if (lane == 0) {
        T.M[gb] = rm;
        T.K[gb] = rk;
    }
}

// MB = exclusive prefix of M over all buckets of the level, in three steps:
// per-chunk sums, a scan of the chunk sums (with the level total), and the
// scan inside every chunk.
__global__ __launch_bounds__(kTabThreads) void k_ws_chunk_sums(LevelTables T)
{
    __shared__ uint64_t part[kTabThreads];
    const uint64_t c0 = static_cast<uint64_t>(blockIdx.x) * kScanChunk;
    uint64_t s = 0;
    const uint64_t nb = n_buckets(T);
    for (uint64_t i = c0 + threadIdx.x; i < c0 + kScanChunk && i < nb; i += kTabThreads)
        s += T.M[i];
    part[threadIdx.x] = s;
    block_sync();
    for (uint32_t d = kTabThreads / 2; d > 0; d >>= 1) {
        if (threadIdx.x < d) part[threadIdx.x] += part[threadIdx.x + d];
        block_sync();
    }
    if (threadIdx.x == 0) T.wsp[blockIdx.x] = part[0];
}

// One wave: the partial sums 64 at a time (one load per lane, a wave scan),
// rather than one dependent load after the other.
__global__ __launch_bounds__(64) void k_ws_scan_sums(LevelTables T, uint32_t nparts)
{
    const uint32_t lane = threadIdx.x;
    uint64_t run = 0;
    for (uint32_t i0 = 0; i0 < nparts; i0 += 64) {
        const uint32_t i = i0 + lane;
        const uint64_t v = i < nparts ? T.wsp[i] : 0;
        uint64_t incl = v;
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t u = __shfl_up(incl, d, 64);
            if (lane >= d) incl += u;
        }
        if (i < nparts) T.wsp[i] = run + (incl - v);
        run += __shfl(incl, 63, 64);
    }
    if (lane == 0) *T.total = run;
}

__global__ __launch_bounds__(kTabThreads) void k_ws_chunk_scan(LevelTables T)
{
    constexpr uint32_t per = kScanChunk / kTabThreads;  // consecutive buckets per thread
    __shared__ uint64_t part[kTabThreads];
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kScanChunk + threadIdx.x * per;
    const uint64_t nb = n_buckets(T);
    uint64_t s = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (b0 + j < nb) s += T.M[b0 + j];
    part[threadIdx.x] = s;
    block_sync();
    if (threadIdx.x == 0) {
        uint64_t run = T.wsp[blockIdx.x];
        for (uint32_t i = 0; i < kTabThreads; ++i) {
            const uint64_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    block_sync();
    uint64_t run = part[threadIdx.x];
    for (uint32_t j = 0; j < per; ++j) {
        if (b0 + j < nb) {
            const uint64_t v = T.M[b0 + j];
            T.MB[b0 + j] = run;
            run += v;
        }
    }
}

// mpre/kpre[tile][b]: movers / kept items of bucket b in earlier tiles
__global__ __launch_bounds__(kTabThreads) void k_chunk_route_prefix(LevelTables T)
{
    const uint64_t g = blockIdx.x;
    if (g >= n_chunks(T)) return;
    const SubDesc sd = T.subs[T.chunk_sub[g]];
    const uint32_t k = 1u << sd.kappa;
    const uint64_t c = g - sd.chunk_off;
    uint64_t t0;
    const uint64_t nt = chunk_tiles(sd, c, &t0);
    for (uint32_t b = threadIdx.x; b < k; b += kTabThreads) {
        const uint64_t S = T.S[sd.bk_off + b], N = T.N[sd.bk_off + b];
        uint64_t rm = T.chA[sd.chtab_off + c * k + b];
        uint64_t rk = T.chB[sd.chtab_off + c * k + b];
        PieceWalk pw(sd, t0, b);
        for (uint64_t i = 0; i < nt; ++i) {
            const uint64_t t = t0 + i;
            const uint64_t e = sd.tab_off + t * k + b;
            const Stats st = piece_stats(pw.next(), T.cnt[e], S, N);
            T.mpre[e] = rm;
            T.kpre[e] = rk;
            rm += st.disp + st.ov;
            rk += st.kept;
        }
    }
}

// ---- children of the level: leaves and subproblems that need another tiled level ----
// One atomic per list and workgroup: the waves' counts are added up in LDS.
constexpr int kChildThreads = 1024;

__global__ __launch_bounds__(kChildThreads) void k_children(LevelTables T, uint32_t tile_limit,
                                                            LeafDesc* leaves, LeafDesc* big,
                                                            unsigned long long* counters)
{
    constexpr uint32_t kW = kChildThreads / 64;
    __shared__ uint32_t wcnt[3][kW];
    __shared__ unsigned long long wbase[2][kW];
    // No early exit: every thread takes part in the barriers.
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint64_t gb = static_cast<uint64_t>(blockIdx.x) * kChildThreads + threadIdx.x;
    uint64_t n = 0;
    LeafDesc c{};
    if (gb < n_buckets(T)) {
        const SubDesc sd = T.subs[T.bk_sub[gb]];
        n = T.N[gb];
        c = LeafDesc{sd.elem_off, sd.base + T.S[gb], n, sd.seed, sd.level + 1, sd.stream_id,
                     sd.owner, 0u};
    }
    const bool leaf = n >= 2 && n <= tile_limit;
    const bool more = n > tile_limit;
    const uint64_t ml = __ballot(leaf), mb = __ballot(more);
    // leaf children hold at most tile_limit < 2^16 items: a workgroup's sum fits 32 bits
    const uint32_t sum = wave_inclusive_sum(leaf ? static_cast<uint32_t>(n) : 0u);
    if (lane == 63) {
        wcnt[0][wv] = static_cast<uint32_t>(__popcll(ml));
        wcnt[1][wv] = static_cast<uint32_t>(__popcll(mb));
        wcnt[2][wv] = sum;
    }
    block_sync();
    if (threadIdx.x == 0) {
        unsigned long long nl = 0, nb = 0, ne = 0;
        for (uint32_t w = 0; w < kW; ++w) {
            wbase[0][w] = nl;
            wbase[1][w] = nb;
            nl += wcnt[0][w];
            nb += wcnt[1][w];
            ne += wcnt[2][w];
        }
        const unsigned long long bl = nl ? atomicAdd(&counters[0], nl) : 0ull;
        const unsigned long long bb = nb ? atomicAdd(&counters[1], nb) : 0ull;
        if (ne) atomicAdd(&counters[2], ne);
        for (uint32_t w = 0; w < kW; ++w) {
            wbase[0][w] += bl;
            wbase[1][w] += bb;
        }
    }
    block_sync();
    if (leaf) leaves[wbase[0][wv] + bits_below(ml)] = c;
    if (more) big[wbase[1][wv] + bits_below(mb)] = c;
}

// ---- gather: movers of one tile into the workspace ----
template <typename E>
__global__ __launch_bounds__(kFixThreads) void k_gather(E* __restrict__ ws, LevelTables T)
{
    __shared__ uint64_t lo[kKmax], kept_lo[kKmax], base_w[kKmax];
    __shared__ uint32_t fill[kKmax], kept[kKmax], disp[kKmax];
    __shared__ uint32_t ovt[kKmax + 1], hot[kKmax + 1], outt[kKmax + 1];
    const uint32_t tid = threadIdx.x, wv = tid >> 6;
    const uint64_t nt = n_tiles(T);
    if (blockIdx.x >= nt) return;
    const uint64_t g = xcd_order(blockIdx.x, static_cast<uint32_t>(nt));
    const SubDesc sd = T.subs[T.tile_sub[g]];
    const uint64_t t = g - sd.tile_off;
    const uint32_t k = 1u << sd.kappa;
    const global_t<E>* X = elem_gptr<E>(sd.elem_off) + sd.base;
    const TilePieces tp(sd.m, sd.kappa, sd.tiles, t, T.tile_pofs + 2 * g);
    for (uint32_t b = tid; b < k; b += kFixThreads) {
        const uint64_t e = sd.tab_off + t * k + b;
        const uint64_t gb = sd.bk_off + b;
        const Stats st = piece_stats(tp.of(b), T.cnt[e], T.S[gb], T.N[gb]);
        lo[b] = st.lo;
        kept_lo[b] = st.kept_lo;
        fill[b] = static_cast<uint32_t>(st.fill);
        kept[b] = static_cast<uint32_t>(st.kept);
        disp[b] = static_cast<uint32_t>(st.disp);
        ovt[b] = static_cast<uint32_t>(st.ov);
        hot[b] = static_cast<uint32_t>(st.cap - st.fill);
        outt[b] = static_cast<uint32_t>(st.disp + st.ov);
        base_w[b] = T.MB[gb] + T.mpre[e];
    }
    block_sync();
    if (wv == 0) wave_exclusive_scan(ovt, k);
    if (wv == 1) wave_exclusive_scan(hot, k);
    if (wv == 2) wave_exclusive_scan(outt, k);
    block_sync();
    const uint32_t nout = outt[k];
    for (uint32_t i = tid; i < nout; i += kFixThreads) {
        const uint32_t b = upper_index(outt, k, i);
        const uint32_t j = i - outt[b];
        uint64_t pos;
        if (j < disp[b]) {
            // displaced: placed ranks outside the final region, in rank order
            const uint64_t before = kept[b] ? kept_lo[b] - lo[b] : fill[b];
            const uint64_t r = j < before ? j : (kept_lo[b] - lo[b]) + kept[b] + (j - before);
            pos = lo[b] + r;
        } else {
            // staged: overflow o of bucket b sits in free slot ovt[b] + o of the tile
            const uint32_t s = ovt[b] + (j - disp[b]);
            const uint32_t bb = upper_index(hot, k, s);
            pos = lo[bb] + fill[bb] + (s - hot[bb]);
        }
        const uint64_t widx = base_w[b] + j;
        if (widx >= T.ws_cap || pos >= sd.m) {
            atomicOr(T.err, 1u);
            continue;
        }
        ws[widx] = X[pos];
    }
}

// ---- scatter: free slots of the tile's pieces from the workspace ----
template <typename E>
__global__ __launch_bounds__(kFixThreads) void k_scatter(const E* __restrict__ ws, LevelTables T)
{
    __shared__ uint64_t S[kKmax], Ktot[kKmax], MB[kKmax], lo[kKmax], kept_lo[kKmax], kpre[kKmax];
    __shared__ uint32_t kept[kKmax], nkt[kKmax + 1];
    const uint32_t tid = threadIdx.x, wv = tid >> 6;
    const uint64_t nt = n_tiles(T);
    if (blockIdx.x >= nt) return;
    const uint64_t g = xcd_order(blockIdx.x, static_cast<uint32_t>(nt));
    const SubDesc sd = T.subs[T.tile_sub[g]];
    const uint64_t t = g - sd.tile_off;
    const uint32_t k = 1u << sd.kappa;
    global_t<E>* X = elem_gptr<E>(sd.elem_off) + sd.base;
    const TilePieces tp(sd.m, sd.kappa, sd.tiles, t, T.tile_pofs + 2 * g);
    for (uint32_t b = tid; b < k; b += kFixThreads) {
        const uint64_t e = sd.tab_off + t * k + b;
        const uint64_t gb = sd.bk_off + b;
        const Stats st = piece_stats(tp.of(b), T.cnt[e], T.S[gb], T.N[gb]);
        S[b] = T.S[gb];
        Ktot[b] = T.K[gb];
        MB[b] = T.MB[gb];
        lo[b] = st.lo;
        kept_lo[b] = st.kept_lo;
        kept[b] = static_cast<uint32_t>(st.kept);
        kpre[b] = T.kpre[e];
        nkt[b] = static_cast<uint32_t>(st.cap - st.kept);
    }
    block_sync();
    if (wv == 0) wave_exclusive_scan(nkt, k);
    block_sync();
    const uint32_t nfree = nkt[k];
    for (uint32_t i = tid; i < nfree; i += kFixThreads) {
        const uint32_t b = upper_index(nkt, k, i);  // piece of the free slot
        const uint64_t j = i - nkt[b];
        uint64_t x;
        if (kept[b] == 0) {
            x = lo[b] + j;
        } else {
            const uint64_t before = kept_lo[b] - lo[b];
            x = j < before ? lo[b] + j : kept_lo[b] + kept[b] + (j - before);
        }
        const uint32_t fb = upper_index64(S, k, x);  // final bucket holding slot x
        uint64_t kb;  // kept items of bucket fb below x
        if (fb == b) {
            kb = kpre[b] + ((kept[b] && x >= kept_lo[b] + kept[b]) ? kept[b] : 0);
        } else {
            // kept items of fb lie in its equal region, wholly below or above x
            kb = fb < b ? Ktot[fb] : 0;
        }
        const uint64_t widx = MB[fb] + (x - S[fb]) - kb;
        if (widx >= T.ws_cap || x >= sd.m) {
            atomicOr(T.err, 2u);
            continue;
        }
        X[x] = ws[widx];
    }
}

}  // namespace

hipError_t launch_level_maps(const SubDesc* subs, uint32_t nsub, uint64_t ntiles, uint64_t nchunks,
                             uint64_t nbuckets, uint32_t* tile_sub, uint64_t* tile_pofs,
                             uint32_t* chunk_sub, uint32_t* bk_sub, hipStream_t stream,
                             const uint64_t* dsz)
{
    const uint64_t n = ntiles + nchunks + nbuckets;
    if (n == 0 || nsub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_level_maps, dim3(static_cast<uint32_t>((n + kTabThreads - 1) / kTabThreads)),
                       dim3(kTabThreads), 0, stream, subs, nsub, ntiles, nchunks, nbuckets, tile_sub,
                       tile_pofs, chunk_sub, bk_sub, dsz);
    return hipGetLastError();
}

hipError_t launch_tables_sizes(const LevelTables& t, hipStream_t stream)
{
    if (t.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_count_sum, dim3(static_cast<uint32_t>(t.nchunks)), dim3(kTabThreads),
                       0, stream, t);
    if (t.max_chunks > kWaveChunks)
        hipLaunchKernelGGL(k_bucket_count_total_wave,
                           dim3(static_cast<uint32_t>((t.nbuckets + kTabThreads / 64 - 1) / (kTabThreads / 64))),
                           dim3(kTabThreads), 0, stream, t);
    else
        hipLaunchKernelGGL(k_bucket_count_total,
                           dim3(static_cast<uint32_t>((t.nbuckets + kTabThreads - 1) / kTabThreads)),
                           dim3(kTabThreads), 0, stream, t);
    hipLaunchKernelGGL(k_bucket_starts, dim3(static_cast<uint32_t>(t.nsubs)), dim3(64), 0, stream, t);
    return hipGetLastError();
}

hipError_t launch_tables_routes(const LevelTables& t, hipStream_t stream)
{
    if (t.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_route_sum, dim3(static_cast<uint32_t>(t.nchunks)), dim3(kTabThreads),
                       0, stream, t);
    if (t.max_chunks > kWaveChunks)
        hipLaunchKernelGGL(k_bucket_route_scan_wave,
                           dim3(static_cast<uint32_t>((t.nbuckets + kTabThreads / 64 - 1) / (kTabThreads / 64))),
                           dim3(kTabThreads), 0, stream, t);
    else
        hipLaunchKernelGGL(k_bucket_route_scan,
                           dim3(static_cast<uint32_t>((t.nbuckets + kTabThreads - 1) / kTabThreads)),
                           dim3(kTabThreads), 0, stream, t);
    const uint32_t nparts = static_cast<uint32_t>((t.nbuckets + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_ws_chunk_sums, dim3(nparts), dim3(kTabThreads), 0, stream, t);
    hipLaunchKernelGGL(k_ws_scan_sums, dim3(1), dim3(64), 0, stream, t, nparts);
    hipLaunchKernelGGL(k_ws_chunk_scan, dim3(nparts), dim3(kTabThreads), 0, stream, t);
    hipLaunchKernelGGL(k_chunk_route_prefix, dim3(static_cast<uint32_t>(t.nchunks)),
                       dim3(kTabThreads), 0, stream, t);
    return hipGetLastError();
}

hipError_t launch_children(const LevelTables& t, uint32_t tile_limit, LeafDesc* leaves,
                           LeafDesc* big, unsigned long long* counters, hipStream_t stream)
{
    if (t.nbuckets == 0) return hipSuccess;
    hipLaunchKernelGGL(k_children,
                       dim3(static_cast<uint32_t>((t.nbuckets + kChildThreads - 1) / kChildThreads)),
                       dim3(kChildThreads), 0, stream, t, tile_limit, leaves, big, counters);
    return hipGetLastError();
}

template <typename E>
static hipError_t gather_t(uint8_t* ws, const LevelTables& t, hipStream_t stream)
{
    hipLaunchKernelGGL(k_gather<E>, dim3(static_cast<uint32_t>(t.ntiles)), dim3(kFixThreads), 0,
                       stream, reinterpret_cast<E*>(ws), t);
    return hipGetLastError();
}

template <typename E>
static hipError_t scatter_t(const uint8_t* ws, const LevelTables& t, hipStream_t stream)
{
    hipLaunchKernelGGL(k_scatter<E>, dim3(static_cast<uint32_t>(t.ntiles)), dim3(kFixThreads), 0,
                       stream, reinterpret_cast<const E*>(ws), t);
    return hipGetLastError();
}

hipError_t launch_gather(uint32_t w, uint8_t* ws, const LevelTables& t, hipStream_t stream)
{
    if (t.ntiles == 0) return hipSuccess;
    switch (w) {
    case 4: return gather_t<uint32_t>(ws, t, stream);
    case 8: return gather_t<uint64_t>(ws, t, stream);
    case 16: return gather_t<Elem16>(ws, t, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scatter(uint32_t w, const uint8_t* ws, const LevelTables& t,
                          hipStream_t stream)
{
    if (t.ntiles == 0) return hipSuccess;
    switch (w) {
    case 4: return scatter_t<uint32_t>(ws, t, stream);
    case 8: return scatter_t<uint64_t>(ws, t, stream);
    case 16: return scatter_t<Elem16>(ws, t, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ipss
