// Shared descriptors and small device helpers for the in-place ScatterShuffle
// kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipss {

constexpr int kThreads = 512;              // threads of a leaf workgroup
constexpr int kWaves = kThreads / 64;      // wave64
constexpr int kRoughThreads = 1024;        // threads of a tile workgroup
constexpr int kRoughWaves = kRoughThreads / 64;
constexpr uint32_t kTileBytesMax = 65536;  // most bytes of one tile's elements
constexpr uint32_t kKmax = 256;            // labels live in one byte
constexpr uint32_t kChunk = 256;           // tiles per chunk of the table scans
constexpr uint32_t kLdsBytesMax = 163840;  // LDS of one CU on gfx950

struct Params {
    uint32_t tile;      // T: most elements a tile holds
    uint32_t kmax_log2; // largest bucket-count exponent
    uint32_t n0;        // base-case size
    uint32_t lmax;      // recursion cap
    // How the kernels compute stable ranks (not part of the definition: both
    // give the same ranks): 1 = one LDS atomic add per item, which needs the
    // device to serve one wave's same-address LDS atomics in lane order
    // (checked once per device); 0 = one ballot per label bit.
    uint32_t rank_atomic;
    // 1 = the tile kernel finds the slot of every staged item by a search
    // over the pieces' free slots, as it does when they do not fit its list;
    // 0 = by the list whenever it fits (both give the same slots; 1 exists
    // so that tests can run the search).
    uint32_t slot_search;
};

// Device memory seen through the global address space: its loads and stores
// are global instructions, not flat ones, so they do not count on the LDS
// counter and a wait for an LDS result does not wait for them.
// (The qualifier applies to the device pass; the host pass of the same source
// only needs the kernels' types to exist.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using global_t = __attribute__((address_space(1))) T;
#else
template <typename T>
using global_t = T;
#endif

// Elements are addressed absolutely: an array at device address A holds
// element i at element address A / w + i (arrays are aligned to w), so one
// launch can serve arrays of any number of allocations.
template <typename E>
__device__ __forceinline__ global_t<E>* elem_gptr(uint64_t elem_addr)
{
    return (global_t<E>*)(static_cast<uintptr_t>(elem_addr * sizeof(E)));
}

// One subproblem of the tiled regime at the current level.
struct SubDesc {
    uint64_t elem_off;  // element address of its array's first element
    uint64_t base;      // start of the subproblem inside its array (positions)
    uint64_t m;         // elements
    uint64_t tiles;     // P
    uint64_t tile_off;  // first global tile of the level's launch
    uint64_t tab_off;   // first entry of its per-(tile, bucket) tables (row = tile)
    uint64_t chunk_off; // first chunk of its table scans
    uint64_t chtab_off; // first entry of its per-(chunk, bucket) tables (row = chunk)
    uint64_t seed;      // Philox key of its array
    uint32_t bk_off;    // first entry of its per-bucket tables
    uint32_t kappa;     // k = 2^kappa
    uint32_t level;
    uint32_t stream_id;
    uint32_t owner;     // request the array belongs to (host bookkeeping)
    uint32_t pad;
};

// One subproblem finished in LDS (fits a tile) or by the sequential fallback.
struct LeafDesc {
    uint64_t elem_off;  // element address of its array's first element
    uint64_t base;      // start inside its array (positions)
    uint64_t m;
    uint64_t seed;
    uint32_t level;
    uint32_t stream_id;
    uint32_t owner;
    uint32_t pad;
};

// Piece t of equal region b of a subproblem of m elements cut into 2^kappa
// regions and P tiles: [lo, lo + cap), relative to the subproblem start.
// Region b is [floor(b*m/k), floor((b+1)*m/k)); piece t starts at
// floor(t*len/P).  The product t*len is split as t*(len/P) + t*(len%P)/P so
// that it stays inside 64 bits (the host ensures P <= 2^32).
__host__ __device__ __forceinline__ uint64_t piece_offset(uint64_t t, uint64_t len, uint64_t P)
{
    if (((len | P) >> 32) == 0) {  // 32-bit divisions where the operands allow
        const uint32_t l32 = static_cast<uint32_t>(len), p32 = static_cast<uint32_t>(P);
        const uint32_t q = l32 / p32, r = l32 % p32;
        const uint64_t tr = t * r;
        const uint64_t rest = (tr >> 32) == 0 ? static_cast<uint32_t>(tr) / p32 : tr / P;
        return t * q + rest;
    }
    const uint64_t q = len / P, r = len % P;
    return t * q + (t * r) / P;
}

struct Piece {
    uint64_t lo;
    uint64_t cap;
};

__host__ __device__ __forceinline__ Piece piece_of(uint64_t m, uint32_t kappa, uint64_t P,
                                                   uint64_t t, uint32_t b)
{
    const uint64_t e0 = (static_cast<uint64_t>(b) * m) >> kappa;
    const uint64_t e1 = (static_cast<uint64_t>(b + 1) * m) >> kappa;
    const uint64_t len = e1 - e0;
    const uint64_t lo = e0 + piece_offset(t, len, P);
    const uint64_t hi = e0 + piece_offset(t + 1, len, P);
    return {lo, hi - lo};
}

// The pieces of tile t in all k regions of a subproblem: region b starts at
// e0 = floor(b*m/k) and holds floor(m/k) or floor(m/k) + 1 items, so a piece's
// offset inside its region takes one of two values per tile.  The level's
// table holds both for every tile (pofs[2g + s] = piece_offset(t, len0 + s, P)
// for global tile g = tile t of its subproblem); a tile reads its own pair
// and the next tile's, and selects per region.  Same bounds as piece_of.
struct TilePieces {
    uint64_t m, len0, off[2][2];  // off[s][u]: offset at tile t + u for length len0 + s
    uint32_t kappa;

    __host__ __device__ __forceinline__ TilePieces(uint64_t m_, uint32_t kappa_, uint64_t P, uint64_t t,
                                                   const uint64_t* pofs_g)
        : m(m_), len0(m_ >> kappa_), kappa(kappa_)
    {
        const bool last = t + 1 >= P;  // piece_offset(P, len, P) = len
        off[0][0] = pofs_g[0];
        off[1][0] = pofs_g[1];
        off[0][1] = last ? len0 : pofs_g[2];
        off[1][1] = last ? len0 + 1 : pofs_g[3];
    }
    // Start of region b, floor(b*m/k).
    __host__ __device__ __forceinline__ uint64_t region_start(uint32_t b) const
    {
        return (static_cast<uint64_t>(b) * m) >> kappa;
    }
    // The piece of the region [e0, e1).
    __host__ __device__ __forceinline__ Piece of_region(uint64_t e0, uint64_t e1) const
    {
        const uint32_t s = (e1 - e0) != len0 ? 1u : 0u;
        return {e0 + off[s][0], off[s][1] - off[s][0]};
    }
    __host__ __device__ __forceinline__ Piece of(uint32_t b) const
    {
        return of_region(region_start(b), region_start(b + 1));
    }
    // Items of the tile's pieces 0 .. b-1 (b <= k): the regions before b are
    // b*len0 + n1 items long, n1 of them one longer, so the sum is
    // b*c0 + n1*(c1 - c0) with c_s the piece size for length len0 + s
    // (arithmetic mod 2^32: c1 - c0 may be -1).
    __host__ __device__ __forceinline__ uint32_t start(uint32_t b) const
    {
        const uint32_t c0 = static_cast<uint32_t>(off[0][1] - off[0][0]);
        const uint32_t c1 = static_cast<uint32_t>(off[1][1] - off[1][0]);
        const uint32_t n1 = static_cast<uint32_t>(((static_cast<uint64_t>(b) * m) >> kappa) -
                                                  static_cast<uint64_t>(b) * len0);
        return b * c0 + n1 * (c1 - c0);
    }
};

// LDS layout of the tile and leaf kernels (bytes).
__host__ __device__ __forceinline__ uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

struct RoughLayout {
    uint32_t stage;    // T elements of staging; labels, counters and slot tables overlay it
    uint32_t counts;   // per-wave counters: kRoughWaves rows of (kmax + 1) u32
    uint32_t slot_tab; // per-wave slot table: kRoughWaves rows of kmax uint2
    uint32_t tables;   // offset of the per-piece tables
    uint32_t total;
};

__host__ __device__ __forceinline__ RoughLayout rough_layout(uint32_t T, uint32_t w, uint32_t kmax)
{
    RoughLayout L;
    L.counts = align16(T);
    L.slot_tab = L.counts + align16(kRoughWaves * (kmax + 1) * 4u);
    const uint32_t overlay = L.slot_tab + kRoughWaves * kmax * 8u;
    // The staging area spans kTileBytesMax bytes whatever T is: a workgroup's
    // threads read that many bytes of slots into registers at fixed offsets
    // (the slots past the tile are read and ignored).  A shorter tile would
    // not raise occupancy: two 1024-thread workgroups fill a CU already.
    L.stage = align16(T * w);
    if (L.stage < kTileBytesMax) L.stage = kTileBytesMax;
    if (overlay > L.stage) L.stage = align16(overlay);
    // lo: (kmax+1) u64; qoff, cap, fill, ovt, hot, nblk: (kmax+1) u32 each; 16 u32 misc
    L.tables = L.stage;
    L.total = L.tables + align16((kmax + 1) * 8u + 6u * (kmax + 1) * 4u + 64u);
    return L;
}

struct LeafLayout {
    uint32_t idx;      // T u16: original leaf index of the item at each position
    uint32_t lab;      // T bytes: label bytes of the current level
    uint32_t hist;     // kWaves + 1 rows of (kmax + 1) u32 counters (last row: totals)
                       // or a histogram of segment lengths
    uint32_t segs;     // two segment lists of seg_cap packed (start | len << 16) u32
    uint32_t tmpk;     // seg_cap + 1 u32: children per segment, then their offsets
    uint32_t wl;       // seg_cap u32: segments split by one wave
    uint32_t misc;     // 64 u32 of scalars
    uint32_t seg_cap;  // entries of one segment list
    uint32_t total;    // bytes, the final staging copy of the elements overlays all
};

__host__ __device__ __forceinline__ LeafLayout leaf_layout(uint32_t T, uint32_t w, uint32_t kmax,
                                                           uint32_t n0)
{
    // A splitting segment of len items has k < 2*len/G children, G = max(1, n0/2);
    // one level therefore lists fewer than 2*T/G segments.
    uint32_t g = n0 / 2;
    if (g < 1) g = 1;
    const uint32_t seg_cap = 2u * T / g + 64u;
    LeafLayout L;
    L.idx = 0;
    L.lab = align16(T * 2u);
    L.hist = L.lab + align16(T + 32u);  // labels of whole 16-position blocks, plus slack
    // the counters also hold a 257-entry histogram of base-case segment lengths
    uint32_t hist_words = (kWaves + 1) * (kmax + 1);
    if (hist_words < 257u) hist_words = 257u;
    L.segs = L.hist + align16(hist_words * 4u);
    L.tmpk = L.segs + align16(2u * seg_cap * 4u);
    L.wl = L.tmpk + align16((seg_cap + 1) * 4u);
    L.misc = L.wl + align16(seg_cap * 4u);
    L.seg_cap = seg_cap;
    const uint32_t work = L.misc + 64u * 4u;
    const uint32_t stage = align16(T * w);
    L.total = work > stage ? work : stage;
    return L;
}

// ---- wave helpers (device) ----
// A value known to be the same in every lane of the wave, kept in a scalar
// register (loops and branches on it need no lane masks).
__device__ __forceinline__ uint32_t uniform(uint32_t v)
{
    return static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(v)));
}

// A workgroup barrier that waits only for this wave's LDS operations
// (lgkmcnt), not for its outstanding global loads -- among them direct
// global-to-LDS loads, which keep streaming while the workgroup works on
// other LDS data.  The memory clobber keeps the compiler from moving memory
// operations across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Start copying words [j0, nw) of a run, in chunks of 256 words from j0 on
// with a stride of `stride` words (a multiple of 256), from global memory
// straight into LDS (direct global-to-LDS loads: the data land in LDS
// without passing through registers).  Called by a whole wave.  Lane l
// moves words 4l .. 4l + 3 of a chunk with one 16-byte load; the at most
// three words past the last multiple of four move with 4-byte loads by the
// wave that starts at j0 = 0.  Addresses need only be 4-byte aligned.  The
// caller waits (vmcnt) and synchronises before reading the LDS copy.
__device__ __forceinline__ void copy_run_to_lds(const global_t<uint32_t>* src, uint32_t* dst, uint32_t nw,
                                                uint32_t j0, uint32_t stride, uint32_t lane)
{
    const uint32_t nv = nw & ~3u;
    for (uint32_t j = j0; j < nv; j += stride)
        if (j + 4u * lane < nv) __builtin_amdgcn_global_load_lds(src + j + 4u * lane, dst + j, 16, 0, 0);
    if (j0 == 0 && lane < nw - nv) __builtin_amdgcn_global_load_lds(src + nv + lane, dst + nv, 4, 0, 0);
}

// The workgroup barrier of every kernel here: this wave's LDS operations are
// complete before it (an explicit lgkmcnt(0) wait), so every LDS write made
// before the barrier is seen by every wave after it.  The wait is not left to
// the compiler's own wait placement, which has dropped it before a loop-top
// barrier (a store of one lane then raced with the other waves' loads).
__device__ __forceinline__ void block_sync()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);  // gfx9 encoding of lgkmcnt(0), other counters unchanged
    __syncthreads();
}


__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// The hardware hands the workgroups of a launch to the eight XCDs in turn
// (workgroup g to XCD g mod 8), and every XCD has its own L2.  Renumbering so
// that XCD x works through one contiguous run of the n work items keeps
// neighbouring items -- which share the cache lines at their boundaries -- in
// one L2 at about the same time.  A bijection of [0, n).
__device__ __forceinline__ uint32_t xcd_order(uint32_t g, uint32_t n)
{
    const uint32_t x = g & 7u, j = g >> 3, q = n >> 3, rem = n & 7u;
    return x * q + (x < rem ? x : rem) + j;
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t bits_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Inclusive prefix sum across the 64 lanes of a wave, with all 64 lanes
// active.  Data-parallel-primitive moves: a shift by 1, 2, 4, 8 lanes inside
// each row of 16 (lanes shifted in from outside the row contribute 0), then
// lane 15 of rows 0 and 2 added to rows 1 and 3, and lane 31 added to rows 2
// and 3.  Lanes a move does not write keep the initial 0.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v)
{
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xF, 0xF, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xF, 0xF, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xF, 0xF, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xF, 0xF, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xA, 0xF, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xC, 0xF, false));
    return v;
}

// Lanes of the wave whose KAPPA-bit label equals this lane's, among the
// active lanes: one ballot per label bit; the per-bit mask update
// acc & ~(t ^ m) is a single three-input bit operation.  Call it from code
// where exactly the lanes holding a valid label are active.
template <int KAPPA>
__device__ __forceinline__ uint64_t match_label_bits(uint32_t l)
{
    const uint64_t active = __builtin_amdgcn_read_exec();
    uint32_t lo = static_cast<uint32_t>(active), hi = static_cast<uint32_t>(active >> 32);
    uint32_t t[KAPPA];
    uint64_t m[KAPPA];
#pragma unroll
    for (int i = 0; i < KAPPA; ++i) {
        t[i] = static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int>(l), i, 1));
        // the ballot of bit i, written as the plain compare of the extracted
        // bit (the compiler otherwise re-derives the bit with extra shifts)
        asm volatile("v_cmp_ne_u32_e64 %0, 0, %1" : "=s"(m[i]) : "v"(t[i]));
    }
    // two wait states between the last compare and the first use of its result
    asm volatile("s_nop 1");
#pragma unroll
    for (int i = 0; i < KAPPA; ++i) {
        lo = __builtin_amdgcn_bitop3_b32(lo, t[i], static_cast<uint32_t>(m[i]), 0x90);
        hi = __builtin_amdgcn_bitop3_b32(hi, t[i], static_cast<uint32_t>(m[i] >> 32), 0x90);
    }
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Exclusive prefix sum of a[0..n) in place and a[n] = total; called by one
// whole wave.
__device__ __forceinline__ void wave_exclusive_scan(uint32_t* a, uint32_t n)
{
    const uint32_t lane = lane_id();
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n; base += 256) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t j = base + lane * 4 + i;
            v[i] = j < n ? a[j] : 0u;
            s += v[i];
        }
        const uint32_t incl = wave_inclusive_sum(s);
        uint32_t run = carry + incl - s;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t j = base + lane * 4 + i;
            if (j < n) a[j] = run;
            run += v[i];
        }
        carry += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), 63));
    }
    if (lane == 0) a[n] = carry;
}

// Largest i in [0, n) with a[i] <= x, for a non-decreasing a with a[0] <= x.
__device__ __forceinline__ uint32_t upper_index(const uint32_t* a, uint32_t n, uint32_t x)
{
    uint32_t lo = 0, hi = n;  // invariant: a[lo] <= x, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t upper_index64(const uint64_t* a, uint32_t n, uint64_t x)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace ipss
