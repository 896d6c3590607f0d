// Launch wrappers of the shuffle kernels (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace ipss {

// A 16-byte element, moved as one opaque vector of four words (the vector
// type keeps per-thread element arrays in registers).
using Elem16 = uint4;

// Every kernel addresses elements through the descriptors' element
// addresses (see elem_gptr) and keys its randomness with their seeds.

// Rough pass of one tiled level: one workgroup per tile.
hipError_t launch_rough(uint32_t w, const SubDesc* subs, const uint32_t* tile_sub,
                        const uint64_t* tile_pofs, uint32_t* cnt_tab, uint64_t ntiles,
                        const Params& prm, hipStream_t stream, const uint64_t* dsz = nullptr);
hipError_t set_rough_lds_limits();
// Whether one wave's same-address LDS atomic adds return in lane order on the
// current device (a probe kernel over random label patterns, run once);
// `d` is one device word of the caller's.
hipError_t probe_lds_lane_order(hipStream_t stream, unsigned long long* d, bool* lane_ordered);
// The count table of one tiled level without moving elements (planning).
hipError_t launch_count(const SubDesc* subs, const uint32_t* tile_sub, const uint64_t* tile_pofs,
                        uint32_t* cnt_tab, uint64_t ntiles, hipStream_t stream);

// Device tables of one tiled level (see k_fixup.hip).
struct LevelTables {
    const SubDesc* subs;
    const uint32_t* tile_sub;   // global tile -> subproblem
    const uint64_t* tile_pofs;  // [tile][2] piece offsets inside a region (see TilePieces)
    const uint32_t* chunk_sub;  // global chunk -> subproblem
    const uint32_t* bk_sub;     // global bucket -> subproblem
    uint32_t* cnt;              // [tile][bucket] counts from the rough pass
    uint64_t* mpre;             // [tile][bucket] movers of earlier tiles (exclusive)
    uint64_t* kpre;             // [tile][bucket] kept items of earlier tiles (exclusive)
    uint64_t* chA;              // [chunk][bucket] scratch sums / prefixes
    uint64_t* chB;
    uint64_t* N;                // [bucket] final sizes
    uint64_t* S;                // [bucket] final starts, relative to the subproblem
    uint64_t* M;                // [bucket] movers
    uint64_t* K;                // [bucket] kept items
    uint64_t* MB;               // [bucket] workspace start of the bucket's movers
    uint64_t* total;            // [1] workspace elements of the level
    uint64_t* wsp;              // [nbuckets / kScanChunk + 1] partial sums of the workspace scan
    uint32_t* err;              // [1] set non-zero by a kernel that finds an index out of range
    uint64_t ws_cap;            // workspace elements available to gather / scatter
    uint64_t nsubs, ntiles, nchunks, nbuckets;
    uint64_t max_chunks;        // most chunks of one subproblem
    // For a level planned on the device: its sizes {nsubs, ntiles, nchunks,
    // nbuckets} in device memory, the host's fields above then being upper
    // bounds that size the launches (blocks beyond the device's sizes leave
    // at once).  NULL for a level planned on the host.
    const uint64_t* dsz;
};

constexpr uint32_t kScanChunk = 4096;  // buckets per block of the workspace scan

// Children of a tiled level: those that fit a tile are appended to the leaf
// list (leaves[counters[0]++], counters[2] += elements), larger ones to the
// `big` list (big[counters[1]++]); children of at most one element are done.
// The order of either list does not affect the result.
hipError_t launch_children(const LevelTables& t, uint32_t tile_limit, LeafDesc* leaves,
                           LeafDesc* big, unsigned long long* counters, hipStream_t stream);

// Tile, chunk and bucket -> subproblem maps of a level (each subproblem's
// tile_off / chunk_off / bk_off start its ranges, in increasing order), and
// every tile's two piece offsets (see TilePieces).
hipError_t launch_level_maps(const SubDesc* subs, uint32_t nsub, uint64_t ntiles, uint64_t nchunks,
                             uint64_t nbuckets, uint32_t* tile_sub, uint64_t* tile_pofs,
                             uint32_t* chunk_sub, uint32_t* bk_sub, hipStream_t stream,
                             const uint64_t* dsz = nullptr);

// Counts -> final sizes and starts; movers, kept prefixes; workspace bases.
hipError_t launch_tables_sizes(const LevelTables& t, hipStream_t stream);
hipError_t launch_tables_routes(const LevelTables& t, hipStream_t stream);
// Fix-up: gather movers into the workspace, then scatter into free slots.
hipError_t launch_gather(uint32_t w, uint8_t* ws, const LevelTables& t, hipStream_t stream);
hipError_t launch_scatter(uint32_t w, const uint8_t* ws, const LevelTables& t,
                          hipStream_t stream);

// Subproblems that fit a tile: in-LDS levels and Fisher-Yates, launched per
// size class (small, medium, large: caps[0..2] items, LDS sized to match).
void leaf_class_caps(uint32_t w, const Params& prm, uint32_t* caps);
// (dn: the leaf count in device memory, n then being an upper bound)
hipError_t launch_leaf_classes(const LeafDesc* in, uint64_t n, LeafDesc* out, uint64_t stride,
                               const uint32_t* caps, unsigned long long* count, hipStream_t stream,
                               const unsigned long long* dn = nullptr);
// The leaves of class c are leaves[c * stride, c * stride + dcount[c]), the
// counts in device memory: persistent workgroups, as many as the device holds
// at once, take leaves from the per-class work counters qctr[0..2] (zero on
// entry) until none are left.
hipError_t launch_leaf_persistent(uint32_t w, const LeafDesc* leaves, const unsigned long long* dcount,
                                  uint64_t stride, const Params& prm, const uint32_t* caps,
                                  unsigned long long* qctr, hipStream_t stream);
hipError_t set_leaf_lds_limits();
// Device planning of a batched call's first level (see k_plan.hip), and two
// small helpers of the enqueue-only batched call.
hipError_t launch_plan_batched(const uint64_t* offsets, uint64_t count, uint64_t elem_base, uint64_t seed,
                               const Params& prm, uint64_t max_elems, uint64_t max_tiles, uint64_t max_chunks,
                               uint64_t max_buckets, uint64_t total_elems, SubDesc* subs, LeafDesc* leaves,
                               unsigned long long* counters, uint64_t* dsz, uint32_t* err, hipStream_t stream);
hipError_t launch_zero_words(uint32_t* p, uint32_t words, hipStream_t stream);
hipError_t launch_check_one_level(const unsigned long long* counters, uint32_t* err, hipStream_t stream);

// Sequential Fisher-Yates in global memory (recursion cap reached on a
// subproblem that does not fit a tile).
hipError_t launch_fy_global(uint32_t w, const LeafDesc* items, uint64_t count, hipStream_t stream);

}  // namespace ipss
