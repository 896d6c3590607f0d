// Counter-based randomness for the shuffle: Philox4x32-10 keyed by the seed,
// with (block, tag, stream) in the counter, so every label and every
// Fisher-Yates draw is a pure function of (seed, stream, level, position) and
// the permutation does not depend on how the GPU schedules the work
// (arXiv 2302.03317, Sec. 5: reproducible subtask generators).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipss {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products mixed with the key; the key advances by the two Weyl
// increments between rounds.
struct Word4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Word4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        // three-way exclusive or as one three-input bit operation (0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = static_cast<uint32_t>(p1);
        c2 = n2;
        c3 = static_cast<uint32_t>(p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Tag (counter word 2): level | purpose << 8 | attempt << 16.
constexpr uint32_t kPurposeLabel = 1u;
constexpr uint32_t kPurposeFY = 2u;

struct Key {
    uint32_t k0, k1, stream;
};

__device__ __forceinline__ Key make_key(uint64_t seed, uint32_t stream)
{
    return {static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), stream};
}

// The 16 label bytes of positions 16*B .. 16*B+15 at `level`; byte j of the
// result belongs to position 16*B + j.
__device__ __forceinline__ Word4 label_block(const Key& key, uint32_t level, uint64_t block)
{
    return philox10(static_cast<uint32_t>(block), static_cast<uint32_t>(block >> 32),
                    level | (kPurposeLabel << 8), key.stream, key.k0, key.k1);
}

__device__ __forceinline__ uint32_t word_of(const Word4& v, uint32_t i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Byte j (0..15) of a label block.
__device__ __forceinline__ uint32_t block_byte(const Word4& v, uint32_t j)
{
    return (word_of(v, j >> 2) >> (8 * (j & 3))) & 0xFFu;
}

// Fisher-Yates draws, Lemire's multiply-and-reject: a word x is accepted for
// bound s when the low half of x*s is at least (word range) mod s, and the
// high half is the draw; a rejected word is replaced by the same word of the
// block with the next attempt number.
//  - bounds up to 2^16 ("short"): 16-bit words, eight per Philox block
//    (position p uses half (p mod 2) -- low half first -- of word (p mod 8)/2
//    of block p / 8), tag purpose 3;
//  - larger bounds ("long"): 32-bit words, word p mod 4 of block p / 4, tag
//    purpose 2.
// Since (range mod s) < s, a low half of at least s is accepted without
// computing the threshold.  The attempt loops stop after 2^16 attempts so
// that they always terminate (2^16 rejections in a row have probability
// below 2^-65536).
constexpr uint32_t kPurposeFYShort = 3u;

__device__ __forceinline__ Word4 fy_short_block(const Key& key, uint32_t level, uint64_t block,
                                                uint32_t attempt)
{
    return philox10(static_cast<uint32_t>(block), static_cast<uint32_t>(block >> 32),
                    level | (kPurposeFYShort << 8) | (attempt << 16), key.stream, key.k0, key.k1);
}

// 16-bit word h (0..7) of a block.
__device__ __forceinline__ uint32_t half_of(const Word4& v, uint32_t h)
{
    return (word_of(v, h >> 1) >> (16 * (h & 1))) & 0xFFFFu;
}

// Short draw for position `pos` with bound <= 2^16, given its attempt-0 word.
__device__ __forceinline__ uint32_t fy_short_draw(const Key& key, uint32_t level, uint64_t pos,
                                                  uint32_t bound, uint32_t first_word)
{
    // 16-bit word times a bound <= 2^16: both fit 24 bits, the product 32
    uint32_t prod = __umul24(first_word, bound);
    if ((prod & 0xFFFFu) < bound) {
        const uint32_t threshold = 0x10000u % bound;
        uint32_t attempt = 0;
        while ((prod & 0xFFFFu) < threshold && attempt < 65535u) {
            ++attempt;
            const Word4 v = fy_short_block(key, level, pos >> 3, attempt);
            prod = __umul24(half_of(v, static_cast<uint32_t>(pos & 7)), bound);
        }
    }
    return prod >> 16;
}

__device__ __forceinline__ Word4 fy_block(const Key& key, uint32_t level, uint64_t block,
                                          uint32_t attempt)
{
    return philox10(static_cast<uint32_t>(block), static_cast<uint32_t>(block >> 32),
                    level | (kPurposeFY << 8) | (attempt << 16), key.stream, key.k0, key.k1);
}

// Long draw for position `pos` with bound in (2^16, 2^32).
__device__ __forceinline__ uint32_t fy_long_draw(const Key& key, uint32_t level, uint64_t pos,
                                                 uint32_t bound)
{
    const uint32_t j = static_cast<uint32_t>(pos & 3);
    const uint32_t threshold = (0u - bound) % bound;  // 2^32 mod bound
    uint64_t prod = 0;
    for (uint32_t attempt = 0; attempt < 65536u; ++attempt) {
        const Word4 v = fy_block(key, level, pos >> 2, attempt);
        prod = static_cast<uint64_t>(word_of(v, j)) * bound;
        if (static_cast<uint32_t>(prod) >= threshold) break;
    }
    return static_cast<uint32_t>(prod >> 32);
}

}  // namespace ipss
