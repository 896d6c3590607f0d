// Counter-based randomness for the shuffle: Philox4x32-10 keyed by the seed,
// with (block, tag, stream) in the counter, so every label and every
// Fisher-Yates draw is a pure function of (seed, stream, level, position) and
// the permutation does not depend on how the GPU schedules the work
// (arXiv 2302.03317, Sec. 4: reproducible subtask generators).
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
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
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

// Lemire's multiply-and-reject: word x is accepted for bound s when the low
// half of x*s is at least 2^32 mod s; the high half is the draw.  The 32-bit
// word of position p is word (p mod 4) of block p / 4; a rejected word is
// replaced by the same word of the block with the next attempt number.  As
// 2^32 mod s < s, a low half of at least s is accepted without computing the
// threshold.  The attempt loop stops after 2^16 attempts so that it always
// terminates (2^16 rejections in a row have probability below 2^-65536).
// `first` is the attempt-0 block of position `pos`.
__device__ __forceinline__ Word4 fy_block(const Key& key, uint32_t level, uint64_t block,
                                          uint32_t attempt)
{
    return philox10(static_cast<uint32_t>(block), static_cast<uint32_t>(block >> 32),
                    level | (kPurposeFY << 8) | (attempt << 16), key.stream, key.k0, key.k1);
}

__device__ __forceinline__ uint32_t fy_draw_from(const Key& key, uint32_t level, uint64_t pos,
                                                 uint32_t bound, const Word4& first)
{
    const uint32_t j = static_cast<uint32_t>(pos & 3);
    uint64_t prod = static_cast<uint64_t>(word_of(first, j)) * bound;
    if (static_cast<uint32_t>(prod) < bound) {
        const uint32_t threshold = (0u - bound) % bound;  // 2^32 mod bound
        uint32_t attempt = 0;
        while (static_cast<uint32_t>(prod) < threshold && attempt < 65535u) {
            ++attempt;
            const Word4 v = fy_block(key, level, pos >> 2, attempt);
            prod = static_cast<uint64_t>(word_of(v, j)) * bound;
        }
    }
    return static_cast<uint32_t>(prod >> 32);
}

}  // namespace ipss
