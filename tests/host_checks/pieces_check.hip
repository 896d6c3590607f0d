// Host-only check (no GPU): the per-tile piece offsets (two per tile, from the
// level table) used by the tile, count and fix-up kernels give the same piece
// bounds as the direct formula piece_of (region b = [floor(b*m/k),
// floor((b+1)*m/k)), piece t starts at floor(t*len/P)), and the closed-form
// staging offsets equal the running sums of the piece sizes, for random
// subproblem sizes, bucket counts and tile counts, including sizes beyond
// 2^32; and the tile kernel's split of the pieces among its 16 waves covers
// every piece once.  Built with hipcc --cuda-host-only.
#include <cstdio>
#include <random>

#include "common.hpp"

using namespace ipss;

int main()
{
    std::mt19937_64 rng(7);
    long checked = 0;
    for (int it = 0; it < 20000; ++it) {
        const uint32_t kappa = 1 + static_cast<uint32_t>(rng() % 8);
        const uint64_t k = 1ull << kappa;
        uint64_t m;
        switch (it % 4) {
        case 0: m = rng() % 4096; break;
        case 1: m = rng() % (1ull << 22); break;
        case 2: m = rng() % (1ull << 34); break;
        default: m = (1ull << 32) + rng() % 100000; break;
        }
        const uint64_t tile = 1 + rng() % 16384;
        uint64_t P = m / (tile > k ? tile - k + 1 : 1) + 1;
        if (P > (1ull << 32)) P = 1ull << 32;
        for (int r = 0; r < 4; ++r) {
            const uint64_t t = rng() % P;
            // the level table's entries of tiles t and t + 1, as the maps kernel writes them
            const uint64_t len0 = m >> kappa;
            const uint64_t pofs[4] = {piece_offset(t, len0, P), piece_offset(t, len0 + 1, P),
                                      piece_offset(t + 1, len0, P), piece_offset(t + 1, len0 + 1, P)};
            const TilePieces tp(m, kappa, P, t, pofs);
            uint64_t before = 0;  // items of pieces 0 .. b-1
            for (uint32_t b = 0; b <= k; ++b) {
                if (tp.start(b) != static_cast<uint32_t>(before)) {
                    std::printf("start mismatch m=%llu kappa=%u P=%llu t=%llu b=%u\n",
                                static_cast<unsigned long long>(m), kappa,
                                static_cast<unsigned long long>(P),
                                static_cast<unsigned long long>(t), b);
                    return 1;
                }
                if (b == k) break;
                const Piece a = piece_of(m, kappa, P, t, b), c = tp.of(b);
                before += a.cap;
                if (a.lo != c.lo || a.cap != c.cap) {
                    std::printf("mismatch m=%llu kappa=%u P=%llu t=%llu b=%u\n",
                                static_cast<unsigned long long>(m), kappa,
                                static_cast<unsigned long long>(P),
                                static_cast<unsigned long long>(t), b);
                    return 1;
                }
                ++checked;
            }
        }
    }
    // The tile kernel's loads: wave w (of 16) takes the consecutive pieces
    // [w k / 16, (w + 1) k / 16); for every k these ranges cover [0, k) once.
    for (uint32_t kap = 0; kap <= 8; ++kap) {
        const uint32_t k = 1u << kap;
        uint32_t next = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            const uint32_t b0 = (w * k) >> 4, b1 = ((w + 1) * k) >> 4;
            if (b0 != next || b1 < b0) {
                std::printf("wave ranges k=%u w=%u: [%u, %u) after %u\n", k, w, b0, b1, next);
                return 1;
            }
            next = b1;
        }
        if (next != k) {
            std::printf("wave ranges k=%u end at %u\n", k, next);
            return 1;
        }
    }
    std::printf("ok %ld\n", checked);
    return 0;
}
