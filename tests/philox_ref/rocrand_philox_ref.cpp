// Test-only helper: exposes rocRAND's own Philox4x32-10 block function on the
// host, so the CPU oracle's Philox can be checked against an independent,
// installed implementation.  Built for the host only; runs no GPU code.
#include <stdint.h>
#include <rocrand/rocrand_philox4x32_10.h>

namespace {
struct BlockProbe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};
}  // namespace

extern "C" void rocrand_philox_block(const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    BlockProbe probe;
    uint4 c = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint2 k = {key[0], key[1]};
    uint4 r = probe.block(c, k);
    out[0] = r.x;
    out[1] = r.y;
    out[2] = r.z;
    out[3] = r.w;
}
