// Host planner and C ABI of the in-place ScatterShuffle.
//
// The recursion of arXiv 2302.03317 (Fig. 2, Theorem 1) is flattened level by
// level: all subproblems of one level that need the tiled pass share one
// rough-pass launch, one set of table kernels and one fix-up; all subproblems
// that fit a tile (from any level, any array) share one LDS leaf launch at
// the end.  After the tables of a level the host reads the exact bucket sizes
// (to plan the next level) and the number of movers (to size the workspace).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "ipscshuf.h"
#include "kernels.hpp"

namespace ipss {
namespace {

constexpr uint32_t kDefinitionVersion = 1;
constexpr uint64_t kMaxElements = 1ull << 40;

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap && p) return hipSuccess;
        if (p) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return e;
            e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = want;
        return hipSuccess;
    }
};

// Grow a device buffer to `bytes`, keeping its first `used` bytes.
hipError_t grow_keep(DevBuf& d, size_t bytes, size_t used, hipStream_t s)
{
    if (bytes <= d.cap && d.p) return hipSuccess;
    void* np = nullptr;
    const size_t want = std::max<size_t>(bytes + bytes / 2, 4096);
    hipError_t e = hipMalloc(&np, want);
    if (e != hipSuccess) return e;
    if (d.p && used) {
        e = hipMemcpyAsync(np, d.p, used, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            (void)hipFree(np);
            return e;
        }
    }
    if (d.p) {
        e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipFree(d.p);
        if (e != hipSuccess) return e;
    }
    d.p = np;
    d.cap = want;
    return hipSuccess;
}

struct HostBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap && p) return hipSuccess;
        if (p) {
            (void)hipHostFree(p);
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(bytes + bytes / 4, 4096);
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = want;
        return hipSuccess;
    }
    template <typename T> T* as() { return static_cast<T*>(p); }
};

struct Context {
    std::mutex mu;
    bool init = false;
    DevBuf subs, tile_sub, chunk_sub, bk_sub, cnt, mpre, kpre, chA, chB, N, S, M, K, MB, wsp, total, ws,
        leaves, leaves_cls, big, gfy, err, counters;
    HostBuf h_subs, h_tile_sub, h_chunk_sub, h_bk_sub, h_total, h_leaves, h_big, h_gfy, h_err,
        h_counters;
    shuf_stats_t stats{};
    // timing
    bool timing = false;
    shuf_kernel_time_t times[SHUF_KERNEL_KINDS]{};
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
    struct Span {
        hipEvent_t a, b;
        int kind;
        double bytes;
    };
    std::vector<Span> spans;
};

// Event pairs around launch groups when timing is on.
struct SpanGuard {
    Context& C;
    hipStream_t s;
    int kind;
    double bytes;
    hipEvent_t a = nullptr;
    SpanGuard(Context& c, hipStream_t st, int k, double by) : C(c), s(st), kind(k), bytes(by)
    {
        if (!C.timing) return;
        a = next_event();
        if (a) (void)hipEventRecord(a, s);
    }
    ~SpanGuard()
    {
        if (!C.timing || !a) return;
        hipEvent_t b = next_event();
        if (!b) return;
        (void)hipEventRecord(b, s);
        C.spans.push_back({a, b, kind, bytes});
    }
    hipEvent_t next_event()
    {
        if (C.events_used == C.event_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            C.event_pool.push_back(e);
        }
        return C.event_pool[C.events_used++];
    }
};

void collect_spans(Context& C)
{
    for (const Context::Span& sp : C.spans) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) {
            C.times[sp.kind].ms += ms;
            C.times[sp.kind].launches += 1;
            C.times[sp.kind].bytes += sp.bytes;
        }
    }
    C.spans.clear();
    C.events_used = 0;
}

constexpr int kMaxDevices = 64;
Context g_ctx[kMaxDevices];

struct HostSub {
    uint64_t elem_off, base, m;
    uint32_t level, stream_id;
};

struct ArraySpec {
    uint64_t elem_off, n;
    uint32_t stream_id;
};

uint32_t kappa_of(uint64_t m, bool tiled, const Params& p)
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
    return std::min(kap, p.kmax_log2);
}

int check_params(const shuf_params_t* p, uint32_t w)
{
    if (!p) return SHUF_EINVAL;
    if (p->kmax_log2 < 1 || p->kmax_log2 > 8) return SHUF_EINVAL;
    if (p->tile < (1u << p->kmax_log2) + 1) return SHUF_EINVAL;
    if (p->n0 < 1 || p->lmax > 255) return SHUF_EINVAL;
    if (static_cast<uint64_t>(p->tile) * w > kTileBytesMax) return SHUF_EUNSUPPORTED;
    const uint32_t kmax = 1u << p->kmax_log2;
    if (rough_layout(p->tile, w, kmax).total > kLdsBytesMax) return SHUF_EUNSUPPORTED;
    if (leaf_layout(p->tile, w, kmax, p->n0).total > kLdsBytesMax) return SHUF_EUNSUPPORTED;
    return SHUF_OK;
}

bool valid_width(uint32_t w) { return w == 4 || w == 8 || w == 16; }

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_error_code(e_); \
    } while (0)

int hip_error_code(hipError_t e)
{
    return e == hipErrorOutOfMemory ? SHUF_ENOMEM : SHUF_EHIP;
}

template <typename T>
hipError_t upload(DevBuf& d, HostBuf& h, const std::vector<T>& v, hipStream_t s)
{
    const size_t bytes = v.size() * sizeof(T);
    hipError_t e = d.ensure(bytes);
    if (e != hipSuccess) return e;
    e = h.ensure(bytes);
    if (e != hipSuccess) return e;
    if (bytes == 0) return hipSuccess;
    std::memcpy(h.p, v.data(), bytes);
    return hipMemcpyAsync(d.p, h.p, bytes, hipMemcpyHostToDevice, s);
}

int run(Context& C, uint8_t* buf, uint32_t w, uint64_t seed, const Params& prm,
        const std::vector<ArraySpec>& arrays, hipStream_t stream)
{
    if (!C.init) {
        HIP_TRY(set_rough_lds_limits());
        HIP_TRY(set_leaf_lds_limits());
        C.init = true;
    }
    shuf_stats_t st{};
    const uint32_t kmax = 1u << prm.kmax_log2;
    const uint64_t tile_limit = prm.tile - kmax;  // subproblems up to this size finish in LDS
    C.spans.clear();
    C.events_used = 0;
    HIP_TRY(C.err.ensure(4));
    HIP_TRY(C.h_err.ensure(4));
    HIP_TRY(hipMemsetAsync(C.err.p, 0, 4, stream));
    HIP_TRY(C.counters.ensure(24));
    HIP_TRY(C.h_counters.ensure(24));
    HIP_TRY(C.total.ensure(8));
    HIP_TRY(C.h_total.ensure(8));

    // Roots: arrays that fit a tile are leaves right away.
    std::vector<LeafDesc> root_leaves, gfy;
    std::vector<HostSub> cur;
    for (const ArraySpec& a : arrays) {
        if (a.n < 2) continue;
        if (a.n > tile_limit) cur.push_back({a.elem_off, 0, a.n, 0, a.stream_id});
        else root_leaves.push_back({a.elem_off, 0, a.n, 0, a.stream_id});
    }
    uint64_t nleaves = root_leaves.size();
    HIP_TRY(upload(C.leaves, C.h_leaves, root_leaves, stream));
    unsigned long long* hc = C.h_counters.as<unsigned long long>();
    hc[0] = nleaves;
    hc[1] = 0;
    hc[2] = 0;
    for (const LeafDesc& l : root_leaves) hc[2] += l.m;
    uint64_t leaf_elems = hc[2];
    HIP_TRY(hipMemcpyAsync(C.counters.p, hc, 24, hipMemcpyHostToDevice, stream));

    std::vector<SubDesc> subs;
    std::vector<uint32_t> tile_sub, chunk_sub, bk_sub;
    while (!cur.empty()) {
        std::vector<HostSub> tiled;
        for (const HostSub& s : cur) {
            if (s.m <= prm.n0 || s.level >= prm.lmax) gfy.push_back({s.elem_off, s.base, s.m, s.level, s.stream_id});
            else tiled.push_back(s);
        }
        cur.clear();
        if (tiled.empty()) break;

        subs.clear();
        tile_sub.clear();
        chunk_sub.clear();
        bk_sub.clear();
        uint64_t ntiles = 0, tab = 0, nchunks = 0, chtab = 0, nbk = 0;
        for (const HostSub& s : tiled) {
            SubDesc d{};
            d.elem_off = s.elem_off;
            d.base = s.base;
            d.m = s.m;
            d.kappa = kappa_of(s.m, true, prm);
            const uint64_t k = 1ull << d.kappa;
            d.tiles = (s.m + (prm.tile - k) - 1) / (prm.tile - k);
            if (d.tiles > (1ull << 32)) return SHUF_EUNSUPPORTED;
            d.tile_off = ntiles;
            d.tab_off = tab;
            d.chunk_off = nchunks;
            d.chtab_off = chtab;
            d.bk_off = static_cast<uint32_t>(nbk);
            d.level = s.level;
            d.stream_id = s.stream_id;
            const uint64_t nch = (d.tiles + kChunk - 1) / kChunk;
            ntiles += d.tiles;
            tab += d.tiles * k;
            nchunks += nch;
            chtab += nch * k;
            nbk += k;
            if (ntiles >= (1ull << 31) || nbk >= (1ull << 32)) return SHUF_EUNSUPPORTED;
            subs.push_back(d);
        }
        const uint32_t nsub = static_cast<uint32_t>(subs.size());
        tile_sub.resize(ntiles);
        chunk_sub.resize(nchunks);
        bk_sub.resize(nbk);
        uint64_t level_elems = 0;
        for (uint32_t i = 0; i < nsub; ++i) {
            const SubDesc& d = subs[i];
            std::fill(tile_sub.begin() + d.tile_off, tile_sub.begin() + d.tile_off + d.tiles, i);
            const uint64_t nch = (d.tiles + kChunk - 1) / kChunk;
            std::fill(chunk_sub.begin() + d.chunk_off, chunk_sub.begin() + d.chunk_off + nch, i);
            std::fill(bk_sub.begin() + d.bk_off, bk_sub.begin() + d.bk_off + (1u << d.kappa), i);
            level_elems += d.m;
        }
        HIP_TRY(upload(C.subs, C.h_subs, subs, stream));
        HIP_TRY(upload(C.tile_sub, C.h_tile_sub, tile_sub, stream));
        HIP_TRY(upload(C.chunk_sub, C.h_chunk_sub, chunk_sub, stream));
        HIP_TRY(upload(C.bk_sub, C.h_bk_sub, bk_sub, stream));
        HIP_TRY(C.cnt.ensure(tab * 4));
        HIP_TRY(C.mpre.ensure(tab * 8));
        HIP_TRY(C.kpre.ensure(tab * 8));
        HIP_TRY(C.chA.ensure(chtab * 8));
        HIP_TRY(C.chB.ensure(chtab * 8));
        HIP_TRY(C.N.ensure(nbk * 8));
        HIP_TRY(C.S.ensure(nbk * 8));
        HIP_TRY(C.M.ensure(nbk * 8));
        HIP_TRY(C.K.ensure(nbk * 8));
        HIP_TRY(C.MB.ensure(nbk * 8));
        HIP_TRY(C.wsp.ensure((nbk / kScanChunk + 2) * 8));
        HIP_TRY(grow_keep(C.leaves, (nleaves + nbk) * sizeof(LeafDesc), nleaves * sizeof(LeafDesc),
                          stream));
        HIP_TRY(C.big.ensure(nbk * sizeof(LeafDesc)));

        LevelTables T{};
        T.subs = static_cast<const SubDesc*>(C.subs.p);
        T.tile_sub = static_cast<const uint32_t*>(C.tile_sub.p);
        T.chunk_sub = static_cast<const uint32_t*>(C.chunk_sub.p);
        T.bk_sub = static_cast<const uint32_t*>(C.bk_sub.p);
        T.cnt = static_cast<uint32_t*>(C.cnt.p);
        T.mpre = static_cast<uint64_t*>(C.mpre.p);
        T.kpre = static_cast<uint64_t*>(C.kpre.p);
        T.chA = static_cast<uint64_t*>(C.chA.p);
        T.chB = static_cast<uint64_t*>(C.chB.p);
        T.N = static_cast<uint64_t*>(C.N.p);
        T.S = static_cast<uint64_t*>(C.S.p);
        T.M = static_cast<uint64_t*>(C.M.p);
        T.K = static_cast<uint64_t*>(C.K.p);
        T.MB = static_cast<uint64_t*>(C.MB.p);
        T.wsp = static_cast<uint64_t*>(C.wsp.p);
        T.total = static_cast<uint64_t*>(C.total.p);
        T.err = static_cast<uint32_t*>(C.err.p);
        T.nsubs = nsub;
        T.ntiles = ntiles;
        T.nchunks = nchunks;
        T.nbuckets = nbk;

        {
            SpanGuard g(C, stream, 0, 2.0 * level_elems * w);
            HIP_TRY(launch_rough(w, buf, T.subs, T.tile_sub, T.cnt, ntiles, seed, prm, stream));
        }
        {
            SpanGuard g(C, stream, 1, 0.0);
            HIP_TRY(launch_tables_sizes(T, stream));
            HIP_TRY(launch_tables_routes(T, stream));
            unsigned long long* dc = static_cast<unsigned long long*>(C.counters.p);
            HIP_TRY(hipMemsetAsync(dc + 1, 0, 8, stream));
            HIP_TRY(launch_children(T, static_cast<uint32_t>(tile_limit),
                                    static_cast<LeafDesc*>(C.leaves.p),
                                    static_cast<LeafDesc*>(C.big.p), dc, stream));
        }
        HIP_TRY(hipMemcpyAsync(C.h_total.p, T.total, 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(hc, C.counters.p, 24, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const uint64_t movers = C.h_total.as<uint64_t>()[0];
        nleaves = hc[0];
        leaf_elems = hc[2];
        const uint64_t nbig = hc[1];
        if (nbig) {
            HIP_TRY(C.h_big.ensure(nbig * sizeof(LeafDesc)));
            HIP_TRY(hipMemcpyAsync(C.h_big.p, C.big.p, nbig * sizeof(LeafDesc),
                                   hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            const LeafDesc* bl = C.h_big.as<LeafDesc>();
            for (uint64_t i = 0; i < nbig; ++i)
                cur.push_back({bl[i].elem_off, bl[i].base, bl[i].m, bl[i].level, bl[i].stream_id});
            // the device appends in no particular order; plan in position order
            std::sort(cur.begin(), cur.end(), [](const HostSub& a, const HostSub& b) {
                return a.elem_off != b.elem_off ? a.elem_off < b.elem_off : a.base < b.base;
            });
        }
        HIP_TRY(C.ws.ensure(std::max<uint64_t>(movers, 1) * w));
        T.ws_cap = movers;
        {
            SpanGuard g(C, stream, 2, 2.0 * movers * w);
            HIP_TRY(launch_gather(w, buf, static_cast<uint8_t*>(C.ws.p), T, stream));
        }
        {
            SpanGuard g(C, stream, 3, 2.0 * movers * w);
            HIP_TRY(launch_scatter(w, buf, static_cast<const uint8_t*>(C.ws.p), T, stream));
        }
        st.tiled_levels++;
        st.tiles += ntiles;
        st.movers += movers;
        st.workspace_bytes = std::max<uint64_t>(st.workspace_bytes, movers * w);
    }

    for (const LeafDesc& f : gfy)
        if (f.m > 0xFFFFFFFFull) return SHUF_EUNSUPPORTED;
    if (nleaves) {
        SpanGuard g(C, stream, 4, 2.0 * static_cast<double>(leaf_elems) * w);
        uint32_t caps[3];
        leaf_class_caps(w, prm, caps);
        HIP_TRY(C.leaves_cls.ensure(3 * nleaves * sizeof(LeafDesc)));
        unsigned long long* dc = static_cast<unsigned long long*>(C.counters.p);
        HIP_TRY(hipMemsetAsync(dc, 0, 24, stream));
        HIP_TRY(launch_leaf_classes(static_cast<const LeafDesc*>(C.leaves.p), nleaves,
                                    static_cast<LeafDesc*>(C.leaves_cls.p), nleaves, caps, dc,
                                    stream));
        HIP_TRY(hipMemcpyAsync(hc, dc, 24, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const uint64_t count[3] = {hc[0], hc[1], hc[2]};
        if (count[0] + count[1] + count[2] != nleaves) return SHUF_EHIP;
        HIP_TRY(launch_leaf(w, buf, static_cast<const LeafDesc*>(C.leaves_cls.p), count, nleaves,
                            seed, prm, caps, stream));
    }
    if (!gfy.empty()) {
        HIP_TRY(upload(C.gfy, C.h_gfy, gfy, stream));
        uint64_t elems = 0;
        for (const LeafDesc& l : gfy) elems += l.m;
        SpanGuard g(C, stream, 5, 2.0 * elems * w);
        HIP_TRY(launch_fy_global(w, buf, static_cast<const LeafDesc*>(C.gfy.p), gfy.size(), seed,
                                 stream));
    }
    HIP_TRY(hipMemcpyAsync(C.h_err.p, C.err.p, 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (C.h_err.as<uint32_t>()[0] != 0) return SHUF_EHIP;  // an index check failed in a kernel
    if (C.timing) collect_spans(C);
    st.leaves = nleaves;
    st.fy_fallback = gfy.size();
    C.stats = st;
    return SHUF_OK;
}

int run_locked(uint8_t* buf, uint32_t w, uint64_t seed, const shuf_params_t& p,
               const std::vector<ArraySpec>& arrays, void* stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SHUF_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return SHUF_EUNSUPPORTED;
    Context& C = g_ctx[dev];
    std::lock_guard<std::mutex> lock(C.mu);
    const Params prm{p.tile, p.kmax_log2, p.n0, p.lmax};
    return run(C, buf, w, seed, prm, arrays, static_cast<hipStream_t>(stream));
}

}  // namespace
}  // namespace ipss

using namespace ipss;

extern "C" {

uint32_t shuffle_definition_version(void) { return kDefinitionVersion; }

int shuf_default_params(uint64_t n, uint32_t elem_bytes, shuf_params_t* out)
{
    (void)n;
    if (!out || !valid_width(elem_bytes)) return SHUF_EINVAL;
    out->tile = kTileBytesMax / elem_bytes;
    out->kmax_log2 = 8;
    out->n0 = 64;
    out->lmax = 32;
    return SHUF_OK;
}

int shuffle_inplace_ex(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                       uint32_t stream_id, const shuf_params_t* params, void* stream)
{
    if (!valid_width(elem_bytes)) return SHUF_EINVAL;
    int rc = check_params(params, elem_bytes);
    if (rc != SHUF_OK) return rc;
    if (n <= 1) return SHUF_OK;
    if (!ptr) return SHUF_EINVAL;
    if (reinterpret_cast<uintptr_t>(ptr) % elem_bytes) return SHUF_EINVAL;
    if (n >= kMaxElements) return SHUF_EUNSUPPORTED;
    std::vector<ArraySpec> arrays{{0, n, stream_id}};
    return run_locked(static_cast<uint8_t*>(ptr), elem_bytes, seed, *params, arrays, stream);
}

int shuffle_inplace(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream)
{
    shuf_params_t p;
    int rc = shuf_default_params(n, elem_bytes, &p);
    if (rc != SHUF_OK) return rc;
    return shuffle_inplace_ex(ptr, n, elem_bytes, seed, 0, &p, stream);
}

int shuffle_batched(void* ptr, const uint64_t* offsets, uint64_t count, uint32_t elem_bytes,
                    uint64_t seed, void* stream)
{
    if (!valid_width(elem_bytes) || !offsets) return SHUF_EINVAL;
    if (count >= (1ull << 32)) return SHUF_EUNSUPPORTED;
    std::vector<ArraySpec> arrays;
    arrays.reserve(count);
    bool any = false;
    for (uint64_t j = 0; j < count; ++j) {
        if (offsets[j + 1] < offsets[j]) return SHUF_EINVAL;
        const uint64_t n = offsets[j + 1] - offsets[j];
        if (n >= kMaxElements || offsets[j + 1] >= (1ull << 48)) return SHUF_EUNSUPPORTED;
        if (n >= 2) any = true;
        arrays.push_back({offsets[j], n, static_cast<uint32_t>(j)});
    }
    if (!any) return SHUF_OK;
    if (!ptr) return SHUF_EINVAL;
    if (reinterpret_cast<uintptr_t>(ptr) % elem_bytes) return SHUF_EINVAL;
    shuf_params_t p;
    shuf_default_params(0, elem_bytes, &p);
    int rc = check_params(&p, elem_bytes);
    if (rc != SHUF_OK) return rc;
    return run_locked(static_cast<uint8_t*>(ptr), elem_bytes, seed, p, arrays, stream);
}

const char* shuffle_strerror(int code)
{
    switch (code) {
    case SHUF_OK: return "success";
    case SHUF_EINVAL: return "invalid argument";
    case SHUF_ENOMEM: return "out of device or pinned host memory";
    case SHUF_EHIP: return "HIP call or kernel launch failed";
    case SHUF_EUNSUPPORTED: return "unsupported size or parameters";
    default: return "unknown error";
    }
}

int shuffle_timing_enable(int on)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SHUF_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return SHUF_EUNSUPPORTED;
    Context& C = g_ctx[dev];
    std::lock_guard<std::mutex> lock(C.mu);
    C.timing = on != 0;
    for (auto& t : C.times) t = shuf_kernel_time_t{};
    C.spans.clear();
    C.events_used = 0;
    return SHUF_OK;
}

int shuffle_timing_read(shuf_kernel_time_t* out)
{
    if (!out) return SHUF_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SHUF_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return SHUF_EUNSUPPORTED;
    Context& C = g_ctx[dev];
    std::lock_guard<std::mutex> lock(C.mu);
    for (int i = 0; i < SHUF_KERNEL_KINDS; ++i) out[i] = C.times[i];
    return SHUF_OK;
}

int shuffle_last_stats(shuf_stats_t* out)
{
    if (!out) return SHUF_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SHUF_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return SHUF_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_ctx[dev].mu);
    *out = g_ctx[dev].stats;
    return SHUF_OK;
}

}  // extern "C"
