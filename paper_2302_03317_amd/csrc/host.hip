// Host planner and C ABI of the in-place ScatterShuffle.
//
// The recursion of arXiv 2302.03317 (Fig. 2; Sec. 3.5, Theorem 1) is flattened into
// steps: in one step every waiting subproblem that needs the tiled pass gets
// one level (one shared rough-pass launch, one set of table kernels, one
// fix-up) and every waiting subproblem that fits a tile is finished in LDS
// (shared leaf launches by size class), whatever array, request or level it
// belongs to.  After the tables of a level the host reads the exact bucket
// sizes (to plan the next step) and the number of movers (to size the
// workspace).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "ipscshuf.h"
#include "kernels.hpp"

// Device memory of the allocation-free entry point (shuffle_inplace_noalloc):
// one array per device, part of this file's code object, held until the
// process ends.  Host code must not pass `scratch` itself to a kernel (on the
// host the name is a stand-in, not a device address): it takes the device
// address once per device with hipGetSymbolAddress and uses only that.
__device__ __align__(256) uint8_t scratch[64ull << 20];

namespace ipss {
namespace {

constexpr uint32_t kDefinitionVersion = 1;
constexpr uint64_t kMaxElements = 1ull << 40;

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    bool fixed = false;  // a region of memory the buffer does not own: never freed or grown
    void release()
    {
        if (p && !fixed) (void)hipFree(p);
        if (!fixed) {
            p = nullptr;
            cap = 0;
        }
    }
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap && p) return hipSuccess;
        if (fixed) return hipErrorOutOfMemory;
        if (p) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return e;
            e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        // half again as much, so that the sizes of later steps and calls,
        // which vary with the bucket sizes drawn, rarely force a regrowth
        // (a device-wide synchronization)
        size_t want = std::max<size_t>(bytes + bytes / 2, 4096);
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
    if (d.fixed) return hipErrorOutOfMemory;
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

// Where a step's device buffers come from: the device's pools (grown as
// needed and kept), a caller's workspace (a region reused by every step), or
// the pools while recording the largest step (planning a workspace).
struct Mem {
    enum Mode { kPool, kArena, kTally } mode = kPool;
    uint8_t* base = nullptr;
    uint64_t size = 0, off = 0, peak = 0;
    static uint64_t align(uint64_t b) { return (b + 255) & ~static_cast<uint64_t>(255); }
    void begin_step() { off = 0; }
    hipError_t take(DevBuf& pool, uint64_t bytes, void** out)
    {
        if (mode == kArena) {
            if (off + align(bytes) > size) return hipErrorOutOfMemory;
            *out = base + off;
            off += align(bytes);
            return hipSuccess;
        }
        const hipError_t e = pool.ensure(bytes);
        if (e != hipSuccess) return e;
        *out = pool.p;
        if (mode == kTally) {
            off += align(bytes);
            peak = std::max(peak, off);
        }
        return hipSuccess;
    }
};

struct HostBuf {
    void* p = nullptr;
    size_t cap = 0;
    bool fixed = false;  // a region of (pageable) host memory the buffer does not own
    void release()
    {
        if (p && !fixed) (void)hipHostFree(p);
        if (!fixed) {
            p = nullptr;
            cap = 0;
        }
    }
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap && p) return hipSuccess;
        if (fixed) return hipErrorOutOfMemory;
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

// Device leaf lists of an engine: leaves[which] holds the leaves of the next
// step, the other receives the children of the current one.
struct LeafLists {
    DevBuf leaves[2];
    HostBuf h_new;  // staging of newly submitted leaves
    void release()
    {
        leaves[0].release();
        leaves[1].release();
        h_new.release();
    }
};

// Host staging of one engine step: uploads of the level's subproblems and
// fallback items, read-backs of the level totals, counters, error flag and
// the subproblems of the next level.
struct HostSet {
    HostBuf subs, total, big, gfy, err, counters;
    void release()
    {
        for (HostBuf* h : {&subs, &total, &big, &gfy, &err, &counters}) h->release();
    }
};

// The allocation-free entry point's memory on one device: the static scratch
// array (its device address, taken once per device) split into the probe's
// word, two leaf lists and the per-step arena; host staging in a static
// pageable array.
constexpr uint64_t kScratchBytes = 64ull << 20;
constexpr uint64_t kScratchListBytes = 4ull << 20;  // each of the two leaf lists
constexpr uint64_t kScratchProbeBytes = 256;
constexpr uint64_t kNoAllocHostBytes = 256ull << 10;
constexpr uint64_t kNoAllocMaxDataBytes = 48ull << 20;  // larger arrays are rejected up front

struct NoAllocState {
    bool ready = false;
    uint8_t* scratch = nullptr;  // device address of `scratch` on this device
    LeafLists lists;
    HostSet host;
};

struct Context {
    std::mutex mu;
    LeafLists lists;  // used by blocking calls (under mu)
    bool init = false;
    bool rank_atomic = false;  // see Params::rank_atomic
    bool slot_search = false;  // see Params::slot_search (IPSCSHUF_SLOTS=search)
    DevBuf subs, tile_sub, tile_pofs, chunk_sub, bk_sub, cnt, mpre, kpre, chA, chB, N, S, M, K, MB, wsp, total, ws,
        leaves, leaves_cls, big, gfy, err, counters, probe;
    HostSet host;
    NoAllocState na;
    std::vector<SubDesc> hv_subs;  // the level's subproblems (kept to reuse its memory)
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

// Frees every device pool, pinned staging buffer and timing event the library
// holds, on every device it has used (later calls allocate them again).  Runs
// at process exit as well (registered once at the first call), so that none of
// it outlives the HIP runtime or a profiler attached to it.
void release_all()
{
    bool any = false;  // no HIP call at all unless a device was used
    for (int d = 0; d < kMaxDevices; ++d) {
        std::lock_guard<std::mutex> lock(g_ctx[d].mu);
        any = any || g_ctx[d].init;
    }
    if (!any) return;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) cur = -1;
    for (int d = 0; d < kMaxDevices; ++d) {
        Context& C = g_ctx[d];
        std::lock_guard<std::mutex> lock(C.mu);
        if (!C.init) continue;
        if (hipSetDevice(d) != hipSuccess) continue;
        (void)hipDeviceSynchronize();
        for (DevBuf* b : {&C.subs, &C.tile_sub, &C.tile_pofs, &C.chunk_sub, &C.bk_sub, &C.cnt, &C.mpre,
                          &C.kpre, &C.chA, &C.chB, &C.N, &C.S, &C.M, &C.K, &C.MB, &C.wsp, &C.total,
                          &C.ws, &C.leaves, &C.leaves_cls, &C.big, &C.gfy, &C.err, &C.counters, &C.probe})
            b->release();
        C.host.release();
        C.lists.release();
        for (hipEvent_t e : C.event_pool) (void)hipEventDestroy(e);
        C.event_pool.clear();
        C.spans.clear();
        C.events_used = 0;
    }
    if (cur >= 0) (void)hipSetDevice(cur);
}

std::once_flag g_exit_hook;

// Host staging of the allocation-free entry point, one static area per
// device (pageable: nothing is registered or pinned).
alignas(256) uint8_t g_noalloc_host[kMaxDevices][kNoAllocHostBytes];

// Set-up of the allocation-free entry point on the current device (under the
// context's lock): the device address of `scratch` on this device, and the
// fixed regions carved from it and from the static host area.
int noalloc_setup(Context& C, int dev)
{
    NoAllocState& na = C.na;
    if (na.ready) return SHUF_OK;
    static_assert(sizeof(scratch) == kScratchBytes, "scratch size");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return SHUF_EHIP;
    na.scratch = static_cast<uint8_t*>(ptr);
    for (int i = 0; i < 2; ++i) {
        na.lists.leaves[i].p = na.scratch + kScratchProbeBytes + i * kScratchListBytes;
        na.lists.leaves[i].cap = kScratchListBytes;
        na.lists.leaves[i].fixed = true;
    }
    // host area: new-leaf staging, subproblem uploads, fallback uploads,
    // next-level subproblems, and the small read-backs
    uint8_t* h = g_noalloc_host[dev];
    const uint64_t part = kNoAllocHostBytes / 4;
    HostBuf* bufs[4] = {&na.lists.h_new, &na.host.subs, &na.host.gfy, &na.host.big};
    for (int i = 0; i < 4; ++i) {
        bufs[i]->p = h + i * part;
        bufs[i]->cap = part - 256;
        bufs[i]->fixed = true;
    }
    HostBuf* small[3] = {&na.host.total, &na.host.err, &na.host.counters};
    for (int i = 0; i < 3; ++i) {
        small[i]->p = h + 3 * part + (part - 256) + 64 * i;
        small[i]->cap = 64;
        small[i]->fixed = true;
    }
    na.ready = true;
    return SHUF_OK;
}

struct HostSub {
    uint64_t elem_off, base, m, seed;
    uint32_t level, stream_id, owner;
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

// Copy a host vector to a device buffer taken from `mem` (staged through a
// pinned buffer); *out receives the device pointer.
template <typename T>
hipError_t upload(Mem& mem, DevBuf& d, HostBuf& h, const std::vector<T>& v, hipStream_t s,
                  void** out)
{
    const size_t bytes = v.size() * sizeof(T);
    hipError_t e = mem.take(d, bytes, out);
    if (e != hipSuccess) return e;
    e = h.ensure(bytes);
    if (e != hipSuccess) return e;
    if (bytes == 0) return hipSuccess;
    std::memcpy(h.p, v.data(), bytes);
    return hipMemcpyAsync(*out, h.p, bytes, hipMemcpyHostToDevice, s);
}

// Work of one engine: subproblems waiting for a tiled level and leaves
// waiting for the leaf launch, for any number of arrays ("requests").  One
// step runs one tiled level of every waiting subproblem and every waiting
// leaf; their children wait for the next step.  A request is complete after
// the first step in which it had no tiled subproblem: by then every leaf of
// it has run.  Blocking calls use a temporary engine; a session keeps one
// between steps, and new requests join at the next step.
struct Engine {
    uint32_t w = 0;
    Params prm{};
    std::vector<HostSub> cur;          // tiled subproblems (and fallback items) of the next step
    std::vector<LeafDesc> new_leaves;  // leaves of newly submitted arrays
    LeafLists* lists = nullptr;        // device leaf lists (the context's or a session's)
    int which = 0;
    uint64_t nleaves = 0, leaf_elems = 0;
    std::vector<uint64_t> ticket;  // owner slot -> ticket (0 = free)
    std::vector<uint32_t> free_slots;
    std::vector<uint64_t> done_queue;
    uint64_t next_ticket = 1, inflight = 0;
    bool broken = false;
    bool dry = false;  // planning run: counts and tables only, no element moves
    bool noalloc = false;  // every buffer from the static scratch: no allocation, no timing events
    HostSet* host = nullptr;  // host staging (the context's, or the static one)
    void* probe_buf = nullptr;  // device word for the lane-order probe (allocation-free runs)
    Mem mem;
};

// Timing off for the duration of a planning step.
struct TimingOff {
    Context& C;
    bool was;
    TimingOff(Context& c, bool off) : C(c), was(c.timing)
    {
        if (off) C.timing = false;
    }
    ~TimingOff() { C.timing = was; }
};

uint64_t engine_submit(Engine& E, uint64_t elem_addr, uint64_t n, uint64_t seed, uint32_t stream_id,
                       uint64_t ticket = 0)
{
    uint32_t slot;
    if (!E.free_slots.empty()) {
        slot = E.free_slots.back();
        E.free_slots.pop_back();
    } else {
        slot = static_cast<uint32_t>(E.ticket.size());
        E.ticket.push_back(0);
    }
    const uint64_t t = ticket ? ticket : E.next_ticket++;
    E.ticket[slot] = t;
    ++E.inflight;
    const uint64_t tile_limit = E.prm.tile - (1u << E.prm.kmax_log2);
    if (n >= 2) {
        if (n > tile_limit) E.cur.push_back({elem_addr, 0, n, seed, 0, stream_id, slot});
        else E.new_leaves.push_back({elem_addr, 0, n, seed, 0, stream_id, slot, 0});
    }
    return t;
}

// One step (see Engine).  Appends the tickets of completed requests to
// E.done_queue and adds the step's work to `st`.
int engine_step(Context& C, Engine& E, hipStream_t stream, shuf_stats_t& st)
{
    if (E.broken) return SHUF_EHIP;
    const uint32_t w = E.w;
    Params prm = E.prm;
    if (!C.init) {
        HIP_TRY(set_rough_lds_limits());
        HIP_TRY(set_leaf_lds_limits());
        // stable ranks by LDS atomics where the device serves them in lane
        // order; IPSCSHUF_RANK=ballot keeps the ballot method
        bool lane_ordered = false;
        void* pbuf = nullptr;
        if (E.noalloc) {
            pbuf = E.probe_buf;  // the first word of the static scratch
        } else {
            HIP_TRY(C.probe.ensure(kScratchProbeBytes));
            pbuf = C.probe.p;
        }
        HIP_TRY(probe_lds_lane_order(stream, static_cast<unsigned long long*>(pbuf), &lane_ordered));
        const char* rank_env = std::getenv("IPSCSHUF_RANK");
        C.rank_atomic = lane_ordered && !(rank_env && std::strcmp(rank_env, "ballot") == 0);
        const char* slot_env = std::getenv("IPSCSHUF_SLOTS");
        C.slot_search = slot_env && std::strcmp(slot_env, "search") == 0;
        C.init = true;
        std::call_once(g_exit_hook, [] { std::atexit(release_all); });
    }
    prm.rank_atomic = C.rank_atomic ? 1u : 0u;
    prm.slot_search = C.slot_search ? 1u : 0u;
    const uint32_t kmax = 1u << prm.kmax_log2;
    const uint64_t tile_limit = prm.tile - kmax;  // subproblems up to this size finish in LDS
    const bool dry = E.dry;
    TimingOff timing_guard(C, dry || E.noalloc);
    HostSet& H = *E.host;
    Mem& mem = E.mem;
    mem.begin_step();
    void *p_err, *p_counters, *p_total;
    HIP_TRY(mem.take(C.err, 4, &p_err));
    HIP_TRY(H.err.ensure(4));
    HIP_TRY(hipMemsetAsync(p_err, 0, 4, stream));
    HIP_TRY(mem.take(C.counters, 72, &p_counters));
    HIP_TRY(H.counters.ensure(48));
    HIP_TRY(mem.take(C.total, 8, &p_total));
    HIP_TRY(H.total.ensure(8));
    unsigned long long* dc = static_cast<unsigned long long*>(p_counters);
    unsigned long long* hc = H.counters.as<unsigned long long>();
    // [0] leaf children, [1] big children, [2] leaf child elements, [3..5] leaves per class,
    // [6..8] the leaf classes' work counters
    HIP_TRY(hipMemsetAsync(dc, 0, 72, stream));

    std::vector<uint8_t> had_tiled(E.ticket.size(), 0);

    // Leaves of newly submitted arrays join this step's leaf list.
    if (!E.new_leaves.empty()) {
        const size_t add = E.new_leaves.size() * sizeof(LeafDesc);
        DevBuf& L = E.lists->leaves[E.which];
        HIP_TRY(grow_keep(L, E.nleaves * sizeof(LeafDesc) + add, E.nleaves * sizeof(LeafDesc), stream));
        HIP_TRY(E.lists->h_new.ensure(add));
        std::memcpy(E.lists->h_new.p, E.new_leaves.data(), add);
        HIP_TRY(hipMemcpyAsync(static_cast<uint8_t*>(L.p) + E.nleaves * sizeof(LeafDesc),
                               E.lists->h_new.p, add, hipMemcpyHostToDevice, stream));
        for (const LeafDesc& l : E.new_leaves) E.leaf_elems += l.m;
        E.nleaves += E.new_leaves.size();
        E.new_leaves.clear();
    }
    const uint64_t run_leaves = E.nleaves, run_leaf_elems = E.leaf_elems;
    const LeafDesc* leaves_now = static_cast<const LeafDesc*>(E.lists->leaves[E.which].p);
    uint32_t caps[3];
    leaf_class_caps(w, prm, caps);
    void* p_cls = nullptr;
    if (run_leaves) {
        HIP_TRY(mem.take(C.leaves_cls, 3 * run_leaves * sizeof(LeafDesc), &p_cls));
        if (!dry)
            HIP_TRY(launch_leaf_classes(leaves_now, run_leaves, static_cast<LeafDesc*>(p_cls),
                                        run_leaves, caps, dc + 3, stream));
    }

    // Tiled level of every waiting subproblem; the recursion cap sends a
    // subproblem to the sequential fallback.
    std::vector<HostSub> tiled;
    std::vector<LeafDesc> gfy;
    for (const HostSub& s : E.cur) {
        if (s.m <= prm.n0 || s.level >= prm.lmax) {
            if (s.m > 0xFFFFFFFFull) return SHUF_EUNSUPPORTED;
            gfy.push_back({s.elem_off, s.base, s.m, s.seed, s.level, s.stream_id, s.owner, 0});
        } else {
            tiled.push_back(s);
            had_tiled[s.owner] = 1;
        }
    }
    E.cur.clear();

    std::vector<SubDesc>& subs = C.hv_subs;
    subs.clear();
    LevelTables T{};
    void* p_big = nullptr;
    uint64_t ntiles = 0;
    if (!tiled.empty()) {
        uint64_t tab = 0, nchunks = 0, chtab = 0, nbk = 0, max_chunks = 0;
        for (const HostSub& s : tiled) {
            SubDesc d{};
            d.elem_off = s.elem_off;
            d.base = s.base;
            d.m = s.m;
            d.seed = s.seed;
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
            d.owner = s.owner;
            const uint64_t nch = (d.tiles + kChunk - 1) / kChunk;
            ntiles += d.tiles;
            tab += d.tiles * k;
            nchunks += nch;
            if (nch > max_chunks) max_chunks = nch;
            chtab += nch * k;
            nbk += k;
            if (ntiles >= (1ull << 31) || nbk >= (1ull << 32)) return SHUF_EUNSUPPORTED;
            subs.push_back(d);
        }
        const uint32_t nsub = static_cast<uint32_t>(subs.size());
        uint64_t level_elems = 0;
        for (const SubDesc& d : subs) level_elems += d.m;
        void *p_subs, *p_tile_sub, *p_tile_pofs, *p_chunk_sub, *p_bk_sub, *p_cnt, *p_mpre, *p_kpre, *p_chA, *p_chB,
            *p_N, *p_S, *p_M, *p_K, *p_MB, *p_wsp;
        HIP_TRY(upload(mem, C.subs, H.subs, subs, stream, &p_subs));
        // tile / chunk / bucket -> subproblem maps, built on the device
        HIP_TRY(mem.take(C.tile_sub, ntiles * 4, &p_tile_sub));
        HIP_TRY(mem.take(C.tile_pofs, ntiles * 16, &p_tile_pofs));
        HIP_TRY(mem.take(C.chunk_sub, nchunks * 4, &p_chunk_sub));
        HIP_TRY(mem.take(C.bk_sub, nbk * 4, &p_bk_sub));
        HIP_TRY(launch_level_maps(static_cast<const SubDesc*>(p_subs), nsub, ntiles, nchunks, nbk,
                                  static_cast<uint32_t*>(p_tile_sub), static_cast<uint64_t*>(p_tile_pofs),
                                  static_cast<uint32_t*>(p_chunk_sub), static_cast<uint32_t*>(p_bk_sub),
                                  stream));
        HIP_TRY(mem.take(C.cnt, tab * 4, &p_cnt));
        HIP_TRY(mem.take(C.mpre, tab * 8, &p_mpre));
        HIP_TRY(mem.take(C.kpre, tab * 8, &p_kpre));
        HIP_TRY(mem.take(C.chA, chtab * 8, &p_chA));
        HIP_TRY(mem.take(C.chB, chtab * 8, &p_chB));
        HIP_TRY(mem.take(C.N, nbk * 8, &p_N));
        HIP_TRY(mem.take(C.S, nbk * 8, &p_S));
        HIP_TRY(mem.take(C.M, nbk * 8, &p_M));
        HIP_TRY(mem.take(C.K, nbk * 8, &p_K));
        HIP_TRY(mem.take(C.MB, nbk * 8, &p_MB));
        HIP_TRY(mem.take(C.wsp, (nbk / kScanChunk + 2) * 8, &p_wsp));
        HIP_TRY(E.lists->leaves[1 - E.which].ensure(nbk * sizeof(LeafDesc)));
        HIP_TRY(mem.take(C.big, nbk * sizeof(LeafDesc), &p_big));

        T.subs = static_cast<const SubDesc*>(p_subs);
        T.tile_sub = static_cast<const uint32_t*>(p_tile_sub);
        T.tile_pofs = static_cast<const uint64_t*>(p_tile_pofs);
        T.chunk_sub = static_cast<const uint32_t*>(p_chunk_sub);
        T.bk_sub = static_cast<const uint32_t*>(p_bk_sub);
        T.cnt = static_cast<uint32_t*>(p_cnt);
        T.mpre = static_cast<uint64_t*>(p_mpre);
        T.kpre = static_cast<uint64_t*>(p_kpre);
        T.chA = static_cast<uint64_t*>(p_chA);
        T.chB = static_cast<uint64_t*>(p_chB);
        T.N = static_cast<uint64_t*>(p_N);
        T.S = static_cast<uint64_t*>(p_S);
        T.M = static_cast<uint64_t*>(p_M);
        T.K = static_cast<uint64_t*>(p_K);
        T.MB = static_cast<uint64_t*>(p_MB);
        T.wsp = static_cast<uint64_t*>(p_wsp);
        T.total = static_cast<uint64_t*>(p_total);
        T.err = static_cast<uint32_t*>(p_err);
        T.nsubs = nsub;
        T.ntiles = ntiles;
        T.nchunks = nchunks;
        T.nbuckets = nbk;
        T.max_chunks = max_chunks;
        if (dry) {
            HIP_TRY(launch_count(T.subs, T.tile_sub, T.tile_pofs, T.cnt, ntiles, stream));
        } else {
            SpanGuard g(C, stream, 0, 2.0 * level_elems * w);
            HIP_TRY(launch_rough(w, T.subs, T.tile_sub, T.tile_pofs, T.cnt, ntiles, prm, stream));
        }
        {
            SpanGuard g(C, stream, 1, 0.0);
            HIP_TRY(launch_tables_sizes(T, stream));
            HIP_TRY(launch_tables_routes(T, stream));
            HIP_TRY(launch_children(T, static_cast<uint32_t>(tile_limit),
                                    static_cast<LeafDesc*>(E.lists->leaves[1 - E.which].p),
                                    static_cast<LeafDesc*>(p_big), dc, stream));
        }
        HIP_TRY(hipMemcpyAsync(H.total.p, T.total, 8, hipMemcpyDeviceToHost, stream));
    }
    HIP_TRY(hipMemcpyAsync(hc, dc, 48, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const uint64_t child_leaves = hc[0], nbig = hc[1], child_elems = hc[2];
    const uint64_t count[3] = {hc[3], hc[4], hc[5]};
    if (!dry && run_leaves && count[0] + count[1] + count[2] != run_leaves) {
        E.broken = true;
        return SHUF_EHIP;
    }

    if (!tiled.empty()) {
        const uint64_t movers = H.total.as<uint64_t>()[0];
        if (nbig) {
            HIP_TRY(H.big.ensure(nbig * sizeof(LeafDesc)));
            HIP_TRY(hipMemcpyAsync(H.big.p, p_big, nbig * sizeof(LeafDesc),
                                   hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            const LeafDesc* bl = H.big.as<LeafDesc>();
            for (uint64_t i = 0; i < nbig; ++i)
                E.cur.push_back({bl[i].elem_off, bl[i].base, bl[i].m, bl[i].seed, bl[i].level,
                                 bl[i].stream_id, bl[i].owner});
            // (the device appends in no particular order; a level's results do not
            // depend on the order of its subproblems)
        }
        void* p_ws;
        HIP_TRY(mem.take(C.ws, std::max<uint64_t>(movers, 1) * w, &p_ws));
        T.ws_cap = movers;
        if (!dry) {
            {
                SpanGuard g(C, stream, 2, 2.0 * movers * w);
                HIP_TRY(launch_gather(w, static_cast<uint8_t*>(p_ws), T, stream));
            }
            {
                SpanGuard g(C, stream, 3, 2.0 * movers * w);
                HIP_TRY(launch_scatter(w, static_cast<const uint8_t*>(p_ws), T, stream));
            }
        }
        st.tiled_levels++;
        st.tiles += ntiles;
        st.movers += movers;
        st.workspace_bytes = std::max<uint64_t>(st.workspace_bytes, movers * w);
    }
    if (run_leaves && !dry) {
        SpanGuard g(C, stream, 4, 2.0 * static_cast<double>(run_leaf_elems) * w);
        HIP_TRY(launch_leaf_persistent(w, static_cast<const LeafDesc*>(p_cls), dc + 3, run_leaves, prm, caps,
                                       dc + 6, stream));
    }
    if (!gfy.empty()) {
        void* p_gfy;
        HIP_TRY(upload(mem, C.gfy, H.gfy, gfy, stream, &p_gfy));
        uint64_t elems = 0;
        for (const LeafDesc& l : gfy) elems += l.m;
        if (!dry) {
            SpanGuard g(C, stream, 5, 2.0 * elems * w);
            HIP_TRY(launch_fy_global(w, static_cast<const LeafDesc*>(p_gfy), gfy.size(), stream));
        }
    }
    HIP_TRY(hipMemcpyAsync(H.err.p, p_err, 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (H.err.as<uint32_t>()[0] != 0) {  // an index check failed in a kernel
        E.broken = true;
        return SHUF_EHIP;
    }
    if (C.timing) collect_spans(C);
    st.leaves += run_leaves;
    st.fy_fallback += gfy.size();

    // Children leaves wait for the next step.
    E.which = 1 - E.which;
    E.nleaves = child_leaves;
    E.leaf_elems = child_elems;
    for (uint32_t slot = 0; slot < E.ticket.size(); ++slot) {
        if (E.ticket[slot] == 0 || had_tiled[slot]) continue;
        E.done_queue.push_back(E.ticket[slot]);
        E.ticket[slot] = 0;
        E.free_slots.push_back(slot);
        --E.inflight;
    }
    return SHUF_OK;
}

Context* current_context(int* dev_out = nullptr)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    if (dev_out) *dev_out = dev;
    return &g_ctx[dev];
}

// Run an engine's submitted work to completion, under the context's lock.
int engine_run_locked(Context& C, Engine& E, void* stream)
{
    C.spans.clear();
    C.events_used = 0;
    if (!E.lists) E.lists = &C.lists;
    if (!E.host) E.host = &C.host;
    shuf_stats_t st{};
    while (E.inflight) {
        const int rc = engine_step(C, E, static_cast<hipStream_t>(stream), st);
        if (rc != SHUF_OK) return rc;
    }
    if (!E.dry) C.stats = st;
    return SHUF_OK;
}

// Run an engine's submitted work to completion (blocking calls).
int engine_drain(Engine& E, void* stream)
{
    Context* C = current_context();
    if (!C) return SHUF_EHIP;
    std::lock_guard<std::mutex> lock(C->mu);
    return engine_run_locked(*C, E, stream);
}

Engine make_engine(uint32_t w, const shuf_params_t& p)
{
    Engine E;
    E.w = w;
    E.prm = Params{p.tile, p.kmax_log2, p.n0, p.lmax, 0, 0};
    return E;
}

}  // namespace
}  // namespace ipss

using namespace ipss;

extern "C" {

uint32_t shuffle_definition_version(void) { return kDefinitionVersion; }

int shuffle_rank_method(void)
{
    Context* C = current_context();
    if (!C) return -1;
    std::lock_guard<std::mutex> lock(C->mu);
    return C->init ? (C->rank_atomic ? 1 : 0) : -1;
}

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
    Engine E = make_engine(elem_bytes, *params);
    engine_submit(E, reinterpret_cast<uintptr_t>(ptr) / elem_bytes, n, seed, stream_id);
    return engine_drain(E, stream);
}

int shuffle_workspace_bytes(uint64_t n, uint32_t elem_bytes, uint64_t seed, uint32_t stream_id,
                            const shuf_params_t* params, uint64_t* out_bytes, void* stream)
{
    if (!out_bytes || !valid_width(elem_bytes)) return SHUF_EINVAL;
    int rc = check_params(params, elem_bytes);
    if (rc != SHUF_OK) return rc;
    *out_bytes = 0;
    if (n <= 1) return SHUF_OK;
    if (n >= kMaxElements) return SHUF_EUNSUPPORTED;
    Engine E = make_engine(elem_bytes, *params);
    E.dry = true;
    E.mem.mode = Mem::kTally;
    engine_submit(E, 0, n, seed, stream_id);  // a planning run never touches elements
    rc = engine_drain(E, stream);
    if (rc != SHUF_OK) return rc;
    *out_bytes = E.mem.peak;
    return SHUF_OK;
}

int shuffle_inplace_ws(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                       uint32_t stream_id, const shuf_params_t* params, void* workspace,
                       uint64_t workspace_bytes, void* stream)
{
    if (!valid_width(elem_bytes)) return SHUF_EINVAL;
    int rc = check_params(params, elem_bytes);
    if (rc != SHUF_OK) return rc;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return SHUF_EINVAL;
    if (!workspace && workspace_bytes) return SHUF_EINVAL;
    if (n <= 1) return SHUF_OK;
    if (!ptr) return SHUF_EINVAL;
    if (reinterpret_cast<uintptr_t>(ptr) % elem_bytes) return SHUF_EINVAL;
    if (n >= kMaxElements) return SHUF_EUNSUPPORTED;
    Engine E = make_engine(elem_bytes, *params);
    E.mem.mode = Mem::kArena;
    E.mem.base = static_cast<uint8_t*>(workspace);
    E.mem.size = workspace_bytes;
    engine_submit(E, reinterpret_cast<uintptr_t>(ptr) / elem_bytes, n, seed, stream_id);
    return engine_drain(E, stream);
}

int shuffle_inplace_noalloc(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                            uint32_t stream_id, const shuf_params_t* params, void* stream)
{
    if (!valid_width(elem_bytes)) return SHUF_EINVAL;
    int rc = check_params(params, elem_bytes);
    if (rc != SHUF_OK) return rc;
    if (n <= 1) return SHUF_OK;
    if (!ptr) return SHUF_EINVAL;
    if (reinterpret_cast<uintptr_t>(ptr) % elem_bytes) return SHUF_EINVAL;
    if (n >= kMaxElements || n * elem_bytes > kNoAllocMaxDataBytes) return SHUF_EUNSUPPORTED;
    int dev = 0;
    Context* C = current_context(&dev);
    if (!C) return SHUF_EHIP;
    std::lock_guard<std::mutex> lock(C->mu);
    rc = noalloc_setup(*C, dev);
    if (rc != SHUF_OK) return rc;
    NoAllocState& na = C->na;
    const uint64_t lead = kScratchProbeBytes + 2 * kScratchListBytes;
    // A planning run in the scratch first: every buffer of every step is
    // taken exactly as in the shuffle itself, so a shortage is reported
    // before any element moves.
    for (int pass = 0; pass < 2; ++pass) {
        Engine E = make_engine(elem_bytes, *params);
        E.noalloc = true;
        E.dry = pass == 0;
        E.mem.mode = Mem::kArena;
        E.mem.base = na.scratch + lead;
        E.mem.size = kScratchBytes - lead;
        E.lists = &na.lists;
        E.host = &na.host;
        E.probe_buf = na.scratch;
        engine_submit(E, reinterpret_cast<uintptr_t>(ptr) / elem_bytes, n, seed, stream_id);
        rc = engine_run_locked(*C, E, stream);
        if (rc != SHUF_OK) return rc;
    }
    return SHUF_OK;
}

int shuffle_inplace(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream)
{
    shuf_params_t p;
    int rc = shuf_default_params(n, elem_bytes, &p);
    if (rc != SHUF_OK) return rc;
    return shuffle_inplace_ex(ptr, n, elem_bytes, seed, 0, &p, stream);
}

// ---- the enqueue-only batched call ----
// Workspace layout, all parts 256-byte aligned: a header (error word, level
// counters, device sizes, work counters, class counts, mover total), then the
// level's descriptors and tables sized for upper bounds that follow from
// (count, total_elems), the leaf lists, and the movers' workspace.
struct AsyncLayout {
    uint64_t max_tiles, max_chunks, max_buckets, max_leaves, max_tab, max_chtab, nparts;
    uint64_t header, subs, tile_sub, tile_pofs, chunk_sub, bk_sub, cnt, mpre, kpre, chA, chB, N, S, M, K, MB,
        wsp, leaves, leaves_cls, big, ws, total;
};
constexpr uint64_t kAsyncHeaderBytes = 256;  // err (4) | counters (48) | dsz (32) | qctr (24) | cls (24) | total (8)
constexpr uint64_t kAsyncMaxCount = 1ull << 22;

AsyncLayout async_layout(uint64_t count, uint64_t total_elems, uint32_t w, const Params& prm)
{
    AsyncLayout L{};
    const uint64_t kmax = 1ull << prm.kmax_log2;
    L.max_tiles = total_elems / (prm.tile - kmax) + count;
    L.max_chunks = L.max_tiles / kChunk + count;
    L.max_buckets = count * kmax;
    L.max_leaves = count + L.max_buckets;
    L.max_tab = L.max_tiles * kmax;
    L.max_chtab = L.max_chunks * kmax;
    L.nparts = L.max_buckets / kScanChunk + 1;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = off;
        off += Mem::align(std::max<uint64_t>(bytes, 1));
        return at;
    };
    L.header = take(kAsyncHeaderBytes);
    L.subs = take(count * sizeof(SubDesc));
    L.tile_sub = take(L.max_tiles * 4);
    L.tile_pofs = take(L.max_tiles * 16);
    L.chunk_sub = take(L.max_chunks * 4);
    L.bk_sub = take(L.max_buckets * 4);
    L.cnt = take(L.max_tab * 4);
    L.mpre = take(L.max_tab * 8);
    L.kpre = take(L.max_tab * 8);
    L.chA = take(L.max_chtab * 8);
    L.chB = take(L.max_chtab * 8);
    L.N = take(L.max_buckets * 8);
    L.S = take(L.max_buckets * 8);
    L.M = take(L.max_buckets * 8);
    L.K = take(L.max_buckets * 8);
    L.MB = take(L.max_buckets * 8);
    L.wsp = take((L.nparts + 2) * 8);
    L.leaves = take(L.max_leaves * sizeof(LeafDesc));
    L.leaves_cls = take(3 * L.max_leaves * sizeof(LeafDesc));
    L.big = take(L.max_buckets * sizeof(LeafDesc));
    L.ws = take(total_elems * w);
    L.total = off;
    return L;
}

int shuffle_batched(void* ptr, const uint64_t* offsets, uint64_t count, uint32_t elem_bytes,
                    uint64_t seed, void* stream)
{
    return shuffle_batched_ex(ptr, offsets, count, elem_bytes, seed, nullptr, stream);
}

// Parameters of a batched call: the caller's, or the defaults for the width.
static int batched_params(const shuf_params_t* params, uint32_t w, shuf_params_t* out)
{
    if (params) {
        *out = *params;
    } else {
        const int rc = shuf_default_params(0, w, out);
        if (rc != SHUF_OK) return rc;
    }
    return check_params(out, w);
}

int shuffle_batched_ex(void* ptr, const uint64_t* offsets, uint64_t count, uint32_t elem_bytes,
                       uint64_t seed, const shuf_params_t* params, void* stream)
{
    if (!valid_width(elem_bytes) || !offsets) return SHUF_EINVAL;
    if (count >= (1ull << 32)) return SHUF_EUNSUPPORTED;
    bool any = false;
    for (uint64_t j = 0; j < count; ++j) {
        if (offsets[j + 1] < offsets[j]) return SHUF_EINVAL;
        const uint64_t n = offsets[j + 1] - offsets[j];
        if (n >= kMaxElements || offsets[j + 1] >= (1ull << 48)) return SHUF_EUNSUPPORTED;
        if (n >= 2) any = true;
    }
    if (!any) return SHUF_OK;
    if (!ptr) return SHUF_EINVAL;
    if (reinterpret_cast<uintptr_t>(ptr) % elem_bytes) return SHUF_EINVAL;
    shuf_params_t p;
    int rc = batched_params(params, elem_bytes, &p);
    if (rc != SHUF_OK) return rc;
    Engine E = make_engine(elem_bytes, p);
    const uint64_t base = reinterpret_cast<uintptr_t>(ptr) / elem_bytes;
    for (uint64_t j = 0; j < count; ++j)
        if (offsets[j + 1] - offsets[j] >= 2)
            engine_submit(E, base + offsets[j], offsets[j + 1] - offsets[j], seed,
                          static_cast<uint32_t>(j));
    return engine_drain(E, stream);
}

int shuffle_batched_async_workspace_bytes(uint64_t count, uint64_t total_elems, uint32_t elem_bytes,
                                          const shuf_params_t* params, uint64_t* out_bytes)
{
    if (!out_bytes || !valid_width(elem_bytes)) return SHUF_EINVAL;
    shuf_params_t p;
    const int rc = batched_params(params, elem_bytes, &p);
    if (rc != SHUF_OK) return rc;
    if (count == 0 || count > kAsyncMaxCount || total_elems >= kMaxElements) return SHUF_EUNSUPPORTED;
    *out_bytes = async_layout(count, total_elems, elem_bytes, Params{p.tile, p.kmax_log2, p.n0, p.lmax, 0, 0}).total;
    return SHUF_OK;
}

uint64_t shuffle_batched_async_max_elems(uint32_t elem_bytes, const shuf_params_t* params)
{
    if (!valid_width(elem_bytes)) return 0;
    shuf_params_t p;
    if (batched_params(params, elem_bytes, &p) != SHUF_OK) return 0;
    // one tiled level leaves subproblems that fit a tile: kappa covers every
    // label bit the size needs when (T / 2) * 2^KMAXLOG2 >= n
    return static_cast<uint64_t>(p.tile / 2) << p.kmax_log2;
}

int shuffle_batched_async(void* ptr, const uint64_t* offsets, uint64_t count, uint32_t elem_bytes,
                          uint64_t seed, const shuf_params_t* params, uint64_t total_elems, void* workspace,
                          uint64_t workspace_bytes, void* stream)
{
    if (!valid_width(elem_bytes) || !offsets || !workspace) return SHUF_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 || reinterpret_cast<uintptr_t>(offsets) % 8)
        return SHUF_EINVAL;
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % elem_bytes) return SHUF_EINVAL;
    shuf_params_t sp;
    int rc = batched_params(params, elem_bytes, &sp);
    if (rc != SHUF_OK) return rc;
    if (count == 0 || count > kAsyncMaxCount || total_elems >= kMaxElements) return SHUF_EUNSUPPORTED;
    Params prm{sp.tile, sp.kmax_log2, sp.n0, sp.lmax, 0, 0};
    const AsyncLayout L = async_layout(count, total_elems, elem_bytes, prm);
    if (workspace_bytes < L.total) return SHUF_ENOMEM;
    Context* C = current_context();
    if (!C) return SHUF_EHIP;
    std::lock_guard<std::mutex> lock(C->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!C->init) {
        // the device's first call: LDS limits and the lane-order probe (it
        // synchronises the stream, so it must not happen under capture)
        HIP_TRY(set_rough_lds_limits());
        HIP_TRY(set_leaf_lds_limits());
        bool lane_ordered = false;
        HIP_TRY(C->probe.ensure(kScratchProbeBytes));
        HIP_TRY(probe_lds_lane_order(st, static_cast<unsigned long long*>(C->probe.p), &lane_ordered));
        const char* rank_env = std::getenv("IPSCSHUF_RANK");
        C->rank_atomic = lane_ordered && !(rank_env && std::strcmp(rank_env, "ballot") == 0);
        const char* slot_env = std::getenv("IPSCSHUF_SLOTS");
        C->slot_search = slot_env && std::strcmp(slot_env, "search") == 0;
        C->init = true;
        std::call_once(g_exit_hook, [] { std::atexit(release_all); });
    }
    prm.rank_atomic = C->rank_atomic ? 1u : 0u;
    prm.slot_search = C->slot_search ? 1u : 0u;
    uint8_t* W = static_cast<uint8_t*>(workspace);
    uint32_t* err = reinterpret_cast<uint32_t*>(W + L.header);
    unsigned long long* counters = reinterpret_cast<unsigned long long*>(W + L.header + 8);  // 6 words
    uint64_t* dsz = reinterpret_cast<uint64_t*>(W + L.header + 56);                           // 4 words
    unsigned long long* qctr = reinterpret_cast<unsigned long long*>(W + L.header + 88);      // 3 words
    unsigned long long* cls = reinterpret_cast<unsigned long long*>(W + L.header + 112);      // 3 words
    uint64_t* total = reinterpret_cast<uint64_t*>(W + L.header + 136);
    const uint64_t kmax = 1ull << prm.kmax_log2;
    const uint64_t tile_limit = prm.tile - kmax;
    const uint64_t max_elems = std::min<uint64_t>(shuffle_batched_async_max_elems(elem_bytes, &sp), total_elems);

    HIP_TRY(launch_zero_words(err, static_cast<uint32_t>(kAsyncHeaderBytes / 4), st));
    SubDesc* subs = reinterpret_cast<SubDesc*>(W + L.subs);
    LeafDesc* leaves = reinterpret_cast<LeafDesc*>(W + L.leaves);
    HIP_TRY(launch_plan_batched(offsets, count, reinterpret_cast<uintptr_t>(ptr) / elem_bytes, seed, prm,
                                max_elems, L.max_tiles, L.max_chunks, L.max_buckets, total_elems, subs, leaves,
                                counters, dsz, err, st));
    LevelTables T{};
    T.subs = subs;
    T.tile_sub = reinterpret_cast<const uint32_t*>(W + L.tile_sub);
    T.tile_pofs = reinterpret_cast<const uint64_t*>(W + L.tile_pofs);
    T.chunk_sub = reinterpret_cast<const uint32_t*>(W + L.chunk_sub);
    T.bk_sub = reinterpret_cast<const uint32_t*>(W + L.bk_sub);
    T.cnt = reinterpret_cast<uint32_t*>(W + L.cnt);
    T.mpre = reinterpret_cast<uint64_t*>(W + L.mpre);
    T.kpre = reinterpret_cast<uint64_t*>(W + L.kpre);
    T.chA = reinterpret_cast<uint64_t*>(W + L.chA);
    T.chB = reinterpret_cast<uint64_t*>(W + L.chB);
    T.N = reinterpret_cast<uint64_t*>(W + L.N);
    T.S = reinterpret_cast<uint64_t*>(W + L.S);
    T.M = reinterpret_cast<uint64_t*>(W + L.M);
    T.K = reinterpret_cast<uint64_t*>(W + L.K);
    T.MB = reinterpret_cast<uint64_t*>(W + L.MB);
    T.wsp = reinterpret_cast<uint64_t*>(W + L.wsp);
    T.total = total;
    T.err = err;
    T.ws_cap = total_elems;
    T.nsubs = count;
    T.ntiles = L.max_tiles;
    T.nchunks = L.max_chunks;
    T.nbuckets = L.max_buckets;
    T.max_chunks = (max_elems / (prm.tile - kmax) + 1 + kChunk - 1) / kChunk;
    T.dsz = dsz;
    HIP_TRY(launch_level_maps(subs, static_cast<uint32_t>(count), L.max_tiles, L.max_chunks, L.max_buckets,
                              const_cast<uint32_t*>(T.tile_sub), const_cast<uint64_t*>(T.tile_pofs),
                              const_cast<uint32_t*>(T.chunk_sub), const_cast<uint32_t*>(T.bk_sub), st, dsz));
    HIP_TRY(launch_rough(elem_bytes, T.subs, T.tile_sub, T.tile_pofs, T.cnt, L.max_tiles, prm, st, dsz));
    HIP_TRY(launch_tables_sizes(T, st));
    HIP_TRY(launch_tables_routes(T, st));
    HIP_TRY(launch_children(T, static_cast<uint32_t>(tile_limit), leaves, reinterpret_cast<LeafDesc*>(W + L.big),
                            counters, st));
    HIP_TRY(launch_gather(elem_bytes, W + L.ws, T, st));
    HIP_TRY(launch_scatter(elem_bytes, W + L.ws, T, st));
    uint32_t caps[3];
    leaf_class_caps(elem_bytes, prm, caps);
    LeafDesc* cls_lists = reinterpret_cast<LeafDesc*>(W + L.leaves_cls);
    HIP_TRY(launch_leaf_classes(leaves, L.max_leaves, cls_lists, L.max_leaves, caps, cls, st, counters));
    HIP_TRY(launch_leaf_persistent(elem_bytes, cls_lists, cls, L.max_leaves, prm, caps, qctr, st));
    HIP_TRY(launch_check_one_level(counters, err, st));
    return SHUF_OK;
}

static int check_array(const shuf_array_t& a, uint32_t w)
{
    if (a.n <= 1) return SHUF_OK;
    if (!a.ptr) return SHUF_EINVAL;
    if (reinterpret_cast<uintptr_t>(a.ptr) % w) return SHUF_EINVAL;
    if (a.n >= kMaxElements) return SHUF_EUNSUPPORTED;
    return SHUF_OK;
}

int shuffle_many(const shuf_array_t* arrays, uint64_t count, uint32_t elem_bytes, void* stream)
{
    if (!valid_width(elem_bytes) || (!arrays && count)) return SHUF_EINVAL;
    if (count >= (1ull << 32)) return SHUF_EUNSUPPORTED;
    for (uint64_t j = 0; j < count; ++j) {
        const int rc = check_array(arrays[j], elem_bytes);
        if (rc != SHUF_OK) return rc;
    }
    shuf_params_t p;
    shuf_default_params(0, elem_bytes, &p);
    Engine E = make_engine(elem_bytes, p);
    for (uint64_t j = 0; j < count; ++j)
        if (arrays[j].n >= 2)  // arrays of 0 or 1 element need no work
            engine_submit(E, reinterpret_cast<uintptr_t>(arrays[j].ptr) / elem_bytes, arrays[j].n,
                          arrays[j].seed, arrays[j].stream_id);
    if (!E.inflight) return SHUF_OK;
    return engine_drain(E, stream);
}

struct shuf_session {
    int device;
    Engine E;
    LeafLists lists;
    // admission: requests wait in `queue` until their charge (data bytes plus
    // the workspace the library computes for them alone) fits the budget
    struct Pending {
        shuf_array_t a;
        uint64_t ticket, charge;
        bool exact;  // charge is the planning run's figure (else the cheap upper bound)
    };
    uint64_t budget = 0;  // bytes; 0: no limit
    uint64_t used = 0;    // charges of admitted, unfinished requests
    uint64_t next_ticket = 1;
    uint64_t reported_free = 0;  // entries of E.done_queue whose charges are released
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, uint64_t> charge_of;  // admitted ticket -> charge
};

// The charge of a request: its data plus the device workspace it needs alone.
// `exact`: the planning run of shuffle_workspace_bytes (counts and tables on
// the device, no element moves); otherwise an upper bound that needs no GPU
// work: the movers of a level are at most its items (n * w), and the level
// tables and lists take less than 24 bytes per item plus 16 KiB.  (A level
// has at most e n buckets, e = 256 / (T - KMAX), since every subproblem of a
// tiled level holds more than T - KMAX items, and at most 2 e n (tile,
// bucket) and (chunk, bucket) entries; at about 236 bytes per bucket (its
// totals, map entry and child descriptor, and the next step's leaf lists),
// 20 per (tile, bucket) and 16 per (chunk, bucket) entry that is at most
// 310 e n bytes, 21 n at the smallest default tile of 4096 items; the 256-byte
// rounding of about 25 buffers stays below 16 KiB.)
static int session_charge(const shuf_session_t* s, const shuf_array_t& a, bool exact, uint64_t* out)
{
    const uint64_t w = s->E.w;
    if (a.n <= 1) {
        *out = a.n * w;
        return SHUF_OK;
    }
    if (!exact) {
        *out = 2 * a.n * w + 24 * a.n + (16u << 10);
        return SHUF_OK;
    }
    shuf_params_t p;
    shuf_default_params(a.n, static_cast<uint32_t>(w), &p);
    uint64_t ws = 0;
    const int rc = shuffle_workspace_bytes(a.n, static_cast<uint32_t>(w), a.seed, a.stream_id, &p, &ws, nullptr);
    if (rc != SHUF_OK) return rc;
    *out = a.n * w + ws;
    return SHUF_OK;
}

// Admit queued requests in order while their charges fit the budget; a
// request whose cheap bound does not fit is charged exactly before it waits.
static int session_admit(shuf_session_t* s)
{
    while (!s->queue.empty()) {
        shuf_session::Pending& p = s->queue.front();
        if (s->budget && s->used + p.charge > s->budget) {
            if (p.exact) break;
            const int rc = session_charge(s, p.a, true, &p.charge);
            if (rc != SHUF_OK) return rc;
            p.exact = true;
            continue;
        }
        engine_submit(s->E, reinterpret_cast<uintptr_t>(p.a.ptr) / s->E.w, p.a.n, p.a.seed, p.a.stream_id,
                      p.ticket);
        s->used += p.charge;
        s->charge_of[p.ticket] = p.charge;
        s->queue.pop_front();
    }
    return SHUF_OK;
}

int shuf_session_create(uint32_t elem_bytes, shuf_session_t** out)
{
    if (!out || !valid_width(elem_bytes)) return SHUF_EINVAL;
    int dev = 0;
    if (!current_context(&dev)) return SHUF_EHIP;
    shuf_params_t p;
    shuf_default_params(0, elem_bytes, &p);
    shuf_session_t* s = new (std::nothrow) shuf_session_t{dev, make_engine(elem_bytes, p), {}};
    if (!s) return SHUF_ENOMEM;
    s->E.lists = &s->lists;
    *out = s;
    return SHUF_OK;
}

int shuf_session_submit(shuf_session_t* s, const shuf_array_t* a, uint64_t* ticket)
{
    if (!s || !a || !ticket) return SHUF_EINVAL;
    if (s->E.broken) return SHUF_EHIP;
    const int rc = check_array(*a, s->E.w);
    if (rc != SHUF_OK) return rc;
    if (s->E.ticket.size() >= (1ull << 31) && s->E.free_slots.empty()) return SHUF_EUNSUPPORTED;
    uint64_t charge = 0;
    bool exact = false;
    if (s->budget) {
        int rc2 = session_charge(s, *a, false, &charge);
        if (rc2 == SHUF_OK && charge > s->budget) {
            exact = true;
            rc2 = session_charge(s, *a, true, &charge);
        }
        if (rc2 != SHUF_OK) return rc2;
        if (charge > s->budget) return SHUF_ENOMEM;  // could never be admitted
    }
    *ticket = s->next_ticket++;
    s->queue.push_back({*a, *ticket, charge, exact});
    return session_admit(s);
}

int shuf_session_step(shuf_session_t* s, void* stream, uint64_t* done, uint64_t cap,
                      uint64_t* ndone)
{
    if (!s || !ndone || (cap && !done)) return SHUF_EINVAL;
    int dev = 0;
    Context* C = current_context(&dev);
    if (!C) return SHUF_EHIP;
    if (dev != s->device) return SHUF_EINVAL;
    int rc0 = session_admit(s);
    if (rc0 != SHUF_OK) return rc0;
    if (s->E.inflight) {
        std::lock_guard<std::mutex> lock(C->mu);
        C->spans.clear();
        C->events_used = 0;
        s->E.host = &C->host;
        shuf_stats_t st{};
        const int rc = engine_step(*C, s->E, static_cast<hipStream_t>(stream), st);
        if (rc != SHUF_OK) {
            s->E.broken = true;
            return rc;
        }
        C->stats = st;
    }
    // completed requests free their charges, and waiting ones may enter
    for (uint64_t i = s->reported_free; i < s->E.done_queue.size(); ++i) {
        const auto it = s->charge_of.find(s->E.done_queue[i]);
        if (it != s->charge_of.end()) {
            s->used -= it->second;
            s->charge_of.erase(it);
        }
    }
    s->reported_free = s->E.done_queue.size();
    rc0 = session_admit(s);
    if (rc0 != SHUF_OK) return rc0;
    const uint64_t k = std::min<uint64_t>(cap, s->E.done_queue.size());
    for (uint64_t i = 0; i < k; ++i) done[i] = s->E.done_queue[i];
    s->E.done_queue.erase(s->E.done_queue.begin(), s->E.done_queue.begin() + k);
    s->reported_free -= k;
    *ndone = k;
    return SHUF_OK;
}

int shuf_session_set_budget(shuf_session_t* s, uint64_t bytes)
{
    if (!s) return SHUF_EINVAL;
    if (s->E.inflight || !s->queue.empty()) return SHUF_EINVAL;  // only while idle
    s->budget = bytes;
    return SHUF_OK;
}

int shuf_session_queued(const shuf_session_t* s, uint64_t* queued, uint64_t* used_bytes)
{
    if (!s || !queued) return SHUF_EINVAL;
    *queued = s->queue.size();
    if (used_bytes) *used_bytes = s->used;
    return SHUF_OK;
}

int shuf_session_inflight(const shuf_session_t* s, uint64_t* inflight, uint64_t* completed_unread)
{
    if (!s || !inflight) return SHUF_EINVAL;
    *inflight = s->E.inflight + s->queue.size();
    if (completed_unread) *completed_unread = s->E.done_queue.size();
    return SHUF_OK;
}

int shuf_session_destroy(shuf_session_t* s)
{
    if (!s) return SHUF_EINVAL;
    int dev = -1;
    const bool have = current_context(&dev) != nullptr;
    if (have && dev != s->device) (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    s->lists.release();
    if (have && dev != s->device) (void)hipSetDevice(dev);
    delete s;
    return SHUF_OK;
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
    Context* Cp = current_context();
    if (!Cp) return SHUF_EHIP;
    Context& C = *Cp;
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
    Context* Cp = current_context();
    if (!Cp) return SHUF_EHIP;
    Context& C = *Cp;
    std::lock_guard<std::mutex> lock(C.mu);
    for (int i = 0; i < SHUF_KERNEL_KINDS; ++i) out[i] = C.times[i];
    return SHUF_OK;
}

int shuffle_release(void)
{
    release_all();
    return SHUF_OK;
}

int shuffle_last_stats(shuf_stats_t* out)
{
    if (!out) return SHUF_EINVAL;
    Context* C = current_context();
    if (!C) return SHUF_EHIP;
    std::lock_guard<std::mutex> lock(C->mu);
    *out = C->stats;
    return SHUF_OK;
}

}  // extern "C"
