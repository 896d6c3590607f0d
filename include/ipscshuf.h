/*
 * ipscshuf: in-place parallel ScatterShuffle on one MI355X (gfx950).
 *
 * Generates a uniformly random permutation of a device array in place, as
 * defined by M. Penschuck, "Engineering Shared-Memory Parallel Shuffling to
 * Generate Random Permutations In-Place" (arXiv 2302.03317):
 *   - ScatterShuffle (Sec. 2.2, Sec. 3.1): every element gets a uniform random
 *     bucket, buckets become contiguous regions, every region is shuffled
 *     recursively, and Fisher-Yates (Fig. 1) finishes small regions;
 *   - one recursion level is RoughScatter (Sec. 3.3) with each tile owning a
 *     piece of every bucket (Sec. 4.1), followed by the fix-up that
 *     FineScatter performs (Sec. 3.4);
 *   - the permutation is reproducible from the seed and independent of
 *     scheduling (Sec. 5): every random draw is a Philox4x32-10 output keyed by
 *     (seed, stream id, recursion level, position).
 *
 * The exact permutation is fixed by definition version 1 (see
 * shuffle_definition_version) and the parameters shuf_params_t: two calls
 * with the same (n, elem_bytes, seed, stream_id, params) apply the same
 * permutation to any input contents.
 *
 * Conventions for every entry point:
 *   - return 0 on success, a negative SHUF_E* code on failure;
 *   - `ptr` is device memory owned by the caller (e.g. a torch tensor's
 *     data_ptr()); the library never frees it;
 *   - `stream` is a hipStream_t (NULL = the null stream).  The work runs on
 *     that stream; the call returns after it has completed (the library
 *     synchronises the stream to plan each recursion level), except
 *     shuffle_batched_async, which only enqueues its work;
 *   - device memory is addressed absolutely: every array, wherever it lives,
 *     is reached through its own pointer;
 *   - argument errors are detected before any GPU work starts, and then the
 *     data is untouched; after SHUF_EHIP the contents are unspecified;
 *   - calls may come from several host threads; calls on one device are
 *     serialised by the library.
 */
#ifndef IPSCSHUF_H
#define IPSCSHUF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHUF_OK 0
#define SHUF_EINVAL -1       /* invalid argument */
#define SHUF_ENOMEM -2       /* device or pinned host memory could not be obtained */
#define SHUF_EHIP -3         /* a HIP call or kernel launch failed */
#define SHUF_EUNSUPPORTED -4 /* valid, but beyond what this implementation handles */

/* Parameters that are part of the permutation's definition.
 *   tile       T: elements one tile holds; tile * elem_bytes <= 65536 and
 *              tile >= 2^kmax_log2 + 1
 *   kmax_log2  largest bucket-count exponent (k <= 2^kmax_log2), 1..8
 *   n0         base-case size: subproblems of at most n0 elements are
 *              finished by Fisher-Yates; >= 1
 *   lmax       recursion cap: a subproblem at level lmax is finished by
 *              Fisher-Yates; <= 255 */
typedef struct {
    uint32_t tile;
    uint32_t kmax_log2;
    uint32_t n0;
    uint32_t lmax;
} shuf_params_t;

/* Version of the permutation definition implemented; changes whenever the
 * output for given (inputs, n, elem_bytes, seed, stream_id, params) changes.
 * Version 1 is one fixed rendition of IpScShuf (Sec. 3.2, Fig. 2): per level
 * RoughScatter into equal regions with one piece of every region per tile
 * (Sec. 3.3, Sec. 4.1), the exact label counts as final bucket sizes and a
 * deterministic routing of the remaining items (the role of FineScatter,
 * Sec. 3.4), recursion on every bucket (Sec. 3.5) and Fisher-Yates below the
 * base-case size (Fig. 1). */
uint32_t shuffle_definition_version(void);

/* How the kernels compute the stable ranks of the counting sorts on the
 * current device.  A rank is the number of earlier items of a tile with the
 * same label, i.e. the order in which RoughScatter (Sec. 3.3) would place
 * them; it is not part of the definition: both ways give the same ranks,
 * hence the same permutation:
 *   1  one LDS atomic add per item.  Chosen where the device serves the LDS
 *      atomic adds of one wave instruction that hit the same address in lane
 *      order, which a probe kernel checks at the device's first call;
 *   0  one ballot per label bit (the probe failed, or the environment has
 *      IPSCSHUF_RANK=ballot when the device's first call runs);
 *  -1  no call has run on the current device yet. */
int shuffle_rank_method(void);

/* Default parameters for n elements of elem_bytes each (4, 8 or 16):
 * tile = 65536 / elem_bytes, kmax_log2 = 8, n0 = 64, lmax = 32.  The paper
 * keeps k at most 256 (Sec. 3.1) and tunes k and the base-case size by hand
 * (Sec. 5); here k per level follows from n and these parameters.
 *   n     unused (the defaults do not depend on it)
 *   out   receives the parameters; caller-owned
 * Returns SHUF_EINVAL for a null `out` or an unsupported width. */
int shuf_default_params(uint64_t n, uint32_t elem_bytes, shuf_params_t* out);

/* Shuffle n elements of elem_bytes (4, 8 or 16) bytes at device pointer ptr
 * in place, with stream id 0 and the default parameters: a uniformly random
 * permutation (Sec. 2.2) by the in-place ScatterShuffle (IpScShuf, Sec. 3.2,
 * Fig. 2), parallelised per level over tiles (Sec. 4.1).
 *   ptr         device pointer, aligned to elem_bytes; may be NULL if n <= 1
 *   n           element count, n < 2^40
 *   elem_bytes  4, 8 or 16; elements are moved as opaque words of that size
 *   seed        64-bit seed
 * Errors: SHUF_EINVAL (NULL ptr with n > 1, bad width, misaligned ptr),
 * SHUF_EUNSUPPORTED (n too large), SHUF_ENOMEM, SHUF_EHIP. */
int shuffle_inplace(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream);

/* As shuffle_inplace with an explicit stream id (the fourth Philox counter
 * word; distinct ids give independent permutations for one seed) and explicit
 * parameters.  Every random draw is a pure function of (seed, stream id,
 * level, position), the GPU form of Sec. 5's reproducible subtask
 * generators; the pool supplies the workspace (see shuffle_inplace_ws for a
 * caller-supplied one).  `params` must not be NULL.  Additional errors: SHUF_EINVAL for
 * parameters outside the ranges above, SHUF_EUNSUPPORTED when the parameters
 * need more LDS than one workgroup has. */
int shuffle_inplace_ex(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                       uint32_t stream_id, const shuf_params_t* params, void* stream);

/* Exact device workspace, in bytes, that shuffle_inplace_ws needs for these
 * arguments.  The workspace holds the items a level routes after its rough
 * pass (the remainder FineScatter handles, Sec. 3.4; about 5 % of a level)
 * and the level's tables; the paper's sequential version needs only O(k)
 * words per level instead (Sec. 3.5).  The size is exact (the permutation's recursion depends on the seed and stream id,
 * not on the data).  It runs the planning part of the shuffle on the device
 * (labels counted per tile, the level tables) without touching any element,
 * using the library's own memory; it takes some of the time of a shuffle.
 * *out_bytes = 0 for n <= 1.  Errors: SHUF_EINVAL (NULL out_bytes, bad width
 * or parameters), SHUF_EUNSUPPORTED, SHUF_ENOMEM, SHUF_EHIP. */
int shuffle_workspace_bytes(uint64_t n, uint32_t elem_bytes, uint64_t seed, uint32_t stream_id,
                            const shuf_params_t* params, uint64_t* out_bytes, void* stream);

/* As shuffle_inplace_ex (same passages), with every per-level device buffer
 * (the movers of a level and all level tables) carved from the caller's
 * `workspace` of
 * `workspace_bytes` bytes, 256-byte aligned, owned by the caller and not
 * touched after the call returns.  The library still keeps its leaf lists
 * (48 bytes per finished subproblem) and pinned staging in its own pools.
 * `workspace_bytes` must be at least what shuffle_workspace_bytes reports for
 * the same (n, elem_bytes, seed, stream_id, params); a smaller workspace fails
 * with SHUF_ENOMEM, possibly after the data has been partly permuted.
 * Additional errors: SHUF_EINVAL for a misaligned workspace, or NULL with
 * workspace_bytes > 0. */
int shuffle_inplace_ws(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                       uint32_t stream_id, const shuf_params_t* params, void* workspace,
                       uint64_t workspace_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): shuffle_inplace_ex
 * with every device buffer -- level tables, the movers' workspace, leaf lists,
 * counters -- taken from a static device array of the library (64 MiB per
 * device, part of its code object, held until the process ends) and host
 * staging from a static host array.  The call makes no hipMalloc, hipFree,
 * hipHostMalloc or hipEventCreate (timing is off for it); its host-side
 * bookkeeping uses the C++ heap.  It first runs the planning part of the
 * shuffle in that memory, so a shortage is reported before any element moves.
 * The output equals shuffle_inplace_ex with the same arguments.
 *   ptr, n, elem_bytes, seed, stream_id, params, stream: as shuffle_inplace_ex
 * Limits: n * elem_bytes <= 48 MiB, else SHUF_EUNSUPPORTED before any GPU
 * work; SHUF_ENOMEM (data untouched) when the parameters need more than the
 * static memory holds.  Calls on one device share its static array; the
 * library serialises them, so calls that reach the device concurrently from
 * outside the library (e.g. a second copy of the library) would race.
 * Errors otherwise as shuffle_inplace_ex. */
int shuffle_inplace_noalloc(void* ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                            uint32_t stream_id, const shuf_params_t* params, void* stream);

/* Shuffle `count` independent arrays packed back to back at ptr, each in
 * place: many independent shuffles run concurrently, the setting of
 * Sec. 6.3, here in shared launches instead of one task per array.  Array j occupies elements [offsets[j], offsets[j+1]) and is shuffled
 * exactly as shuffle_inplace_ex(ptr + offsets[j] * elem_bytes,
 * offsets[j+1] - offsets[j], elem_bytes, seed, j, default params).  All arrays
 * are processed together, level by level, in shared launches.
 *   offsets     HOST array of count + 1 non-decreasing element offsets
 *   count       number of arrays, < 2^32
 * Errors: SHUF_EINVAL (NULL ptr or offsets, decreasing offsets, bad width or
 * alignment), SHUF_EUNSUPPORTED, SHUF_ENOMEM, SHUF_EHIP. */
int shuffle_batched(void* ptr, const uint64_t* offsets, uint64_t count, uint32_t elem_bytes,
                    uint64_t seed, void* stream);

/* shuffle_batched with explicit parameters for every array of the batch (an
 * autotuned Π of the batched workload; Sec. 5 tunes k and the base-case size
 * per workload by hand): array j is shuffled exactly as
 * shuffle_inplace_ex(..., j, params).  params NULL means the defaults.
 * Errors as shuffle_batched, plus SHUF_EINVAL / SHUF_EUNSUPPORTED for
 * parameters that shuffle_inplace_ex refuses. */
int shuffle_batched_ex(void* ptr, const uint64_t* offsets, uint64_t count, uint32_t elem_bytes,
                       uint64_t seed, const shuf_params_t* params, void* stream);

/* Enqueue-only form of shuffle_batched (many independent shuffles run
 * together, Sec. 6.3): the call only launches kernels on `stream` -- no
 * host synchronisation, no allocation, no memset -- so a caller may capture it
 * into a HIP graph and replay it.  The first level is planned on the device
 * from the offsets in DEVICE memory; tile kernels, level tables and the fix-up
 * run with grids sized from upper bounds (surplus workgroups leave at once);
 * the leaves run in persistent workgroups that take work from per-size-class
 * counters.  Array j is shuffled exactly as shuffle_inplace_ex(ptr +
 * offsets[j] * elem_bytes, offsets[j+1] - offsets[j], elem_bytes, seed, j,
 * params), the same as shuffle_batched_ex.
 *   offsets      DEVICE array of count + 1 non-decreasing element offsets,
 *                8-byte aligned, read when the kernels run
 *   count        1 .. 2^22 arrays
 *   params       parameters of every array (NULL: the defaults); the same
 *                pointer or equal values go to the two size queries below
 *   total_elems  an upper bound of offsets[count] (sizes the workspace)
 *   workspace    device memory of at least shuffle_batched_async_workspace_bytes
 *                (count, total_elems, elem_bytes, params) bytes, 256-byte
 *                aligned, owned by the caller and in use until the stream
 *                reaches the end of the call's work
 * Limit: every array holds at most shuffle_batched_async_max_elems(elem_bytes,
 * params) elements ((tile / 2) * 2^kmax_log2: one tiled level then leaves
 * subproblems that fit a tile; 2^21 for 4-byte elements with the defaults;
 * 0 for invalid parameters).  Errors detected on the host (before any
 * launch): SHUF_EINVAL (NULL or misaligned pointers, bad width or
 * parameters), SHUF_EUNSUPPORTED (count or total_elems out of range, or
 * parameters beyond the LDS), SHUF_ENOMEM (workspace too small), SHUF_EHIP.  Errors detected on the device are reported in the first 4 bytes
 * of the workspace, to be read after the stream has completed: 0 success;
 * 32 decreasing offsets, an array above the limit or sizes beyond total_elems
 * (nothing was moved); 16 a subproblem needed a second tiled level (never
 * seen in practice at these sizes; the data are then unspecified); 1 or 2 an
 * index check of the fix-up failed.  The device's first call of the library
 * runs a short probe that synchronises the stream: make it outside a capture. */
int shuffle_batched_async(void* ptr, const uint64_t* offsets, uint64_t count, uint32_t elem_bytes,
                          uint64_t seed, const shuf_params_t* params, uint64_t total_elems, void* workspace,
                          uint64_t workspace_bytes, void* stream);
int shuffle_batched_async_workspace_bytes(uint64_t count, uint64_t total_elems, uint32_t elem_bytes,
                                          const shuf_params_t* params, uint64_t* out_bytes);
uint64_t shuffle_batched_async_max_elems(uint32_t elem_bytes, const shuf_params_t* params);

/* One array of a multi-array call or a serving request: n elements at device
 * pointer ptr (aligned to elem_bytes; may be NULL if n <= 1), shuffled with
 * its own seed and stream id. */
typedef struct {
    void* ptr;
    uint64_t n;
    uint64_t seed;
    uint32_t stream_id;
    uint32_t reserved;
} shuf_array_t;

/* Shuffle `count` independent arrays, each in place and anywhere in device
 * memory (independent shuffles run together, as in Sec. 6.3): array j is shuffled exactly as shuffle_inplace_ex(arrays[j].ptr,
 * arrays[j].n, elem_bytes, arrays[j].seed, arrays[j].stream_id, default
 * params).  All arrays are processed together, level by level, in shared
 * launches.  Arrays must not overlap.  `arrays` is a HOST array.
 * Errors: SHUF_EINVAL (NULL arrays with count > 0, bad width, NULL or
 * misaligned ptr with n > 1), SHUF_EUNSUPPORTED, SHUF_ENOMEM, SHUF_EHIP. */
int shuffle_many(const shuf_array_t* arrays, uint64_t count, uint32_t elem_bytes, void* stream);

/* Continuous batching (a serving loop; no passage of the paper describes
 * one: each request is the single-array shuffle above, Sec. 3.2 and 4.1).
 * A session accepts shuffle requests at any time and
 * advances all of them together, one step per call: a step gives every
 * in-flight request's pending subproblems one recursion level in shared
 * launches and finishes every pending subproblem that fits a tile.  Requests
 * submitted between steps join at the next step.  Each request's result is
 * exactly shuffle_inplace_ex(ptr, n, elem_bytes, seed, stream_id, default
 * params), whatever else is in flight (the permutation is a function of the
 * request alone).
 *   shuf_session_create   session for elements of elem_bytes on the current
 *                         device (later calls must run with that device
 *                         current); *out receives the handle
 *   shuf_session_submit   queue a request; the caller keeps ptr valid and does
 *                         not touch its data until the ticket is reported done;
 *                         *ticket receives a positive id
 *   shuf_session_step     run one step on `stream` (blocking, as the other
 *                         calls) if anything is in flight, then report up to
 *                         `cap` completed tickets in done[0..*ndone); further
 *                         completions are reported by later calls
 *   shuf_session_inflight requests submitted and not yet complete (queued
 *                         ones included), and
 *                         completed tickets not yet reported (may be NULL)
 *   shuf_session_destroy  waits for the session's device and frees the session
 *                         and its device memory (requests still in flight are
 *                         abandoned, their data unspecified)
 * A session is used by one host thread at a time; steps of sessions and other
 * calls on one device are serialised by the library.  After a step fails with
 * SHUF_EHIP the session only returns SHUF_EHIP.  Errors otherwise as above. */
typedef struct shuf_session shuf_session_t;
int shuf_session_create(uint32_t elem_bytes, shuf_session_t** out);
int shuf_session_submit(shuf_session_t* s, const shuf_array_t* a, uint64_t* ticket);
int shuf_session_step(shuf_session_t* s, void* stream, uint64_t* done, uint64_t cap,
                      uint64_t* ndone);
int shuf_session_inflight(const shuf_session_t* s, uint64_t* inflight, uint64_t* completed_unread);
/* Admission by memory budget (a serving loop's HBM budget; no passage of the
 * paper).  With a budget of `bytes` (> 0), every submitted request waits in a
 * queue in submission order and joins the next step only while the charges
 * of the admitted, unfinished requests fit the budget.  A request is charged
 * its data bytes plus a workspace bound that needs no GPU work (2 n w + 24 n
 * + 16 KiB in all); when that does not fit, the exact figure replaces it:
 * its data plus the workspace the library computes for it alone (the
 * planning run of shuffle_workspace_bytes, on the null stream).  A request
 * whose exact charge alone exceeds the budget is refused with SHUF_ENOMEM.
 * Completed requests release their charges.  Set while the session is idle
 * (SHUF_EINVAL otherwise); 0 removes the limit.
 *   shuf_session_queued  requests waiting for admission, and the charges of
 *                        the admitted ones (may be NULL) */
int shuf_session_set_budget(shuf_session_t* s, uint64_t bytes);
int shuf_session_queued(const shuf_session_t* s, uint64_t* queued, uint64_t* used_bytes);
int shuf_session_destroy(shuf_session_t* s);

/* Free the device pools, pinned host staging and timing events the library
 * keeps between calls, on every device it has used (no passage; resource
 * management).  Waits for each such device first.  Later calls allocate them
 * again.  It also runs by itself at process exit, before the HIP runtime is
 * torn down.  Sessions keep their own memory until shuf_session_destroy.
 * Must not overlap other calls of the library.  Returns SHUF_OK. */
int shuffle_release(void);

/* Human-readable text of an error code (static storage; no passage). */
const char* shuffle_strerror(int code);

/* Statistics of the most recent successful call on the calling thread's
 * current device (instrumentation; the mover count is the remainder that
 * Sec. 3.3 bounds and Sec. 3.4 assigns): levels run through the tiled pass, tiles launched, mover
 * elements routed through the workspace, subproblems finished in LDS, and
 * peak workspace bytes.  For tests and benchmarks; returns SHUF_EINVAL for a
 * NULL pointer. */
typedef struct {
    uint32_t tiled_levels;
    uint32_t reserved;
    uint64_t tiles;
    uint64_t movers;
    uint64_t leaves;
    uint64_t fy_fallback;
    uint64_t workspace_bytes;
} shuf_stats_t;
int shuffle_last_stats(shuf_stats_t* out);

/* Per-kernel timing (instrumentation, no passage) with HIP events recorded
 * on the caller's stream around every launch group (instrumentation for benchmarks; it adds one event pair
 * per launch).  Kinds, in this order: 0 rough pass, 1 level tables,
 * 2 fix-up gather, 3 fix-up scatter, 4 LDS leaves, 5 sequential fallback.
 * `bytes` is the algorithmic HBM traffic of the launches: every element the
 * kernel moves is counted once read and once written.
 * shuffle_timing_enable(1) clears the accumulators of the current device and
 * starts timing, (0) stops; shuffle_timing_read fills out[0..5].  Both return
 * SHUF_EINVAL for a NULL `out`. */
typedef struct {
    double ms;
    uint64_t launches;
    double bytes;
} shuf_kernel_time_t;
#define SHUF_KERNEL_KINDS 6
int shuffle_timing_enable(int on);
int shuffle_timing_read(shuf_kernel_time_t* out);

#ifdef __cplusplus
}
#endif

#endif
