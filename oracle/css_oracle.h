/*
 * CPU oracle for the in-place ScatterShuffle definition, version 1.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference the GPU path
 * is checked against.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg may load it.  It shares no code with the HIP library and
 * the HIP library never calls it.
 *
 * Paper: M. Penschuck, "Engineering Shared-Memory Parallel Shuffling to
 * Generate Random Permutations In-Place" (arXiv 2302.03317).
 */
#ifndef CSS_ORACLE_H
#define CSS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Parameters that are part of the permutation's definition.
 *   tile      T: elements one tile may hold (>= 2^kmax_log2 + 1)
 *   kmax_log2 largest bucket-count exponent, 1..8 (labels live in one byte)
 *   n0        base-case size: subproblems of at most n0 elements go to FY
 *   lmax      recursion cap: a subproblem at level lmax goes to FY (<= 255) */
typedef struct {
    uint64_t tile;
    uint32_t kmax_log2;
    uint32_t n0;
    uint32_t lmax;
} css_params_t;

/* Randomness provider.  The default provider is Philox4x32-10 keyed by the
 * seed; tests substitute scripted providers to enumerate every outcome. */
typedef struct css_rng {
    uint32_t (*label)(struct css_rng* self, uint32_t level, uint64_t pos, uint32_t kappa);
    uint64_t (*draw)(struct css_rng* self, uint32_t level, uint64_t pos, uint64_t bound);
    uint64_t seed;
    uint32_t stream_id;
    void* ctx;
} css_rng_t;

/* error codes */
#define CSS_OK 0
#define CSS_EINVAL -1
#define CSS_ENOMEM -2
#define CSS_EUNSUPPORTED -4

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void css_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* kappa-bit bucket label of position `pos` at recursion level `level`. */
uint32_t css_label(uint64_t seed, uint32_t stream_id, uint32_t level, uint64_t pos, uint32_t kappa);

/* Uniform draw from [0, bound) for the Fisher-Yates step at `pos`
 * (1 <= bound <= 2^32), Lemire's multiply-and-reject with the attempt
 * number in the counter: 16-bit words for bounds up to 2^16, else 32-bit. */
uint64_t css_draw(uint64_t seed, uint32_t stream_id, uint32_t level, uint64_t pos, uint64_t bound);

/* One Lemire step on a given 32-bit word: returns 1 and sets *out when the
 * word is accepted for `bound`, else returns 0. */
int css_lemire_step(uint32_t word, uint64_t bound, uint64_t* out);

/* Exhaustive check helper: for every 32-bit word, run one Lemire step with
 * `bound` (<= 2^20) and add accepted results into counts[0..bound). */
void css_lemire_histogram(uint64_t bound, uint64_t* counts);

/* Exhaustive check helper for the 16-bit rule (bound <= 2^16). */
void css_lemire16_histogram(uint32_t bound, uint64_t* counts);

/* Bucket-count exponent chosen for a subproblem of m elements. */
uint32_t css_kappa(uint64_t m, int hbm_regime, const css_params_t* p);

/* Validate parameters; returns CSS_OK or CSS_EINVAL. */
int css_check_params(const css_params_t* p);

/* One IpSc level on a subproblem of m elements whose labels are given.
 * hbm_regime != 0 selects the tiled rough placement with routing fix-up,
 * else the exact stable counting sort.  dest[i] receives the position
 * (relative to the subproblem start) where the item at relative position i
 * goes.  Returns CSS_OK or an error. */
int css_level(const uint8_t* labels, uint64_t m, uint32_t kappa, uint64_t tile,
              int hbm_regime, uint64_t* dest);

/* Fisher-Yates permutation of m items as a destination map using the given
 * rng at `level` and absolute start position `base`: dest[i] = final
 * relative position of the item initially at relative position i. */
int css_fy_dest(css_rng_t* rng, uint32_t level, uint64_t base, uint64_t m, uint64_t* dest);

/* Whole shuffle, in place on `data` (n elements of `w` bytes each), with the
 * Philox provider. */
int css_shuffle(void* data, uint64_t n, uint32_t w, uint64_t seed, uint32_t stream_id,
                const css_params_t* p);

/* The same shuffle with the independent buckets of the top level solved on
 * `threads` host threads (and its labels computed on them); the result is
 * identical for every thread count. */
int css_shuffle_mt(void* data, uint64_t n, uint32_t w, uint64_t seed, uint32_t stream_id,
                   const css_params_t* p, uint32_t threads);

/* Whole shuffle with an arbitrary provider. */
int css_shuffle_rng(void* data, uint64_t n, uint32_t w, css_rng_t* rng, const css_params_t* p);

/* Plain sequential Fisher-Yates over the whole array with the same draws as
 * the oracle's base case at level 0 (the same-RNG sequential baseline). */
int css_fisher_yates(void* data, uint64_t n, uint32_t w, uint64_t seed, uint32_t stream_id);

/* Exhaustive enumeration of every random outcome for m <= 8 items under the
 * given parameters.  prob[r] receives the probability of the permutation
 * whose lexicographic rank is r (m! entries).  *paths receives the number of
 * decision paths visited.  Returns CSS_OK or an error. */
int css_enumerate(uint32_t m, const css_params_t* p, double* prob, uint64_t* paths);

/* Statistics helpers: permutation histogram over consecutive seeds (m <= 8)
 * and item-by-position histogram (n x n counts). */
int css_perm_histogram(uint32_t m, uint64_t seed0, uint64_t nseeds, const css_params_t* p,
                       uint64_t* counts);
int css_position_histogram(uint32_t n, uint64_t seed0, uint64_t nseeds, const css_params_t* p,
                           uint64_t* counts);

#ifdef __cplusplus
}
#endif

#endif
