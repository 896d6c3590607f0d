/*
 * CPU oracle for the in-place ScatterShuffle definition, version 1.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, plain reference that the GPU library is
 * compared against element by element.  Nothing in the product path loads or
 * calls this file; it shares no code with the HIP sources.
 *
 * What it computes, following arXiv 2302.03317 (Penschuck):
 *   - ScatterShuffle (Sec. 2.2 and 3.1): every item of a subproblem gets an
 *     independent uniform bucket label in [0, k); the subproblem is rearranged
 *     so that bucket b occupies one contiguous region; each region is shuffled
 *     recursively; small subproblems finish with Fisher-Yates (Fig. 1, Sec. 2.2).
 *   - IpSc = RoughScatter + FineScatter (Sec. 3.2-3.4): the subproblem is cut
 *     into k equal regions, each bucket region holds a "placed" front and a
 *     "staged" rest; most items are placed directly, the few remaining ones are
 *     assigned afterwards.
 *   - ParRoughScatter (Sec. 4.1): every parallel worker owns one piece of every
 *     bucket; here a "tile" owns piece t of each of the k equal regions.
 *   - FineScatter's role (Sec. 3.4): final bucket sizes are the exact label
 *     counts, bucket boundaries move from the equal split to the exact split,
 *     and the items not yet in their final region are routed into the free
 *     positions of it.
 *   - Sampling (Sec. 2.3): k = 2^kappa so a label is a shift of random bits;
 *     bounded integers for Fisher-Yates use Lemire's multiply-and-reject.
 *   - Reproducibility (Sec. 5 "Implementation"): randomness is a pure function
 *     of (seed, stream, level, position) via the Philox4x32-10 counter-based
 *     generator, so the result does not depend on scheduling.
 *
 * The oracle is deliberately out of place: each level computes a destination
 * for every item and then copies.  It follows the definition's steps in
 * order with no blocking or fusion.
 */
#include "css_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Ten rounds; each round multiplies counter words
 * 0 and 2 by the two Philox multipliers, mixes the high halves with the other
 * counter words and the key; the key is bumped by the two Weyl constants
 * between rounds. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void css_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter word 2 ("tag"): level | purpose << 8 | attempt << 16. */
#define PURPOSE_LABEL 1u
#define PURPOSE_FY 2u

static void philox_for(uint64_t seed, uint32_t stream_id, uint64_t block, uint32_t tag,
                       uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)block, (uint32_t)(block >> 32), tag, stream_id};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    css_philox4x32_10(ctr, key, out);
}

/* Label: one Philox block serves 16 consecutive positions, one byte each;
 * the label is the top kappa bits of the position's byte.  Because 2^kappa
 * divides 256 the label is exactly uniform on [0, 2^kappa). */
uint32_t css_label(uint64_t seed, uint32_t stream_id, uint32_t level, uint64_t pos, uint32_t kappa)
{
    uint32_t x[4];
    philox_for(seed, stream_id, pos >> 4, level | (PURPOSE_LABEL << 8), x);
    uint32_t j = (uint32_t)(pos & 15);
    uint32_t byte = (x[j >> 2] >> (8 * (j & 3))) & 0xFFu;
    return byte >> (8 - kappa);
}

/* Lemire (2019), "Fast random integer generation in an interval": the word
 * x in [0, 2^32) times the bound s gives a 64-bit product; its high half is
 * the result and it is accepted iff its low half is at least 2^32 mod s,
 * which leaves exactly floor(2^32 / s) accepted words per result. */
static int lemire_accept(uint32_t word, uint64_t bound, uint64_t threshold, uint64_t* out)
{
    uint64_t prod = (uint64_t)word * bound;
    if ((prod & 0xFFFFFFFFu) >= threshold) {
        *out = prod >> 32;
        return 1;
    }
    return 0;
}

static uint64_t lemire_threshold(uint64_t bound)
{
    return (UINT64_C(1) << 32) % bound; /* 2^32 mod bound */
}

int css_lemire_step(uint32_t word, uint64_t bound, uint64_t* out)
{
    return lemire_accept(word, bound, lemire_threshold(bound), out);
}

void css_lemire_histogram(uint64_t bound, uint64_t* counts)
{
    uint64_t r, threshold = lemire_threshold(bound);
    for (uint64_t x = 0; x <= 0xFFFFFFFFu; ++x)
        if (lemire_accept((uint32_t)x, bound, threshold, &r))
            counts[r]++;
}

/* Bounds up to 2^16 ("short" draws): one Philox block serves eight
 * consecutive positions, 16 bits each (the low half of a word before the
 * high half), tag purpose 3; Lemire's rule on 16-bit words: x in [0, 2^16),
 * x*s accepted iff its low 16 bits are at least 2^16 mod s, draw = x*s >> 16.
 * Larger bounds ("long" draws): one block serves four positions, 32 bits
 * each, tag purpose 2, Lemire's rule on 32-bit words.  A rejected word is
 * replaced by the same word of the block with the next attempt number. */
#define PURPOSE_FY_SHORT 3u

uint64_t css_draw(uint64_t seed, uint32_t stream_id, uint32_t level, uint64_t pos, uint64_t bound)
{
    if (bound <= 0x10000u) {
        const uint32_t threshold = (uint32_t)(0x10000u % bound);
        for (uint32_t attempt = 0;; ++attempt) {
            uint32_t x[4];
            philox_for(seed, stream_id, pos >> 3,
                       level | (PURPOSE_FY_SHORT << 8) | ((attempt & 0xFFFFu) << 16), x);
            uint32_t h = (uint32_t)(pos & 7);
            uint32_t word16 = (x[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
            uint32_t prod = word16 * (uint32_t)bound;
            if ((prod & 0xFFFFu) >= threshold)
                return prod >> 16;
        }
    }
    for (uint32_t attempt = 0;; ++attempt) {
        uint32_t x[4];
        philox_for(seed, stream_id, pos >> 2,
                   level | (PURPOSE_FY << 8) | ((attempt & 0xFFFFu) << 16), x);
        uint64_t r;
        if (lemire_accept(x[pos & 3], bound, lemire_threshold(bound), &r))
            return r;
    }
}

/* Exhaustive check helper for the 16-bit rule: counts[r] += number of 16-bit
 * words accepted with result r, for bound <= 2^16. */
void css_lemire16_histogram(uint32_t bound, uint64_t* counts)
{
    const uint32_t threshold = 0x10000u % bound;
    for (uint32_t x = 0; x <= 0xFFFFu; ++x) {
        uint32_t prod = x * bound;
        if ((prod & 0xFFFFu) >= threshold) counts[prod >> 16]++;
    }
}

static uint32_t philox_label_cb(css_rng_t* self, uint32_t level, uint64_t pos, uint32_t kappa)
{
    return css_label(self->seed, self->stream_id, level, pos, kappa);
}

static uint64_t philox_draw_cb(css_rng_t* self, uint32_t level, uint64_t pos, uint64_t bound)
{
    return css_draw(self->seed, self->stream_id, level, pos, bound);
}

/* ------------------------------------------------------------------------ */
/* Parameters and the bucket-count schedule.
 *
 * The paper tunes k (64 or 256) and the base-case size by hand (Sec. 5
 * "Implementation").  Here k = 2^kappa is chosen per subproblem: with target
 * child size G (half a tile while the subproblem needs the tiled pass, half
 * the base-case size once it fits one tile), r is the number of label bits
 * needed to get from m down to G, h the number of levels that takes with at
 * most kmax_log2 bits each, and kappa spreads r evenly over those h levels. */
int css_check_params(const css_params_t* p)
{
    if (!p) return CSS_EINVAL;
    if (p->kmax_log2 < 1 || p->kmax_log2 > 8) return CSS_EINVAL;
    if (p->tile < (UINT64_C(1) << p->kmax_log2) + 1) return CSS_EINVAL;
    if (p->n0 < 1) return CSS_EINVAL;
    if (p->lmax > 255) return CSS_EINVAL;
    return CSS_OK;
}

uint32_t css_kappa(uint64_t m, int hbm_regime, const css_params_t* p)
{
    uint64_t g;
    if (hbm_regime) {
        g = p->tile / 2;
    } else {
        g = p->n0 / 2;
    }
    if (g < 1) g = 1;
    uint32_t r = 1;
    uint64_t reach = 2 * g; /* g * 2^r */
    while (reach < m) {
        reach *= 2;
        r++;
    }
    uint32_t h = (r + p->kmax_log2 - 1) / p->kmax_log2;
    uint32_t kappa = (r + h - 1) / h;
    if (kappa > p->kmax_log2) kappa = p->kmax_log2;
    return kappa;
}

/* ------------------------------------------------------------------------ */
/* One IpSc level. */

/* Start of the t-th of P pieces of a region of `len` items: floor(t*len/P). */
static uint64_t piece_start(uint64_t t, uint64_t len, uint64_t P)
{
    return (uint64_t)(((unsigned __int128)t * len) / P);
}

/* Where one level sends its items: the item at relative position x goes to
 * relative position y.  css_level records a destination map; the recursion
 * copies the element straight into the level's output buffer. */
typedef struct {
    void (*put)(void* ctx, uint64_t x, uint64_t y);
    void* ctx;
} sink_t;

static int exact_level(const uint8_t* labels, uint64_t m, uint64_t k, const uint64_t* S,
                       sink_t out)
{
    /* Every bucket occupies exactly its final region; items keep their
     * relative order inside a bucket (a stable counting sort by label). */
    uint64_t* cnt = calloc(k, sizeof(uint64_t));
    if (!cnt) return CSS_ENOMEM;
    for (uint64_t i = 0; i < m; ++i) {
        uint32_t l = labels[i];
        out.put(out.ctx, i, S[l] + cnt[l]++);
    }
    free(cnt);
    return CSS_OK;
}

/* A growable list of positions (the movers of one bucket). */
typedef struct {
    uint64_t* v;
    uint64_t n, cap;
} poslist_t;

static int poslist_push(poslist_t* a, uint64_t x)
{
    if (a->n == a->cap) {
        uint64_t ncap = a->cap ? 2 * a->cap : 64;
        uint64_t* nv = realloc(a->v, ncap * sizeof(uint64_t));
        if (!nv) return CSS_ENOMEM;
        a->v = nv;
        a->cap = ncap;
    }
    a->v[a->n++] = x;
    return CSS_OK;
}

static int rough_level(const uint8_t* labels, uint64_t m, uint64_t k, uint64_t tile,
                       const uint64_t* N, const uint64_t* S, sink_t out)
{
    /* RoughScatter over P tiles.  The subproblem is cut into k equal regions
     * E_b = [e_b, e_{b+1}), e_b = floor(b*m/k) (Sec. 3.3: k buckets of equal
     * size up to rounding).  Region E_b is cut into P pieces; tile t owns
     * piece t of every region (Sec. 4.1: each subtask gets a piece of every
     * bucket).  P is the smallest tile count with at most T items per tile. */
    uint64_t P = (m + (tile - k) - 1) / (tile - k);
    uint64_t* e = malloc((k + 1) * sizeof(uint64_t));
    uint64_t* cnt = malloc(k * sizeof(uint64_t));
    uint64_t* lo_t = malloc(k * sizeof(uint64_t));   /* piece start, this tile */
    uint64_t* cap_t = malloc(k * sizeof(uint64_t));  /* piece length, this tile */
    uint8_t* keeper = calloc(m ? m : 1, 1);          /* by destination position */
    poslist_t* movers = calloc(k, sizeof(poslist_t)); /* per bucket, in order */
    int rc = CSS_OK;
    if (!e || !cnt || !lo_t || !cap_t || !keeper || !movers) {
        rc = CSS_ENOMEM;
        goto out;
    }
    for (uint64_t b = 0; b <= k; ++b)
        e[b] = (uint64_t)(((unsigned __int128)b * m) / k);

    for (uint64_t t = 0; t < P; ++t) {
        for (uint64_t b = 0; b < k; ++b) {
            uint64_t len = e[b + 1] - e[b];
            lo_t[b] = e[b] + piece_start(t, len, P);
            cap_t[b] = e[b] + piece_start(t + 1, len, P) - lo_t[b];
            cnt[b] = 0;
        }
        /* Read order: piece of bucket 0, then bucket 1, ...; ascending
         * positions inside a piece. */
        for (uint64_t b = 0; b < k; ++b) {
            for (uint64_t x = lo_t[b]; x < lo_t[b] + cap_t[b]; ++x) {
                uint32_t l = labels[x];
                uint64_t r = cnt[l]++;
                if (r < cap_t[l]) {
                    /* placed at the front of the tile's piece of region E_l
                     * (Sec. 3.3: placed items sit at the front of a bucket) */
                    uint64_t y = lo_t[l] + r;
                    if (y >= S[l] && y < S[l] + N[l]) {
                        /* inside the final region of bucket l: stays */
                        out.put(out.ctx, x, y);
                        keeper[y] = 1;
                        continue;
                    }
                }
                /* Either the piece was full (a staged item) or the slot lies
                 * outside the final region once the boundaries move: the item
                 * is a mover.  Movers of a bucket are kept in tile order, then
                 * read order. */
                rc = poslist_push(&movers[l], x);
                if (rc != CSS_OK) goto out;
            }
        }
    }
    /* FineScatter's role (Sec. 3.4): bucket b's final region
     * F_b = [S_b, S_b + N_b) holds its kept items; its remaining positions,
     * in ascending order, take the movers of bucket b in order. */
    for (uint64_t b = 0; b < k; ++b) {
        uint64_t j = 0;
        for (uint64_t y = S[b]; y < S[b] + N[b]; ++y) {
            if (keeper[y]) continue;
            if (j >= movers[b].n) { rc = CSS_EINVAL; goto out; }
            out.put(out.ctx, movers[b].v[j], y);
            j++;
        }
        if (j != movers[b].n) { rc = CSS_EINVAL; goto out; }
    }
out:
    if (movers)
        for (uint64_t b = 0; b < k; ++b) free(movers[b].v);
    free(e); free(cnt); free(lo_t); free(cap_t); free(keeper); free(movers);
    return rc;
}

/* One level with given labels and counts N (k entries). */
static int level_to(const uint8_t* labels, uint64_t m, uint64_t k, uint64_t tile, int hbm_regime,
                    const uint64_t* N, sink_t out)
{
    uint64_t* S = calloc(k, sizeof(uint64_t));
    if (!S) return CSS_ENOMEM;
    for (uint64_t b = 1; b < k; ++b) S[b] = S[b - 1] + N[b - 1];
    int rc = hbm_regime ? rough_level(labels, m, k, tile, N, S, out)
                        : exact_level(labels, m, k, S, out);
    free(S);
    return rc;
}

static void put_dest(void* ctx, uint64_t x, uint64_t y) { ((uint64_t*)ctx)[x] = y; }

int css_level(const uint8_t* labels, uint64_t m, uint32_t kappa, uint64_t tile,
              int hbm_regime, uint64_t* dest)
{
    if (kappa < 1 || kappa > 8) return CSS_EINVAL;
    uint64_t k = UINT64_C(1) << kappa;
    if (hbm_regime && tile <= k) return CSS_EINVAL;
    uint64_t* N = calloc(k, sizeof(uint64_t));
    if (!N) return CSS_ENOMEM;
    for (uint64_t i = 0; i < m; ++i) {
        if (labels[i] >= k) { free(N); return CSS_EINVAL; }
        N[labels[i]]++;
    }
    sink_t out = {put_dest, dest};
    int rc = level_to(labels, m, k, tile, hbm_regime, N, out);
    free(N);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Fisher-Yates (Fig. 1, Sec. 2.2): for i from m-1 down to 1, swap item i
 * with a partner drawn uniformly from [0, i].  Expressed as a destination
 * map so that the same routine serves data of any width. */
int css_fy_dest(css_rng_t* rng, uint32_t level, uint64_t base, uint64_t m, uint64_t* dest)
{
    uint64_t* at = malloc((m ? m : 1) * sizeof(uint64_t)); /* at[pos] = original index */
    if (!at) return CSS_ENOMEM;
    for (uint64_t i = 0; i < m; ++i) at[i] = i;
    for (uint64_t i = m; i-- > 1;) {
        if (i + 1 > (UINT64_C(1) << 32)) { free(at); return CSS_EUNSUPPORTED; }
        uint64_t j = rng->draw(rng, level, base + i, i + 1);
        uint64_t tmp = at[i];
        at[i] = at[j];
        at[j] = tmp;
    }
    for (uint64_t pos = 0; pos < m; ++pos) dest[at[pos]] = pos;
    free(at);
    return CSS_OK;
}

/* ------------------------------------------------------------------------ */
/* The recursion (Fig. 2 and Theorem 1; Sec. 3.5): IpSc on the subproblem,
 * then recurse on every bucket; Fisher-Yates at the base case.  The buckets
 * of one level are independent subproblems (Sec. 4: after one IpSc level the
 * k subproblems can be processed in parallel), so the top level may hand its
 * buckets to host threads; every bucket is still solved by the same plain
 * solve(), and the result does not depend on the number of threads. */

typedef struct {
    uint8_t* data;
    uint32_t w;
    css_rng_t* rng;
    const css_params_t* p;
} solve_ctx_t;

typedef struct {
    const uint8_t* src;
    uint8_t* dst;
    uint32_t w;
} copy_ctx_t;

static void put_elem(void* ctx, uint64_t x, uint64_t y)
{
    copy_ctx_t* c = ctx;
    memcpy(c->dst + y * c->w, c->src + x * c->w, c->w);
}

/* Labels of positions base + [i0, i1) at `level`, counted into N. */
static void label_range(css_rng_t* rng, uint32_t level, uint64_t base, uint64_t i0, uint64_t i1,
                        uint32_t kappa, uint8_t* labels, uint64_t* N)
{
    for (uint64_t i = i0; i < i1; ++i) {
        labels[i] = (uint8_t)rng->label(rng, level, base + i, kappa);
        N[labels[i]]++;
    }
}

typedef struct {
    css_rng_t* rng;
    uint32_t level, kappa;
    uint64_t base, i0, i1;
    uint8_t* labels;
    uint64_t N[256];
} label_job_t;

static void* label_job(void* arg)
{
    label_job_t* j = arg;
    label_range(j->rng, j->level, j->base, j->i0, j->i1, j->kappa, j->labels, j->N);
    return NULL;
}

/* Labels of the whole subproblem, split over `threads` host threads. */
static int label_all(css_rng_t* rng, uint32_t level, uint64_t base, uint64_t m, uint32_t kappa,
                     uint32_t threads, uint8_t* labels, uint64_t* N)
{
    uint64_t k = UINT64_C(1) << kappa;
    if (threads <= 1 || m < (UINT64_C(1) << 20)) {
        label_range(rng, level, base, 0, m, kappa, labels, N);
        return CSS_OK;
    }
    label_job_t* jobs = calloc(threads, sizeof(label_job_t));
    pthread_t* tid = calloc(threads, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); return CSS_ENOMEM; }
    uint32_t started = 0;
    int rc = CSS_OK;
    for (uint32_t t = 0; t < threads; ++t) {
        jobs[t] = (label_job_t){rng, level, kappa, base, m * t / threads, m * (t + 1) / threads,
                                labels, {0}};
        if (pthread_create(&tid[t], NULL, label_job, &jobs[t]) != 0) { rc = CSS_ENOMEM; break; }
        started++;
    }
    for (uint32_t t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    if (rc == CSS_OK)
        for (uint32_t t = 0; t < threads; ++t)
            for (uint64_t b = 0; b < k; ++b) N[b] += jobs[t].N[b];
    free(jobs);
    free(tid);
    return rc;
}

static int solve(solve_ctx_t* c, uint64_t base, uint64_t m, uint32_t level, uint32_t threads);

/* Fisher-Yates base case on [base, base + m). */
static int solve_fy(solve_ctx_t* c, uint64_t base, uint64_t m, uint32_t level)
{
    uint64_t* dest = malloc(m * sizeof(uint64_t));
    uint8_t* tmp = malloc(m * c->w);
    int rc = (dest && tmp) ? CSS_OK : CSS_ENOMEM;
    if (rc == CSS_OK) rc = css_fy_dest(c->rng, level, base, m, dest);
    if (rc == CSS_OK) {
        uint8_t* a = c->data + base * c->w;
        for (uint64_t i = 0; i < m; ++i) memcpy(tmp + dest[i] * c->w, a + i * c->w, c->w);
        memcpy(a, tmp, m * c->w);
    }
    free(dest);
    free(tmp);
    return rc;
}

typedef struct {
    solve_ctx_t* c;
    const uint64_t* start;  /* bucket starts */
    const uint64_t* N;      /* bucket sizes */
    uint64_t k;
    uint32_t level;
    uint64_t next;          /* next bucket to take, under mu */
    int rc;
    pthread_mutex_t mu;
} bucket_pool_t;

static void* bucket_worker(void* arg)
{
    bucket_pool_t* bp = arg;
    for (;;) {
        pthread_mutex_lock(&bp->mu);
        uint64_t b = bp->next++;
        int stop = bp->rc != CSS_OK;
        pthread_mutex_unlock(&bp->mu);
        if (stop || b >= bp->k) return NULL;
        int rc = solve(bp->c, bp->start[b], bp->N[b], bp->level, 1);
        if (rc != CSS_OK) {
            pthread_mutex_lock(&bp->mu);
            if (bp->rc == CSS_OK) bp->rc = rc;
            pthread_mutex_unlock(&bp->mu);
        }
    }
}

/* The k children of a level, in order on one thread or taken from a shared
 * counter by `threads` host threads. */
static int solve_children(solve_ctx_t* c, uint64_t base, const uint64_t* N, uint64_t k,
                          uint32_t level, uint32_t threads)
{
    uint64_t* start = malloc(k * sizeof(uint64_t));
    if (!start) return CSS_ENOMEM;
    uint64_t s = base;
    for (uint64_t b = 0; b < k; ++b) {
        start[b] = s;
        s += N[b];
    }
    int rc = CSS_OK;
    if (threads <= 1) {
        for (uint64_t b = 0; b < k && rc == CSS_OK; ++b) rc = solve(c, start[b], N[b], level, 1);
        free(start);
        return rc;
    }
    bucket_pool_t bp = {c, start, N, k, level, 0, CSS_OK, PTHREAD_MUTEX_INITIALIZER};
    pthread_t* tid = calloc(threads, sizeof(pthread_t));
    uint32_t started = 0;
    if (tid)
        for (uint32_t t = 0; t < threads; ++t) {
            if (pthread_create(&tid[t], NULL, bucket_worker, &bp) != 0) break;
            started++;
        }
    if (started == 0) bucket_worker(&bp);  /* no thread could start: do it here */
    for (uint32_t t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    free(tid);
    free(start);
    return bp.rc;
}

static int solve(solve_ctx_t* c, uint64_t base, uint64_t m, uint32_t level, uint32_t threads)
{
    const css_params_t* p = c->p;
    if (m <= 1) return CSS_OK;
    if (m <= p->n0 || level >= p->lmax) return solve_fy(c, base, m, level);
    uint64_t kmax = UINT64_C(1) << p->kmax_log2;
    int hbm = m > p->tile - kmax;
    uint32_t kappa = css_kappa(m, hbm, p);
    uint64_t k = UINT64_C(1) << kappa;

    uint8_t* labels = malloc(m);
    uint8_t* out = malloc(m * c->w);
    uint64_t* N = calloc(k, sizeof(uint64_t));
    int rc = (labels && out && N) ? CSS_OK : CSS_ENOMEM;
    if (rc == CSS_OK) rc = label_all(c->rng, level, base, m, kappa, threads, labels, N);
    if (rc == CSS_OK) {
        uint8_t* a = c->data + base * c->w;
        copy_ctx_t cc = {a, out, c->w};
        sink_t sink = {put_elem, &cc};
        rc = level_to(labels, m, k, p->tile, hbm, N, sink);
        if (rc == CSS_OK) memcpy(a, out, m * c->w);
    }
    free(labels);
    free(out);
    if (rc == CSS_OK) rc = solve_children(c, base, N, k, level + 1, threads);
    free(N);
    return rc;
}

int css_shuffle_rng(void* data, uint64_t n, uint32_t w, css_rng_t* rng, const css_params_t* p)
{
    int rc = css_check_params(p);
    if (rc != CSS_OK) return rc;
    if (w == 0 || (!data && n > 0)) return CSS_EINVAL;
    solve_ctx_t c = {(uint8_t*)data, w, rng, p};
    return solve(&c, 0, n, 0, 1);
}

int css_shuffle(void* data, uint64_t n, uint32_t w, uint64_t seed, uint32_t stream_id,
                const css_params_t* p)
{
    return css_shuffle_mt(data, n, w, seed, stream_id, p, 1);
}

int css_shuffle_mt(void* data, uint64_t n, uint32_t w, uint64_t seed, uint32_t stream_id,
                   const css_params_t* p, uint32_t threads)
{
    int rc = css_check_params(p);
    if (rc != CSS_OK) return rc;
    if (w == 0 || (!data && n > 0)) return CSS_EINVAL;
    css_rng_t rng = {philox_label_cb, philox_draw_cb, seed, stream_id, NULL};
    solve_ctx_t c = {(uint8_t*)data, w, &rng, p};
    return solve(&c, 0, n, 0, threads ? threads : 1);
}

int css_fisher_yates(void* data, uint64_t n, uint32_t w, uint64_t seed, uint32_t stream_id)
{
    if (w == 0 || (!data && n > 0)) return CSS_EINVAL;
    if (n > (UINT64_C(1) << 32)) return CSS_EUNSUPPORTED;
    uint8_t* a = data;
    uint8_t tmp[64];
    if (w > sizeof tmp) return CSS_EINVAL;
    for (uint64_t i = n; i-- > 1;) {
        uint64_t j = css_draw(seed, stream_id, 0, i, i + 1);
        memcpy(tmp, a + i * w, w);
        memcpy(a + i * w, a + j * w, w);
        memcpy(a + j * w, tmp, w);
    }
    return CSS_OK;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive enumeration.  A scripted provider answers every random request
 * from a decision vector; requests beyond the vector's end answer 0 and
 * record their arity.  Visiting decision vectors in odometer order walks
 * every leaf of the decision tree once; a leaf's probability is the product
 * of 1/arity over its decisions. */

#define ENUM_MAX_DEPTH 4096

typedef struct {
    uint64_t choice[ENUM_MAX_DEPTH];
    uint64_t arity[ENUM_MAX_DEPTH];
    uint32_t len;   /* decisions fixed by the odometer */
    uint32_t depth; /* decisions consumed in the current run */
    int overflow;
} script_t;

static uint64_t script_next(script_t* s, uint64_t arity)
{
    if (s->depth >= ENUM_MAX_DEPTH) {
        s->overflow = 1;
        return 0;
    }
    uint32_t i = s->depth++;
    if (i >= s->len) {
        s->choice[i] = 0;
        s->len = i + 1;
    }
    s->arity[i] = arity;
    return s->choice[i];
}

static uint32_t script_label_cb(css_rng_t* self, uint32_t level, uint64_t pos, uint32_t kappa)
{
    (void)level; (void)pos;
    return (uint32_t)script_next((script_t*)self->ctx, UINT64_C(1) << kappa);
}

static uint64_t script_draw_cb(css_rng_t* self, uint32_t level, uint64_t pos, uint64_t bound)
{
    (void)level; (void)pos;
    return script_next((script_t*)self->ctx, bound);
}

static uint64_t perm_rank(const uint8_t* a, uint32_t m)
{
    /* lexicographic rank via the factorial number system */
    uint64_t rank = 0;
    for (uint32_t i = 0; i < m; ++i) {
        uint64_t smaller = 0;
        for (uint32_t j = i + 1; j < m; ++j)
            if (a[j] < a[i]) smaller++;
        uint64_t f = 1;
        for (uint32_t q = 2; q <= m - 1 - i; ++q) f *= q;
        rank += smaller * f;
    }
    return rank;
}

int css_enumerate(uint32_t m, const css_params_t* p, double* prob, uint64_t* paths)
{
    if (m > 8) return CSS_EINVAL;
    int rc = css_check_params(p);
    if (rc != CSS_OK) return rc;
    uint64_t fact = 1;
    for (uint32_t q = 2; q <= m; ++q) fact *= q;
    for (uint64_t r = 0; r < fact; ++r) prob[r] = 0.0;
    script_t* s = calloc(1, sizeof(script_t));
    if (!s) return CSS_ENOMEM;
    css_rng_t rng = {script_label_cb, script_draw_cb, 0, 0, s};
    uint64_t count = 0;
    for (;;) {
        uint8_t a[8];
        for (uint32_t i = 0; i < m; ++i) a[i] = (uint8_t)i;
        s->depth = 0;
        rc = css_shuffle_rng(a, m, 1, &rng, p);
        if (rc != CSS_OK) break;
        if (s->overflow) { rc = CSS_EUNSUPPORTED; break; }
        double wgt = 1.0;
        for (uint32_t i = 0; i < s->depth; ++i) wgt /= (double)s->arity[i];
        prob[perm_rank(a, m)] += wgt;
        count++;
        /* advance the odometer over the decisions of this run */
        int32_t i = (int32_t)s->depth - 1;
        while (i >= 0 && s->choice[i] + 1 >= s->arity[i]) i--;
        if (i < 0) break;
        s->choice[i]++;
        s->len = (uint32_t)i + 1;
    }
    free(s);
    if (paths) *paths = count;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Statistics helpers for the uniformity tests (loops kept in C for speed). */

/* counts[rank] += 1 for the permutation of 0..m-1 produced with each seed in
 * [seed0, seed0 + nseeds); m <= 8. */
int css_perm_histogram(uint32_t m, uint64_t seed0, uint64_t nseeds, const css_params_t* p,
                       uint64_t* counts)
{
    if (m > 8) return CSS_EINVAL;
    for (uint64_t s = 0; s < nseeds; ++s) {
        uint8_t a[8];
        for (uint32_t i = 0; i < m; ++i) a[i] = (uint8_t)i;
        int rc = css_shuffle(a, m, 1, seed0 + s, 0, p);
        if (rc != CSS_OK) return rc;
        counts[perm_rank(a, m)]++;
    }
    return CSS_OK;
}

/* counts[i * n + j] += 1 when item i ends at position j, over nseeds seeds. */
int css_position_histogram(uint32_t n, uint64_t seed0, uint64_t nseeds, const css_params_t* p,
                           uint64_t* counts)
{
    uint32_t* a = malloc((n ? n : 1) * sizeof(uint32_t));
    if (!a) return CSS_ENOMEM;
    for (uint64_t s = 0; s < nseeds; ++s) {
        for (uint32_t i = 0; i < n; ++i) a[i] = i;
        int rc = css_shuffle(a, n, 4, seed0 + s, 0, p);
        if (rc != CSS_OK) { free(a); return rc; }
        for (uint32_t j = 0; j < n; ++j) counts[(uint64_t)a[j] * n + j]++;
    }
    free(a);
    return CSS_OK;
}
