/*
 * Seeded synthetic inputs for one-hot graph encoder embedding: edge lists
 * (stochastic block model, Erdos-Renyi G(n, m), R-MAT) and label vectors.
 *
 * This module holds no part of the embedding's arithmetic. Both the FP64
 * oracle and the GPU path consume what it writes, so every value must be a
 * pure function of (seed, stream, counter): records are generated
 * independently of thread count and scheduling.
 *
 * Random numbers: a counter-based SplitMix64 stream. SplitMix64 is the
 * generator of Steele, Lea and Flood ("Fast splittable pseudorandom number
 * generators", OOPSLA 2014); output i of the stream with key k is the
 * SplitMix64 finaliser applied to k + (i + 1) * golden, where golden is the
 * 64-bit golden-ratio increment. The finaliser constants are the published
 * ones of that generator.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

enum {
    STREAM_ER_SRC = 1,
    STREAM_ER_DST = 2,
    STREAM_ER_W = 3,
    STREAM_RMAT = 4,
    STREAM_LABEL = 5,
    STREAM_UNLABEL_EXACT = 6,
    STREAM_SBM_PAIR = 7,
    STREAM_SHUFFLE = 8,
    STREAM_UNLABEL_BERN = 9,
    STREAM_SCRAMBLE = 10,
    STREAM_SBM_FLIP = 11,
    STREAM_WEIGHT = 12,
    /* 13: per-vector batch parameters (drawn from Python) */
    STREAM_SBMR_TYPE = 14,
    STREAM_SBMR_U = 15,
    STREAM_SBMR_V = 16,
};

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Key of the stream (seed, stream). */
static inline uint64_t rng_key(uint64_t seed, uint64_t stream)
{
    return mix64(seed * GOLDEN + stream * 0xd1b54a32d192ed03ULL + 1);
}

/* Output `ctr` of the SplitMix64 stream with key `key`. */
static inline uint64_t rng_keyed(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * GOLDEN); }

/* Output `ctr` of the SplitMix64 stream keyed by (seed, stream). */
static inline uint64_t rng_at(uint64_t seed, uint64_t stream, uint64_t ctr)
{
    return rng_keyed(rng_key(seed, stream), ctr);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* Integer in [0, m) by multiply-shift of the top 32 bits (m < 2^32). */
static inline uint64_t bounded32(uint64_t x, uint64_t m) { return ((x >> 32) * m) >> 32; }

/* Exposed for tests of the stream itself. */
uint64_t gen_rng_at(uint64_t seed, uint64_t stream, uint64_t ctr) { return rng_at(seed, stream, ctr); }

/* ---------------------------------------------------------------- ER ---- */

/* G(n, m) with m = s records: endpoints i.i.d. uniform over [0, n), so
 * self-loops and repeated pairs occur and are kept. Weights, when w != NULL,
 * are (r + 1) * 2^-24 with r uniform in [0, 2^24): exactly representable in
 * FP32, in (0, 1], on the 2^-24 grid. */
void gen_er(int64_t n, int64_t s, uint64_t seed, int32_t *src, int32_t *dst, float *w)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s; ++i) {
        src[i] = (int32_t)bounded32(rng_at(seed, STREAM_ER_SRC, (uint64_t)i), (uint64_t)n);
        dst[i] = (int32_t)bounded32(rng_at(seed, STREAM_ER_DST, (uint64_t)i), (uint64_t)n);
        if (w) {
            uint64_t r = rng_at(seed, STREAM_ER_W, (uint64_t)i) >> 40; /* 24 bits */
            w[i] = (float)(r + 1) * 0x1.0p-24f;
        }
    }
}

/* Grid weights for an existing edge list: same law as gen_er's weights. */
void gen_grid_weights(int64_t s, uint64_t seed, float *w)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s; ++i) {
        uint64_t r = rng_at(seed, STREAM_WEIGHT, (uint64_t)i) >> 40;
        w[i] = (float)(r + 1) * 0x1.0p-24f;
    }
}

/* -------------------------------------------------------------- R-MAT ---- */

/* A bijection of [0, 2^scale): two affine maps with odd multipliers
 * interleaved with xor-shifts, each invertible on scale-bit integers. */
typedef struct {
    uint64_t mask, m1, c1, m2, c2;
    int sh1, sh2;
} scramble_t;

static scramble_t scramble_make(int scale, uint64_t seed)
{
    scramble_t p;
    p.mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1ULL);
    p.m1 = rng_at(seed, STREAM_SCRAMBLE, 0) | 1ULL;
    p.c1 = rng_at(seed, STREAM_SCRAMBLE, 1);
    p.m2 = rng_at(seed, STREAM_SCRAMBLE, 2) | 1ULL;
    p.c2 = rng_at(seed, STREAM_SCRAMBLE, 3);
    p.sh1 = scale / 2 + 1;
    p.sh2 = scale / 3 + 1;
    return p;
}

static inline uint64_t scramble_apply(const scramble_t *p, uint64_t v)
{
    v = (v * p->m1 + p->c1) & p->mask;
    v ^= v >> p->sh1;
    v = (v * p->m2 + p->c2) & p->mask;
    v ^= v >> p->sh2;
    return v & p->mask;
}

uint64_t gen_scramble(int scale, uint64_t seed, uint64_t v)
{
    scramble_t p = scramble_make(scale, seed);
    return scramble_apply(&p, v);
}

/* R-MAT: each record picks one of four quadrants per level, `scale` levels,
 * with probabilities (a, b, c, 1-a-b-c); quadrant (0,0) keeps both bits 0,
 * b sets the destination bit, c the source bit, d both. No noise. Each level
 * draws 32 bits (two levels per 64-bit output). When `scramble` is set, ids
 * pass through a seeded bijection of [0, 2^scale) so that vertex id carries
 * no degree information. Records keep generation order; self-loops and
 * duplicates are kept. */
void gen_rmat(int scale, int64_t s, double a, double b, double c, uint64_t seed, int scramble,
              int32_t *src, int32_t *dst)
{
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tab = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tabc = (uint64_t)((a + b + c) * 4294967296.0);
    const int nw = (scale + 1) / 2;
    scramble_t p = scramble_make(scale, seed);
    const uint64_t key = rng_key(seed, STREAM_RMAT);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s; ++i) {
        uint64_t u = 0, v = 0;
        const uint64_t base = (uint64_t)i * (uint64_t)nw;
        uint64_t x = 0;
        for (int level = 0; level < scale; ++level) {
            if ((level & 1) == 0) x = rng_keyed(key, base + (uint64_t)(level >> 1));
            const uint64_t r = ((level & 1) == 0) ? (x & 0xffffffffULL) : (x >> 32);
            /* quadrant: r < ta -> (0,0); < tab -> (0,1); < tabc -> (1,0); else (1,1) */
            const uint64_t ge_a = r >= ta, ge_ab = r >= tab, ge_abc = r >= tabc;
            u = (u << 1) | ge_ab;
            v = (v << 1) | (ge_a ^ ge_ab ^ ge_abc);
        }
        if (scramble) {
            u = scramble_apply(&p, u);
            v = scramble_apply(&p, v);
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
}

/* ---------------------------------------------------------------- SBM ---- */

static inline int64_t sbm_block(int64_t v, int64_t n, int64_t nb) { return (v * nb) / n; }

/* Stochastic block model on n vertices in nb equal consecutive blocks: every
 * unordered pair {u < v} is an edge independently with probability p_in
 * (same block) or p_out, decided by the pair's own counter. Each pair is
 * stored once, oriented at random, and the records are then shuffled by a
 * seeded Fisher-Yates pass. Returns the record count, or -1 if it would
 * exceed `cap` (nothing useful is written then). */
/* SBM by record sampling, for graphs too large for pair enumeration: s records, each a
 * within-block pair with probability p_within and a between-block pair otherwise, both
 * endpoints uniform under that constraint (repeats and self-loops possible). With
 * p_within = r W / (r W + B) for W within-block and B between-block vertex pairs, the
 * expected density inside blocks is r times that between them. */
void gen_sbm_records(int64_t n, int64_t nb, double p_within, int64_t s, uint64_t seed, int32_t *src, int32_t *dst)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s; ++i) {
        const int64_t u = (int64_t)bounded32(rng_at(seed, STREAM_SBMR_U, (uint64_t)i), (uint64_t)n);
        const int64_t bu = sbm_block(u, n, nb);
        const int64_t b0 = (bu * n + nb - 1) / nb, b1 = ((bu + 1) * n + nb - 1) / nb; /* block bu = [b0, b1) */
        const uint64_t rv = rng_at(seed, STREAM_SBMR_V, (uint64_t)i);
        int64_t v;
        if (u01(rng_at(seed, STREAM_SBMR_TYPE, (uint64_t)i)) < p_within || b1 - b0 == n) {
            v = b0 + (int64_t)bounded32(rv, (uint64_t)(b1 - b0));
        } else {
            v = (int64_t)bounded32(rv, (uint64_t)(n - (b1 - b0)));
            if (v >= b0) v += b1 - b0;
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
}

int64_t gen_sbm(int64_t n, int64_t nb, double p_in, double p_out, uint64_t seed, int64_t cap,
                int32_t *src, int32_t *dst)
{
    int64_t *rowcnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!rowcnt) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < n; ++u) {
        int64_t cnt = 0, bu = sbm_block(u, n, nb);
        for (int64_t v = u + 1; v < n; ++v) {
            double p = (sbm_block(v, n, nb) == bu) ? p_in : p_out;
            if (u01(rng_at(seed, STREAM_SBM_PAIR, (uint64_t)(u * n + v))) < p) ++cnt;
        }
        rowcnt[u + 1] = cnt;
    }
    for (int64_t u = 0; u < n; ++u) rowcnt[u + 1] += rowcnt[u];
    int64_t s = rowcnt[n];
    if (s > cap) {
        free(rowcnt);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < n; ++u) {
        int64_t pos = rowcnt[u], bu = sbm_block(u, n, nb);
        for (int64_t v = u + 1; v < n; ++v) {
            double p = (sbm_block(v, n, nb) == bu) ? p_in : p_out;
            uint64_t pair = (uint64_t)(u * n + v);
            if (u01(rng_at(seed, STREAM_SBM_PAIR, pair)) < p) {
                int flip = (int)(rng_at(seed, STREAM_SBM_FLIP, pair) & 1u);
                src[pos] = (int32_t)(flip ? v : u);
                dst[pos] = (int32_t)(flip ? u : v);
                ++pos;
            }
        }
    }
    free(rowcnt);
    for (int64_t i = s - 1; i > 0; --i) {
        int64_t j = (int64_t)bounded32(rng_at(seed, STREAM_SHUFFLE, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = src[i];
        src[i] = src[j];
        src[j] = t;
        t = dst[i];
        dst[i] = dst[j];
        dst[j] = t;
    }
    return s;
}

/* ------------------------------------------------------------- labels ---- */

/* Y[v] = 1 + uniform class in [0, K). */
void gen_labels_uniform(int64_t n, int32_t K, uint64_t seed, int32_t *Y)
{
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v)
        Y[v] = 1 + (int32_t)bounded32(rng_at(seed, STREAM_LABEL, (uint64_t)v), (uint64_t)K);
}

/* Set exactly m labels to 0 (unknown), the m chosen uniformly without
 * replacement by a partial Fisher-Yates shuffle of [0, n). */
int gen_unlabel_exact(int64_t n, int64_t m, uint64_t seed, int32_t *Y)
{
    if (m < 0 || m > n) return -1;
    int32_t *idx = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!idx) return -1;
    for (int64_t v = 0; v < n; ++v) idx[v] = (int32_t)v;
    for (int64_t i = 0; i < m; ++i) {
        int64_t j = i + (int64_t)bounded32(rng_at(seed, STREAM_UNLABEL_EXACT, (uint64_t)i), (uint64_t)(n - i));
        int32_t t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
        Y[idx[i]] = 0;
    }
    free(idx);
    return 0;
}

/* Set each label to 0 independently with probability f. */
void gen_unlabel_bernoulli(int64_t n, double f, uint64_t seed, int32_t *Y)
{
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v)
        if (u01(rng_at(seed, STREAM_UNLABEL_BERN, (uint64_t)v)) < f) Y[v] = 0;
}

/* Seeded shuffle of an edge list in place (record order only). */
void gen_shuffle_records(int64_t s, uint64_t seed, int32_t *src, int32_t *dst, float *w)
{
    for (int64_t i = s - 1; i > 0; --i) {
        int64_t j = (int64_t)bounded32(rng_at(seed, STREAM_SHUFFLE, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = src[i];
        src[i] = src[j];
        src[j] = t;
        t = dst[i];
        dst[i] = dst[j];
        dst[j] = t;
        if (w) {
            float tw = w[i];
            w[i] = w[j];
            w[j] = tw;
        }
    }
}
