/*
 * FP64 CPU oracle for one-hot graph encoder embedding (GEE).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or load
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do. It shares no code, header, table or helper with the GPU library.
 *
 * What is computed (Lubonja, Shen, Priebe, Burns, "Edge-Parallel Graph Encoder
 * Embedding", Section II, Algorithm 1 "Semi-Supervised GEE"):
 *   - the projection W: W(v, k) = 1 / count(Y = k) for every v with Y(v) = k,
 *     for k = 1..K; class 0 marks an unknown label and gets no column
 *     (Algorithm 1, projection-matrix initialisation);
 *   - one pass over the s records (u, v, w): Z(u, Y(v)) += W(v, Y(v)) * w and
 *     Z(v, Y(u)) += W(u, Y(u)) * w (Algorithm 1, edge loop). The source node
 *     contributes to the destination's class and vice versa; unweighted graphs
 *     use w = 1 (Section II).
 * The result equals the plain definition Z = (A + A^T) M, A[u][v] = sum of w over
 * the records (u, v), M[v][k-1] = [Y(v) = k] / n_k.
 *
 * The Laplacian version is not spelled out in the paper (Section II leaves out
 * its preprocessing). Reading used here: each record's weight is first
 * multiplied by 1 / sqrt(d_u * d_v), d the weighted degree d = (A + A^T) 1, so
 * that Z = D^-1/2 (A + A^T) D^-1/2 M; a vertex of degree 0 gets factor 0.
 *
 * Conventions (readings of the paper): vertex ids are 0-based in [0, n); class
 * k in 1..K goes to column k-1 of the row-major n x K matrix Z; an update whose
 * target class is 0 (unknown) is skipped while the record's other update still
 * happens; self-loops fire both updates; repeated records add up; an empty
 * class has weight 0 (never read).
 *
 * Arithmetic: FP64 throughout, single thread, records in input order, updates
 * pre-scaled by W exactly as Algorithm 1 writes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Return codes of the oracle (its own; they mirror the meaning of the GPU
 * library's codes without sharing its header). */
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ELABEL (-2)
#define OR_EVERTEX (-3)
#define OR_ENEGW (-4)
#define OR_ENOMEM (-8)

/* Class counts n_k = #{v : Y(v) = k}, k = 0..K (index 0 counts unknown
 * labels). Algorithm 1's count(Y = k). Fails on a label outside [0, K]. */
int oracle_counts(int64_t n, const int32_t *Y, int32_t K, int64_t *counts)
{
    if (n < 1 || K < 1 || !Y || !counts) return OR_EINVAL;
    for (int32_t k = 0; k <= K; ++k) counts[k] = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (Y[v] < 0 || Y[v] > K) return OR_ELABEL;
        counts[Y[v]] += 1;
    }
    return OR_OK;
}

/* The one nonzero of each row of W, per class: inv[k] = 1 / count(Y = k)
 * (Algorithm 1, projection-matrix initialisation); inv[0] = 0 (unknown class
 * has no column) and inv[k] = 0 for an empty class. */
int oracle_weights(const int64_t *counts, int32_t K, double *inv)
{
    if (K < 1 || !counts || !inv) return OR_EINVAL;
    inv[0] = 0.0;
    for (int32_t k = 1; k <= K; ++k) inv[k] = counts[k] > 0 ? 1.0 / (double)counts[k] : 0.0;
    return OR_OK;
}

static int check_records(int64_t n, int64_t s, const int32_t *src, const int32_t *dst)
{
    for (int64_t i = 0; i < s; ++i)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return OR_EVERTEX;
    return OR_OK;
}

/* Weighted degree d[u] = sum over records of w at each endpoint (a self-loop
 * adds 2w), accumulated in record order. */
int oracle_degrees(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w,
                   double *deg)
{
    if (n < 1 || s < 0 || (s > 0 && (!src || !dst)) || !deg) return OR_EINVAL;
    int rc = check_records(n, s, src, dst);
    if (rc) return rc;
    for (int64_t u = 0; u < n; ++u) deg[u] = 0.0;
    for (int64_t i = 0; i < s; ++i) {
        double x = w ? (double)w[i] : 1.0;
        deg[src[i]] += x;
        deg[dst[i]] += x;
    }
    return OR_OK;
}

/* Shared set-up of both embed entry points: validation, counts, W and, for
 * the Laplacian, r = d^-1/2. `r` is allocated here when laplacian != 0. */
static int prepare(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w,
                   const int32_t *Y, int32_t K, int laplacian, double *inv, double **r_out)
{
    int64_t *counts;
    int rc;
    *r_out = NULL;
    if (n < 1 || s < 0 || K < 1 || !Y || (s > 0 && (!src || !dst))) return OR_EINVAL;
    rc = check_records(n, s, src, dst);
    if (rc) return rc;
    if (laplacian && w)
        for (int64_t i = 0; i < s; ++i)
            if (!(w[i] >= 0.0f)) return OR_ENEGW;
    counts = (int64_t *)malloc(sizeof(int64_t) * (size_t)(K + 1));
    if (!counts) return OR_ENOMEM;
    rc = oracle_counts(n, Y, K, counts);
    if (rc == OR_OK) rc = oracle_weights(counts, K, inv);
    free(counts);
    if (rc) return rc;
    if (laplacian) {
        double *d = (double *)malloc(sizeof(double) * (size_t)n);
        if (!d) return OR_ENOMEM;
        rc = oracle_degrees(n, s, src, dst, w, d);
        if (rc) {
            free(d);
            return rc;
        }
        for (int64_t u = 0; u < n; ++u) d[u] = d[u] > 0.0 ? 1.0 / sqrt(d[u]) : 0.0;
        *r_out = d;
    }
    return OR_OK;
}

/* Algorithm 1 over all rows. Z is n x K row-major FP64 and must be zero on
 * entry (the algorithm starts from an all-zero Z); it is accumulated into. */
int oracle_embed(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w,
                 const int32_t *Y, int32_t K, int laplacian, double *Z)
{
    double *inv, *r = NULL;
    int rc;
    if (!Z) return OR_EINVAL;
    inv = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K + 1 : 1));
    if (!inv) return OR_ENOMEM;
    rc = prepare(n, s, src, dst, w, Y, K, laplacian, inv, &r);
    if (rc) {
        free(inv);
        return rc;
    }
    for (int64_t i = 0; i < s; ++i) {
        const int64_t u = src[i], v = dst[i];
        double x = w ? (double)w[i] : 1.0;
        if (laplacian) x = x * r[u] * r[v];
        if (Y[v] > 0) Z[u * K + (Y[v] - 1)] += inv[Y[v]] * x; /* Z(u, Y(v)) += W(v, Y(v)) w */
        if (Y[u] > 0) Z[v * K + (Y[u] - 1)] += inv[Y[u]] * x; /* Z(v, Y(u)) += W(u, Y(u)) w */
    }
    free(r);
    free(inv);
    return OR_OK;
}

/* The same pass restricted to a set of rows: rows[0..nrows) are distinct
 * vertex ids and Zrows is nrows x K (zero on entry); row rows[j] of Z lands
 * in row j of Zrows. Every record is still visited in order, so each sampled
 * row receives exactly the updates, in exactly the order, of oracle_embed. */
int oracle_embed_rows(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w,
                      const int32_t *Y, int32_t K, int laplacian, int64_t nrows, const int64_t *rows,
                      double *Zrows)
{
    double *inv, *r = NULL;
    int32_t *slot;
    uint64_t *mark;
    int rc;
    if (nrows < 0 || (nrows > 0 && (!rows || !Zrows))) return OR_EINVAL;
    inv = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K + 1 : 1));
    if (!inv) return OR_ENOMEM;
    rc = prepare(n, s, src, dst, w, Y, K, laplacian, inv, &r);
    if (rc) {
        free(inv);
        return rc;
    }
    /* a bitmap filters records quickly; slot maps a sampled vertex to its row */
    mark = (uint64_t *)calloc((size_t)(n + 63) / 64, sizeof(uint64_t));
    slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!mark || !slot) {
        free(mark);
        free(slot);
        free(r);
        free(inv);
        return OR_ENOMEM;
    }
    for (int64_t j = 0; j < nrows; ++j) {
        if (rows[j] < 0 || rows[j] >= n) {
            rc = OR_EVERTEX;
            break;
        }
        mark[rows[j] >> 6] |= 1ULL << (rows[j] & 63);
        slot[rows[j]] = (int32_t)j;
    }
    if (rc == OR_OK) {
        for (int64_t i = 0; i < s; ++i) {
            const int64_t u = src[i], v = dst[i];
            const int hu = (int)((mark[u >> 6] >> (u & 63)) & 1u);
            const int hv = (int)((mark[v >> 6] >> (v & 63)) & 1u);
            if (!hu && !hv) continue;
            double x = w ? (double)w[i] : 1.0;
            if (laplacian) x = x * r[u] * r[v];
            if (hu && Y[v] > 0) Zrows[(int64_t)slot[u] * K + (Y[v] - 1)] += inv[Y[v]] * x;
            if (hv && Y[u] > 0) Zrows[(int64_t)slot[v] * K + (Y[u] - 1)] += inv[Y[u]] * x;
        }
    }
    free(mark);
    free(slot);
    free(r);
    free(inv);
    return rc;
}
