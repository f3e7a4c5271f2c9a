/* Edge-parallel GEE on the host's cores, FP64, for timing beside the GPU path.
 *
 * TIMING BASELINE ONLY: the benchmark's CPU comparison and its test use this; the GPU
 * library never links or calls it. It follows the paper's parallel design (Section III):
 * the edge pass runs over the records in parallel and every update of Z is a lock-free
 * atomic add (compare-and-swap on the 64-bit value), since two records can update the
 * same element (Fig. 1's race). Class counts are per-thread histograms summed after the
 * loop; the Laplacian degrees use the same atomic adds. Algorithm 1's W is kept as one
 * weight per class, W(v, Y(v)) = 1 / count(Y = Y(v)), and each update adds
 * W(v, Y(v)) * w as Algorithm 1 writes it.
 *
 * Status codes: 0 ok, -1 bad argument, -2 label outside [0, K], -3 vertex outside
 * [0, n), -4 negative weight in the Laplacian version, -8 out of memory. */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline void atomic_add_f64(double *p, double x)
{
    uint64_t *q = (uint64_t *)p;
    uint64_t old = __atomic_load_n(q, __ATOMIC_RELAXED), nw;
    do {
        double d;
        memcpy(&d, &old, 8);
        d += x;
        memcpy(&nw, &d, 8);
    } while (!__atomic_compare_exchange_n(q, &old, nw, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED));
}

/* Z[0 .. count) = 0 in parallel (also brings the pages in before a timed call). */
void cpu_zero(double *Z, int64_t count, int threads)
{
#pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t i = 0; i < count; ++i) Z[i] = 0.0;
}

int cpu_embed_atomic(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w, const int32_t *Y,
                     int32_t K, int laplacian, double *Z, int threads)
{
    if (n < 1 || s < 0 || K < 1 || !Y || !Z || (s > 0 && (!src || !dst)) || threads < 1) return -1;
    int rc = 0;
    int64_t *cnt = (int64_t *)calloc((size_t)threads * (size_t)(K + 1), sizeof(int64_t));
    double *inv = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    double *r = laplacian ? (double *)calloc((size_t)n, sizeof(double)) : NULL;
    if (!cnt || !inv || (laplacian && !r)) {
        free(cnt);
        free(inv);
        free(r);
        return -8;
    }
    /* class counts: one histogram per thread, then summed */
#pragma omp parallel num_threads(threads)
    {
        int64_t *h = cnt + (size_t)omp_get_thread_num() * (size_t)(K + 1);
        int bad = 0;
#pragma omp for schedule(static)
        for (int64_t v = 0; v < n; ++v) {
            if (Y[v] < 0 || Y[v] > K) bad = 1;
            else h[Y[v]] += 1;
        }
        if (bad) {
#pragma omp atomic write
            rc = -2;
        }
    }
    for (int t = 1; t < threads; ++t)
        for (int32_t k = 0; k <= K; ++k) cnt[k] += cnt[(size_t)t * (size_t)(K + 1) + (size_t)k];
    inv[0] = 0.0;
    for (int32_t k = 1; k <= K; ++k) inv[k] = cnt[k] > 0 ? 1.0 / (double)cnt[k] : 0.0;
    /* record checks, and the Laplacian degrees by atomic adds */
    if (rc == 0) {
#pragma omp parallel for schedule(static) num_threads(threads)
        for (int64_t i = 0; i < s; ++i) {
            const int32_t u = src[i], v = dst[i];
            if (u < 0 || u >= n || v < 0 || v >= n) {
#pragma omp atomic write
                rc = -3;
                continue;
            }
            if (laplacian) {
                const double x = w ? (double)w[i] : 1.0;
                if (!(x >= 0.0)) {
#pragma omp atomic write
                    rc = -4;
                    continue;
                }
                atomic_add_f64(&r[u], x);
                atomic_add_f64(&r[v], x);
            }
        }
    }
    if (rc == 0 && laplacian) {
#pragma omp parallel for schedule(static) num_threads(threads)
        for (int64_t u = 0; u < n; ++u) r[u] = r[u] > 0.0 ? 1.0 / sqrt(r[u]) : 0.0;
    }
    /* the edge pass */
    if (rc == 0) {
#pragma omp parallel for schedule(static) num_threads(threads)
        for (int64_t i = 0; i < s; ++i) {
            const int64_t u = src[i], v = dst[i];
            double x = w ? (double)w[i] : 1.0;
            if (laplacian) x = x * r[u] * r[v];
            const int32_t yu = Y[u], yv = Y[v];
            if (yv > 0) atomic_add_f64(&Z[u * K + (yv - 1)], inv[yv] * x);
            if (yu > 0) atomic_add_f64(&Z[v * K + (yu - 1)], inv[yu] * x);
        }
    }
    free(cnt);
    free(inv);
    free(r);
    return rc;
}
