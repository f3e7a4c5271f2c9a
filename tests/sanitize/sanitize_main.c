/* Runs the C oracle and the seeded generators under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only). The buffers are allocated here,
 * so the sanitizer's allocator puts red zones around every array the two
 * libraries read or write. Each result is printed as "name rc hash" (FNV-1a over
 * the output bytes); the test that builds this program compares every line with
 * the same calls made through the uninstrumented libraries. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_counts(int64_t n, const int32_t *Y, int32_t K, int64_t *counts);
int oracle_weights(const int64_t *counts, int32_t K, double *inv);
int oracle_degrees(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w, double *deg);
int oracle_embed(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w, const int32_t *Y,
                 int32_t K, int laplacian, double *Z);
int oracle_embed_rows(int64_t n, int64_t s, const int32_t *src, const int32_t *dst, const float *w, const int32_t *Y,
                      int32_t K, int laplacian, int64_t nrows, const int64_t *rows, double *Zrows);
void gen_er(int64_t n, int64_t s, uint64_t seed, int32_t *src, int32_t *dst, float *w);
void gen_grid_weights(int64_t s, uint64_t seed, float *w);
void gen_rmat(int scale, int64_t s, double a, double b, double c, uint64_t seed, int scramble, int32_t *src,
              int32_t *dst);
void gen_sbm_records(int64_t n, int64_t nb, double p_within, int64_t s, uint64_t seed, int32_t *src, int32_t *dst);
int64_t gen_sbm(int64_t n, int64_t nb, double p_in, double p_out, uint64_t seed, int64_t cap, int32_t *src,
                int32_t *dst);
void gen_labels_uniform(int64_t n, int32_t K, uint64_t seed, int32_t *Y);
int gen_unlabel_exact(int64_t n, int64_t m, uint64_t seed, int32_t *Y);
void gen_unlabel_bernoulli(int64_t n, double f, uint64_t seed, int32_t *Y);
void gen_shuffle_records(int64_t s, uint64_t seed, int32_t *src, int32_t *dst, float *w);

static uint64_t fnv(const void *p, size_t bytes)
{
    const unsigned char *c = (const unsigned char *)p;
    uint64_t h = 1469598103934665603ULL;
    for (size_t i = 0; i < bytes; ++i) {
        h ^= c[i];
        h *= 1099511628211ULL;
    }
    return h;
}

static void *xcalloc(size_t count, size_t size)
{
    void *p = calloc(count ? count : 1, size);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void out(const char *name, long rc, const void *p, size_t bytes)
{
    printf("%s %ld %016llx\n", name, rc, (unsigned long long)fnv(p, bytes));
}

/* Every oracle entry point on one graph and label vector, both versions. */
static void embed_all(const char *tag, int64_t n, int64_t s, const int32_t *src, const int32_t *dst,
                      const float *w, const int32_t *Y, int32_t K)
{
    char name[96];
    int64_t *cnt = xcalloc((size_t)K + 1, sizeof(int64_t));
    double *inv = xcalloc((size_t)K + 1, sizeof(double));
    double *deg = xcalloc((size_t)n, sizeof(double));
    snprintf(name, sizeof name, "%s.counts", tag);
    out(name, oracle_counts(n, Y, K, cnt), cnt, sizeof(int64_t) * ((size_t)K + 1));
    snprintf(name, sizeof name, "%s.weights", tag);
    out(name, oracle_weights(cnt, K, inv), inv, sizeof(double) * ((size_t)K + 1));
    snprintf(name, sizeof name, "%s.degrees", tag);
    out(name, oracle_degrees(n, s, src, dst, w, deg), deg, sizeof(double) * (size_t)n);
    const int64_t nrows = n < 7 ? n : 7;
    int64_t rows[7];
    for (int64_t j = 0; j < nrows; ++j) rows[j] = (j * 7919) % n;
    for (int lap = 0; lap <= 1; ++lap) {
        double *Z = xcalloc((size_t)(n * K), sizeof(double));
        double *Zr = xcalloc((size_t)(nrows * K), sizeof(double));
        snprintf(name, sizeof name, "%s.embed.lap%d", tag, lap);
        out(name, oracle_embed(n, s, src, dst, w, Y, K, lap, Z), Z, sizeof(double) * (size_t)(n * K));
        snprintf(name, sizeof name, "%s.rows.lap%d", tag, lap);
        out(name, oracle_embed_rows(n, s, src, dst, w, Y, K, lap, nrows, rows, Zr), Zr,
            sizeof(double) * (size_t)(nrows * K));
        free(Z);
        free(Zr);
    }
    free(cnt);
    free(inv);
    free(deg);
}

int main(void)
{
    /* Erdos-Renyi, weighted, uniform labels with exactly 5% unknown */
    {
        const int64_t n = 1000, s = 5000;
        const int32_t K = 7;
        int32_t *src = xcalloc(s, 4), *dst = xcalloc(s, 4), *Y = xcalloc(n, 4);
        float *w = xcalloc(s, 4);
        gen_er(n, s, 2, src, dst, w);
        out("gen.er.src", 0, src, 4 * s);
        out("gen.er.dst", 0, dst, 4 * s);
        out("gen.er.w", 0, w, 4 * s);
        gen_labels_uniform(n, K, 3, Y);
        out("gen.labels", gen_unlabel_exact(n, 50, 4, Y), Y, 4 * n);
        embed_all("er", n, s, src, dst, w, Y, K);
        embed_all("er_unit", n, s, src, dst, NULL, Y, K);
        gen_grid_weights(s, 5, w);
        out("gen.grid", 0, w, 4 * s);
        gen_shuffle_records(s, 6, src, dst, w);
        out("gen.shuffle", 0, src, 4 * s);
        embed_all("er_shuffled", n, s, src, dst, w, Y, K);
        /* errors: a label above K, a vertex id out of range, a negative Laplacian weight */
        int64_t cnt[8];
        double Z1[7000];
        memset(Z1, 0, sizeof Z1);
        Y[3] = K + 1;
        out("err.label", oracle_counts(n, Y, K, cnt), cnt, 0);
        Y[3] = 1;
        dst[11] = (int32_t)n;
        out("err.vertex", oracle_embed(n, s, src, dst, w, Y, K, 0, Z1), Z1, 0);
        dst[11] = 0;
        w[5] = -1.0f;
        out("err.negw", oracle_embed(n, s, src, dst, w, Y, K, 1, Z1), Z1, 0);
        int64_t bad_row = n;
        out("err.row", oracle_embed_rows(n, s, src, dst, NULL, Y, K, 0, 1, &bad_row, Z1), Z1, 0);
        out("err.n", oracle_embed(0, s, src, dst, NULL, Y, K, 0, Z1), Z1, 0);
        free(src);
        free(dst);
        free(Y);
        free(w);
    }
    /* R-MAT scale 10 (hubs and isolated vertices), Bernoulli unknown labels */
    {
        const int scale = 10;
        const int64_t n = 1 << scale, s = 8 * n;
        const int32_t K = 5;
        int32_t *src = xcalloc(s, 4), *dst = xcalloc(s, 4), *Y = xcalloc(n, 4);
        gen_rmat(scale, s, 0.57, 0.19, 0.19, 7, 1, src, dst);
        out("gen.rmat.src", 0, src, 4 * s);
        out("gen.rmat.dst", 0, dst, 4 * s);
        gen_labels_uniform(n, K, 8, Y);
        gen_unlabel_bernoulli(n, 0.3, 9, Y);
        out("gen.bern", 0, Y, 4 * n);
        embed_all("rmat", n, s, src, dst, NULL, Y, K);
        free(src);
        free(dst);
        free(Y);
    }
    /* SBM by pairs and by record sampling */
    {
        const int64_t n = 300, cap = 20000;
        const int32_t K = 3;
        int32_t *src = xcalloc(cap, 4), *dst = xcalloc(cap, 4), *Y = xcalloc(n, 4);
        const int64_t s = gen_sbm(n, 3, 0.2, 0.02, 10, cap, src, dst);
        out("gen.sbm", (long)s, src, 4 * (size_t)(s > 0 ? s : 0));
        out("gen.sbm.cap", (long)gen_sbm(n, 3, 0.9, 0.9, 10, 100, src, dst), src, 0);
        const int64_t s2 = gen_sbm(n, 3, 0.2, 0.02, 10, cap, src, dst);
        for (int64_t v = 0; v < n; ++v) Y[v] = (int32_t)(1 + (v * 3) / n);
        embed_all("sbm", n, s2, src, dst, NULL, Y, K);
        gen_sbm_records(n, 3, 0.8, 4000, 11, src, dst);
        out("gen.sbmr.src", 0, src, 4 * 4000);
        out("gen.sbmr.dst", 0, dst, 4 * 4000);
        free(src);
        free(dst);
        free(Y);
    }
    return 0;
}
