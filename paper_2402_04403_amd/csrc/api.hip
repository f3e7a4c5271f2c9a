// extern "C" entry points of libgee: argument checks, workspace layout and the
// stream-ordered launch sequence of each call. Declarations and contracts are in
// include/gee.h.

#include <limits.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "common.h"
#include "launch.h"

using namespace gee;

namespace {

constexpr int64_t kMaxN = INT32_MAX;
constexpr int64_t kMaxRecords = (int64_t)1 << 40;
constexpr int32_t kMaxK = 65535;
constexpr int32_t kMaxKPull = 4096;
constexpr int32_t kDefaultSegLen = 16384;

// Default segment length of the pull pass: one wavefront per segment, so a small graph
// needs shorter segments to give the GPU enough wavefronts. The power of two at or
// above (n + nnz) / 131072, in [1024, kDefaultSegLen]; it depends only on the graph.
int32_t pull_default_seg_len(int64_t n, int64_t nnz)
{
    const int64_t want = (n + nnz) / 131072;
    int64_t L = 1024;
    while (L < want && L < kDefaultSegLen) L *= 2;
    return (int32_t)L;
}

// Default segment length of the batched pass. Its lanes are vectors, so a wavefront
// walks its segment's entries one at a time: short segments give the GPU enough
// wavefronts (about 16K-32K of them up to graphs of 2^29 work items), at the price of
// more split rows. The power of two at or above (n + nnz) / 32768, in
// [512, kDefaultSegLen]; it depends only on the graph.
int32_t batch_default_seg_len(int64_t n, int64_t nnz)
{
    const int64_t want = (n + nnz) / 32768;
    int64_t L = 512;
    while (L < want && L < kDefaultSegLen) L *= 2;
    return (int32_t)L;
}
constexpr int32_t kMaxSegLen = 65535; // 16-bit per-segment class counters
constexpr size_t kWaveLdsBudget = 16384;
// Real-valued bins (weighted, Laplacian): about 8 KB a wavefront, so four workgroups of
// four wavefronts share a CU and their label gathers overlap.
constexpr size_t kWaveLdsBudgetReal = 8448;

inline bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

struct Plan {
    bool pull = false;
    int64_t n = 0, ns = 0, nnz = 0;
    int32_t K = 0;
    bool lap = false, weighted = false, wide = false, hot6 = false;
    Pack pack = Pack::U8;
    int64_t L = 0, nseg = 0;
    int rw = 0;
    // workspace offsets
    int64_t n_hot = 0;
    size_t o_counts = 0, o_inv = 0, o_lab = 0, o_deg = 0, o_hot = 0, o_segi = 0, o_sege = 0, o_part = 0, o_redo = 0,
           total = 0;
};

int check_coo(const gee_coo *g)
{
    if (!g) return GEE_EINVAL;
    if (g->n < 1 || g->n > kMaxN || g->s < 0) return GEE_EINVAL;
    if (g->s > kMaxRecords) return GEE_EOVERFLOW;
    if (g->s > 0 && (!g->src || !g->dst)) return GEE_EINVAL;
    return GEE_OK;
}

int check_csr(const gee_csr *c)
{
    if (!c) return GEE_EINVAL;
    if (c->n < 1 || c->n > kMaxN || c->nnz < 0 || !c->row_ptr) return GEE_EINVAL;
    if (c->nnz > 2 * kMaxRecords) return GEE_EOVERFLOW;
    if (c->nnz > 0 && !c->col) return GEE_EINVAL;
    if (c->n_hot < 0 || c->n_hot > c->n || (c->n_hot > 0 && !c->hot_ids)) return GEE_EINVAL;
    return GEE_OK;
}

int make_plan(const gee_coo *g, const gee_csr *csr, int32_t K, int laplacian, const gee_embed_opts *o, Plan *p)
{
    if (K < 1 || K > kMaxK) return GEE_EINVAL;
    Plan P;
    P.pull = csr != nullptr;
    P.K = K;
    P.lap = laplacian != 0;
    int rc;
    if (P.pull) {
        if ((rc = check_csr(csr)) != GEE_OK) return rc;
        if (g && g->n != csr->n) return GEE_EINVAL;
        if (K > kMaxKPull) return GEE_EINVAL;
        P.n = csr->n;
        P.nnz = csr->nnz;
        P.weighted = csr->val != nullptr;
        P.n_hot = csr->n_hot;
    } else {
        if ((rc = check_coo(g)) != GEE_OK) return rc;
        P.n = g->n;
        P.ns = g->s;
        P.weighted = g->w != nullptr;
    }
    P.pack = P.lap ? Pack::LAP64 : (K <= 255 ? Pack::U8 : Pack::U16);
    P.wide = P.lap || P.weighted;
    P.hot6 = P.pull && P.n_hot > 0 && !P.wide && P.pack == Pack::U8 && K <= 63;
    if (o) {
        if (o->seg_len != 0 && (o->seg_len < 64 || o->seg_len > kMaxSegLen)) return GEE_EINVAL;
        if (o->rows_per_window < 0 || o->rows_per_window > 64) return GEE_EINVAL;
    }
    if (P.pull) {
        P.L = (o && o->seg_len) ? o->seg_len : pull_default_seg_len(P.n, P.nnz);
        P.nseg = (P.n + P.nnz + P.L - 1) / P.L;
        if (o && o->rows_per_window) {
            P.rw = o->rows_per_window;
        } else {
            P.rw = 64;
            const size_t budget = P.wide ? kWaveLdsBudgetReal : kWaveLdsBudget;
            while (P.rw > 1 && pull_wave_bytes(K, P.wide, P.rw) > budget) --P.rw;
        }
        if (pull_wave_bytes(K, P.wide, P.rw) > 65536) return GEE_EINVAL;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align_up(off, 256);
        const size_t at = off;
        off += bytes;
        return at;
    };
    const size_t lab_bytes = P.pack == Pack::U8 ? 1 : (P.pack == Pack::U16 ? 2 : 8);
    P.o_counts = take(8 * (size_t)(K + 1));
    P.o_inv = take(8 * (size_t)(K + 1));
    P.o_lab = take(lab_bytes * (size_t)P.n + 4); // + one word: 32-bit reads of the last labels
    if (P.lap) P.o_deg = take(8 * (size_t)P.n);
    if (P.pull) {
        P.o_hot = take(P.hot6 ? 4 * (size_t)((P.n_hot + 4) / 5) : lab_bytes * (size_t)P.n_hot);
        P.o_segi = take(4 * (size_t)(P.nseg + 1));
        P.o_sege = take(8 * (size_t)(P.nseg + 1));
        P.o_part = take(8 * 2 * (size_t)P.nseg * (size_t)K);
        if (P.weighted && !P.lap) P.o_redo = take((size_t)P.nseg);
    }
    P.total = align_up(off, 256);
    *p = P;
    return GEE_OK;
}

inline int hip_rc(hipError_t e) { return e == hipSuccess ? GEE_OK : GEE_EHIP; }

constexpr int32_t kMaxBatch = 4096;
constexpr int32_t kMaxBatchK = kBatchMaxKT; // one vector's classes must fit one group

struct BatchPlan {
    int64_t n = 0, nnz = 0, L = 0, nseg = 0, n_hot = 0;
    bool any_lap = false, weighted = false;
    std::vector<GroupDesc> groups;
    std::vector<bool> lap;        // the group holds Laplacian vectors
    std::vector<int64_t> cnt_off; // per vector: offset of its K + 1 class counts
    int64_t cnt_total = 0;
    int Gs_max = 0, KT_max = 0;
    size_t o_cnt = 0, o_lab = 0, o_labhot = 0, o_rsdhot = 0, o_cscale = 0, o_vmeta = 0,
           o_segi = 0, o_sege = 0, o_part = 0, o_deg = 0, o_rsd = 0, total = 0;
};

int make_batch_plan(const gee_csr *csr, const gee_batch *bt, const gee_embed_opts *o, BatchPlan *out)
{
    int rc;
    if ((rc = check_csr(csr)) != GEE_OK) return rc;
    if (!bt || bt->B < 1 || bt->B > kMaxBatch || !bt->K || !bt->laplacian || !bt->zoff || bt->ldz < 1)
        return GEE_EINVAL;
    if (o && o->seg_len != 0 && (o->seg_len < 64 || o->seg_len > kMaxSegLen)) return GEE_EINVAL;
    if (o && (o->group_vectors < 0 || o->group_vectors > kGroupMax)) return GEE_EINVAL;
    const int gmax = (o && o->group_vectors) ? o->group_vectors : kGroupMax;
    if (bt->ldz > INT32_MAX) return GEE_EINVAL; // Z column ids are 32-bit in the edge pass
    BatchPlan P;
    P.n = csr->n;
    P.nnz = csr->nnz;
    P.n_hot = csr->n_hot;
    P.weighted = csr->val != nullptr;
    if (bt->ldz > ((int64_t)1 << 62) / P.n) return GEE_EOVERFLOW;
    const int B = bt->B;
    for (int b = 0; b < B; ++b) {
        if (bt->K[b] < 1 || bt->K[b] > kMaxBatchK || bt->zoff[b] < 0 || bt->zoff[b] + bt->K[b] > bt->ldz)
            return GEE_EINVAL;
        P.any_lap |= bt->laplacian[b] != 0;
    }
    // vectors in column order; blocks must not overlap
    std::vector<int> ord(B);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return bt->zoff[a] < bt->zoff[c]; });
    for (int i = 1; i < B; ++i)
        if (bt->zoff[ord[i]] < bt->zoff[ord[i - 1]] + bt->K[ord[i - 1]]) return GEE_EINVAL;
    P.cnt_off.resize(B);
    for (int b = 0; b < B; ++b) {
        P.cnt_off[b] = P.cnt_total;
        P.cnt_total += bt->K[b] + 1;
    }
    // groups: runs of vectors whose blocks are contiguous in Z (in column order), up
    // to 64 vectors and kBatchMaxKT classes per group, any mix of versions
    for (int i = 0; i < B;) {
        GroupDesc d{};
        bool lap = false;
        while (i < B && d.G < gmax) {
            const int b = ord[i];
            if (d.G > 0 && (d.KT + bt->K[b] > kBatchMaxKT || bt->zoff[b] != d.zoff[0] + d.KT)) break;
            d.vec[d.G] = b;
            d.K[d.G] = bt->K[b];
            d.coff[d.G] = d.KT;
            d.zoff[d.G] = bt->zoff[b];
            d.inv_off[d.G] = P.cnt_off[b];
            d.lap[d.G] = bt->laplacian[b] != 0;
            lap |= bt->laplacian[b] != 0;
            d.KT += bt->K[b];
            ++d.G;
            ++i;
        }
        // label row stride: G rounded up to 8, with at least one zero padding column when
        // G < 64 (lanes without a vector read it)
        d.Gs = std::min(kGroupMax, (d.G + 1 + 7) / 8 * 8);
        P.groups.push_back(d);
        P.lap.push_back(lap);
        P.Gs_max = std::max(P.Gs_max, d.Gs);
        P.KT_max = std::max(P.KT_max, d.KT);
    }
    P.L = (o && o->seg_len) ? o->seg_len : batch_default_seg_len(P.n, P.nnz);
    P.nseg = (P.n + P.nnz + P.L - 1) / P.L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align_up(off, 256);
        const size_t at = off;
        off += bytes;
        return at;
    };
    P.o_cnt = take(8 * (size_t)P.cnt_total);
    P.o_lab = take(2 * (size_t)(P.n + 1) * (size_t)P.Gs_max);
    P.o_labhot = take(2 * (size_t)P.n_hot * (size_t)P.Gs_max);
    P.o_cscale = take(8 * (size_t)P.KT_max);
    P.o_vmeta = take(4 * (size_t)kGroupMax);
    P.o_segi = take(4 * (size_t)(P.nseg + 1));
    P.o_sege = take(8 * (size_t)(P.nseg + 1));
    P.o_part = take(8 * 2 * (size_t)P.nseg * (size_t)P.KT_max);
    if (P.any_lap) {
        P.o_deg = take(8 * (size_t)P.n);
        P.o_rsd = take(4 * (size_t)P.n);
        P.o_rsdhot = take(4 * (size_t)P.n_hot);
    }
    P.total = align_up(off, 256);
    *out = std::move(P);
    return GEE_OK;
}

} // namespace

extern "C" {

const char *gee_strerror(int code)
{
    switch (code) {
    case GEE_OK: return "success";
    case GEE_EINVAL: return "invalid argument";
    case GEE_ELABEL: return "label outside [0, K]";
    case GEE_EVERTEX: return "vertex id outside [0, n)";
    case GEE_ENEGW: return "negative or NaN weight in the Laplacian version";
    case GEE_EOVERFLOW: return "size outside the supported range";
    case GEE_EWORKSPACE: return "workspace missing, misaligned or too small";
    case GEE_EHIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

int gee_counts(const int32_t *labels, int64_t n, int32_t K, int64_t *counts, int32_t *err, hipStream_t stream)
{
    if (!labels || !counts || n < 1 || n > kMaxN || K < 1 || K > kMaxK) return GEE_EINVAL;
    return hip_rc(launch_counts(labels, n, K, reinterpret_cast<uint64_t *>(counts), nullptr, Pack::U8, err, stream));
}

int gee_weights(const int64_t *counts, int32_t K, double *inv, hipStream_t stream)
{
    if (!counts || !inv || K < 1 || K > kMaxK) return GEE_EINVAL;
    return hip_rc(launch_weights(reinterpret_cast<const uint64_t *>(counts), K, inv, stream));
}

int gee_degrees(const gee_coo *g, const gee_csr *csr, double *deg, int32_t *err, hipStream_t stream)
{
    if (!deg) return GEE_EINVAL;
    int rc;
    if (csr) {
        if ((rc = check_csr(csr)) != GEE_OK) return rc;
        if (g && g->n != csr->n) return GEE_EINVAL;
        return hip_rc(launch_degrees_csr(csr->n, csr->row_ptr, csr->val, csr->nnz, deg, false, err, stream));
    }
    if ((rc = check_coo(g)) != GEE_OK) return rc;
    return hip_rc(launch_degrees_coo(g->n, g->s, g->src, g->dst, g->w, deg, false, err, stream));
}

size_t gee_embed_workspace(const gee_coo *g, const gee_csr *csr, int32_t K, int laplacian,
                           const gee_embed_opts *opts)
{
    Plan p;
    if (make_plan(g, csr, K, laplacian, opts, &p) != GEE_OK) return 0;
    return p.total;
}

} // extern "C"

namespace {

int embed_impl(const gee_coo *g, const gee_csr *csr, const int32_t *labels, int32_t K, int laplacian, float *Z,
               void *ws, size_t ws_bytes, int32_t *err, const gee_embed_opts *opts, hipStream_t stream,
               bool atomic_updates)
{
    Plan p;
    int rc = make_plan(g, csr, K, laplacian, opts, &p);
    if (rc != GEE_OK) return rc;
    if (!labels || !Z) return GEE_EINVAL;
    if (!ws || !aligned(ws, 256) || ws_bytes < p.total) return GEE_EWORKSPACE;
    char *w = static_cast<char *>(ws);

    EmbedArgs a;
    a.n = p.n;
    a.K = K;
    a.laplacian = p.lap;
    a.weighted = p.weighted;
    a.pack = p.pack;
    a.hot6 = p.hot6;
    a.atomic_updates = atomic_updates;
    a.labels = labels;
    a.err = err;
    a.counts = reinterpret_cast<uint64_t *>(w + p.o_counts);
    a.inv = reinterpret_cast<double *>(w + p.o_inv);
    a.lab = w + p.o_lab;
    a.deg = p.lap ? reinterpret_cast<double *>(w + p.o_deg) : nullptr;
    a.Z = Z;

    // class counts (+ packed labels for the adjacency version), then W
    if ((rc = hip_rc(launch_counts(labels, p.n, K, a.counts, p.lap ? nullptr : a.lab, p.pack, err, stream))))
        return rc;
    if ((rc = hip_rc(launch_weights(a.counts, K, a.inv, stream)))) return rc;
    if (p.lap) {
        hipError_t e = p.pull ? launch_degrees_csr(p.n, csr->row_ptr, csr->val, p.nnz, a.deg, true, err, stream)
                              : launch_degrees_coo(p.n, p.ns, g->src, g->dst, g->w, a.deg, true, err, stream);
        if ((rc = hip_rc(e))) return rc;
        if ((rc = hip_rc(launch_pack_lap(labels, p.n, K, a.deg, static_cast<uint64_t *>(a.lab), stream)))) return rc;
    }
    if (p.pull && p.n_hot > 0 &&
        (rc = hip_rc(launch_pack_hot(a, csr->hot_ids, p.n_hot, w + p.o_hot, stream))))
        return rc;
    const bool timed = opts && opts->hot_begin && opts->hot_end;
    if (!p.pull) {
        if ((rc = hip_rc(launch_fill_f32(Z, p.n * K, 0.0f, stream)))) return rc;
        if (timed && (rc = hip_rc(hipEventRecord(opts->hot_begin, stream)))) return rc;
        if ((rc = hip_rc(launch_push(a, p.ns, g->src, g->dst, g->w, stream)))) return rc;
        if (timed && (rc = hip_rc(hipEventRecord(opts->hot_end, stream)))) return rc;
        return hip_rc(launch_scale(a, stream));
    }
    int32_t *seg_i = reinterpret_cast<int32_t *>(w + p.o_segi);
    int64_t *seg_e = reinterpret_cast<int64_t *>(w + p.o_sege);
    double *part = reinterpret_cast<double *>(w + p.o_part);
    if ((rc = hip_rc(launch_seg_bounds(p.n, p.nnz, csr->row_ptr, p.L, p.nseg, seg_i, seg_e, stream)))) return rc;
    if (timed && (rc = hip_rc(hipEventRecord(opts->hot_begin, stream)))) return rc;
    uint8_t *redo = (p.weighted && !p.lap) ? reinterpret_cast<uint8_t *>(w + p.o_redo) : nullptr;
    if ((rc = hip_rc(launch_pull(a, p.nnz, csr->row_ptr, csr->col, csr->val, w + p.o_hot, p.n_hot, seg_i, seg_e,
                                 p.nseg, p.rw, part, redo, stream))))
        return rc;
    if (timed && (rc = hip_rc(hipEventRecord(opts->hot_end, stream)))) return rc;
    return hip_rc(launch_merge(a, csr->row_ptr, seg_i, seg_e, p.nseg, part, stream));
}

} // namespace

extern "C" {

int gee_embed(const gee_coo *g, const gee_csr *csr, const int32_t *labels, int32_t K, int laplacian, float *Z,
              void *ws, size_t ws_bytes, int32_t *err, const gee_embed_opts *opts, hipStream_t stream)
{
    return embed_impl(g, csr, labels, K, laplacian, Z, ws, ws_bytes, err, opts, stream, true);
}

} // extern "C"

namespace {

// Scratch of gee_embed_noalloc: one static array per GPU, which the code object brings
// with it when the library is loaded on that device. Host code never passes the
// array's name to a kernel (on the host it names a host-side stand-in): the device
// address is looked up once per device with hipGetSymbolAddress and kept.
__device__ __align__(256) unsigned char scratch[GEE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices];

// Device address of the current device's scratch (looked up on the first call there).
int current_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GEE_EHIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GEE_EHIP;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return GEE_OK;
}

} // namespace

extern "C" {

int gee_embed_noalloc(const gee_coo *g, const gee_csr *csr, const int32_t *labels, int32_t K, int laplacian,
                      float *Z, int32_t *err, const gee_embed_opts *opts, hipStream_t stream)
{
    Plan p;
    int rc = make_plan(g, csr, K, laplacian, opts, &p);
    if (rc != GEE_OK) return rc;
    if (p.total > (size_t)GEE_NOALLOC_SCRATCH_BYTES) return GEE_EWORKSPACE;
    void *ws = nullptr;
    if ((rc = current_scratch(&ws)) != GEE_OK) return rc;
    return embed_impl(g, csr, labels, K, laplacian, Z, ws, (size_t)GEE_NOALLOC_SCRATCH_BYTES, err, opts, stream,
                      true);
}

int gee_embed_push_nonatomic(const gee_coo *g, const int32_t *labels, int32_t K, int laplacian, float *Z, void *ws,
                             size_t ws_bytes, int32_t *err, const gee_embed_opts *opts, hipStream_t stream)
{
    if (!g) return GEE_EINVAL;
    return embed_impl(g, nullptr, labels, K, laplacian, Z, ws, ws_bytes, err, opts, stream, false);
}

size_t gee_embed_batch_workspace(const gee_csr *csr, const gee_batch *batch, const gee_embed_opts *opts)
{
    BatchPlan p;
    if (make_batch_plan(csr, batch, opts, &p) != GEE_OK) return 0;
    return p.total;
}

int gee_embed_batch(const gee_csr *csr, const gee_batch *batch, void *ws, size_t ws_bytes, int32_t *err,
                    const gee_embed_opts *opts, hipStream_t stream)
{
    BatchPlan p;
    int rc = make_batch_plan(csr, batch, opts, &p);
    if (rc != GEE_OK) return rc;
    if (!batch->labels || !batch->Z) return GEE_EINVAL;
    if (!ws || !aligned(ws, 256) || ws_bytes < p.total) return GEE_EWORKSPACE;
    char *w = static_cast<char *>(ws);
    uint64_t *cnt = reinterpret_cast<uint64_t *>(w + p.o_cnt);
    int32_t *seg_i = reinterpret_cast<int32_t *>(w + p.o_segi);
    int64_t *seg_e = reinterpret_cast<int64_t *>(w + p.o_sege);
    float *rsd = p.any_lap ? reinterpret_cast<float *>(w + p.o_rsd) : nullptr;

    // class counts of every vector, one launch per group (the weights 1 / n_k are taken
    // from them where each group's column scales are built)
    if ((rc = hip_rc(launch_fill_u64(cnt, p.cnt_total, 0, stream)))) return rc;
    for (const GroupDesc &d : p.groups)
        if ((rc = hip_rc(launch_counts_group(batch->labels, p.n, d, cnt, err, stream)))) return rc;
    // one degree pass shared by the Laplacian vectors
    if (p.any_lap) {
        double *deg = reinterpret_cast<double *>(w + p.o_deg);
        if ((rc = hip_rc(launch_degrees_csr(p.n, csr->row_ptr, csr->val, p.nnz, deg, true, err, stream)))) return rc;
        if ((rc = hip_rc(launch_rsd(deg, p.n, rsd, stream)))) return rc;
    }
    if ((rc = hip_rc(launch_seg_bounds(p.n, p.nnz, csr->row_ptr, p.L, p.nseg, seg_i, seg_e, stream)))) return rc;
    const bool timed = opts && opts->hot_begin && opts->hot_end;
    if (timed && (rc = hip_rc(hipEventRecord(opts->hot_begin, stream)))) return rc;
    void *labmat = w + p.o_lab;    // sized for 16-bit labels; 8-bit groups use half
    void *labhot = w + p.o_labhot;
    float *rsdhot = p.any_lap ? reinterpret_cast<float *>(w + p.o_rsdhot) : nullptr;
    double *cscale = reinterpret_cast<double *>(w + p.o_cscale);
    uint32_t *vmeta = reinterpret_cast<uint32_t *>(w + p.o_vmeta);
    for (size_t gi = 0; gi < p.groups.size(); ++gi) {
        const GroupDesc &d = p.groups[gi];
        GroupArgs g;
        g.n = p.n;
        g.row_ptr = csr->row_ptr;
        g.col = csr->col;
        g.val = csr->val;
        g.n_hot = p.n_hot;
        g.labmat = labmat;
        g.labhot = labhot;
        int32_t kmax = 0;
        for (int i = 0; i < d.G; ++i) kmax = d.K[i] > kmax ? d.K[i] : kmax;
        g.u8 = kmax <= 255; // 8-bit label rows: half the bytes per gathered row
        g.Gs = d.Gs;
        g.KT = d.KT;
        g.lap = p.lap[gi];
        g.rsd = g.lap ? rsd : nullptr;
        g.rsdhot = g.lap ? rsdhot : nullptr;
        g.vmeta = vmeta;
        g.cscale = cscale;
        g.seg_i = seg_i;
        g.seg_e = seg_e;
        g.nseg = p.nseg;
        g.Z = batch->Z;
        g.ldz = batch->ldz;
        g.zcol = d.zoff[0];
        g.part = reinterpret_cast<double *>(w + p.o_part);
        g.err = err;
        if ((rc = hip_rc(launch_pack_group(batch->labels, p.n, d, labmat, g.u8, err, stream)))) return rc;
        if ((rc = hip_rc(launch_pack_group_hot(csr->hot_ids, p.n_hot, p.n, d.Gs * (g.u8 ? 1 : 2), labmat, labhot,
                                               g.rsd, g.lap ? rsdhot : nullptr, err, stream))))
            return rc;
        if ((rc = hip_rc(launch_group_cols(cnt, d, cscale, vmeta, stream)))) return rc;
        if ((rc = hip_rc(launch_pull_group(g, stream)))) return rc;
    }
    if (timed && (rc = hip_rc(hipEventRecord(opts->hot_end, stream)))) return rc;
    return GEE_OK;
}

int64_t gee_pb_cells(int64_t n, int64_t n_lds)
{
    if (n < 1 || n > kMaxN || n_lds < 0 || n_lds > kPbMaxSlices * kPbSlice) return 0;
    return pb_layout(n, n_lds).cells;
}

int64_t gee_pb_tier_slots(const gee_csr *csr, int64_t min_per_row_block, void *ws, size_t ws_bytes,
                          hipStream_t stream)
{
    int rc;
    if ((rc = check_csr(csr)) != GEE_OK) return rc;
    if (min_per_row_block < 0) return GEE_EINVAL;
    const int64_t cap = csr->hot_ids ? (csr->n_hot < kPbMaxSlices * kPbSlice ? csr->n_hot : kPbMaxSlices * kPbSlice) : 0;
    if (cap == 0) return 0;
    if (!ws || !aligned(ws, 256) || ws_bytes < (size_t)kPbMaxSlices * 8) return GEE_EWORKSPACE;
    int64_t *dev = static_cast<int64_t *>(ws);
    int64_t host[kPbMaxSlices] = {};
    const int64_t n_sl = (cap + kPbSlice - 1) >> kPbSliceBits;
    if ((rc = hip_rc(launch_pb_slice_entries(cap, csr->hot_ids, csr->row_ptr, dev, stream)))) return rc;
    if ((rc = hip_rc(hipMemcpyAsync(host, dev, (size_t)n_sl * 8, hipMemcpyDeviceToHost, stream)))) return rc;
    if ((rc = hip_rc(hipStreamSynchronize(stream)))) return rc;
    const int64_t need = min_per_row_block * ((csr->n + 255) / 256);
    int64_t slices = 0;
    while (slices < n_sl && host[slices] >= need) ++slices;
    return slices == n_sl ? cap : slices * kPbSlice;
}

size_t gee_pb_build_workspace(const gee_csr *csr, int64_t n_lds, int laplacian)
{
    if (check_csr(csr) != GEE_OK || csr->nnz > kPbMaxNnz) return 0;
    if (n_lds < 0 || n_lds > (csr->hot_ids ? csr->n_hot : 0) || n_lds > kPbMaxSlices * kPbSlice) return 0;
    return pb_build_scratch(csr->n, csr->nnz, n_lds, csr->val != nullptr, laplacian != 0);
}

int gee_pb_build(const gee_csr *csr, int64_t n_lds, int laplacian, int32_t *col, uint8_t *ul, int64_t *cell_start,
                 uint32_t *cell_count, uint32_t *cell_word, int32_t *lds_ids, float *val, uint8_t *rb_flag,
                 float *rsd, int64_t *meta, void *ws, size_t ws_bytes, int32_t *err, hipStream_t stream)
{
    int rc;
    if ((rc = check_csr(csr)) != GEE_OK) return rc;
    if (csr->nnz > kPbMaxNnz) return GEE_EOVERFLOW;
    if (n_lds < 0 || n_lds > (csr->hot_ids ? csr->n_hot : 0) || n_lds > kPbMaxSlices * kPbSlice) return GEE_EINVAL;
    if ((csr->nnz > 0 && (!col || !ul)) || !cell_start || !cell_count || !cell_word || !meta || !aligned(col, 16) ||
        !aligned(ul, 16) || (n_lds > 0 && !lds_ids))
        return GEE_EINVAL;
    const bool lap = laplacian != 0;
    const bool carried = csr->val != nullptr || lap; // a value per entry in the layout
    if (carried ? (!rb_flag || (csr->nnz > 0 && !val) || !aligned(val, 16)) : (val || rb_flag)) return GEE_EINVAL;
    if (lap ? !rsd : rsd != nullptr) return GEE_EINVAL;
    const size_t need = pb_build_scratch(csr->n, csr->nnz, n_lds, csr->val != nullptr, lap);
    if (!ws || !aligned(ws, 256) || ws_bytes < need) return GEE_EWORKSPACE;
    return hip_rc(launch_pb_build(csr->n, csr->nnz, csr->row_ptr, csr->col, csr->val, lap, csr->hot_ids, csr->n_hot,
                                  n_lds, col, ul, cell_start, cell_count, cell_word, lds_ids, val, rb_flag, rsd, meta,
                                  ws, err, stream));
}

} // extern "C"

namespace {

int check_pb(const gee_pb *pb)
{
    if (!pb || pb->n < 1 || pb->n > kMaxN || pb->nnz < 0) return GEE_EINVAL;
    if (pb->nnz > kPbMaxNnz) return GEE_EOVERFLOW;
    if (pb->n_lds < 0 || pb->n_lds > kPbMaxSlices * kPbSlice || (pb->n_lds > 0 && !pb->lds_ids)) return GEE_EINVAL;
    const PbLayout L = pb_layout(pb->n, pb->n_lds);
    if (pb->n_rb != L.n_rb || pb->n_cb != L.n_cb) return GEE_EINVAL;
    if ((pb->nnz > 0 && (!pb->col || !pb->ul)) || !pb->cell_start || !pb->cell_count || !pb->cell_word ||
        !pb->meta || !aligned(pb->col, 16) || !aligned(pb->ul, 16))
        return GEE_EINVAL;
    if ((pb->val == nullptr) != (pb->rb_flag == nullptr) || !aligned(pb->val, 16) || (pb->rsd && !pb->val))
        return GEE_EINVAL;
    return GEE_OK;
}

struct PbPlan {
    size_t o_counts = 0, o_inv = 0, o_lab = 0, o_tab = 0, o_yv = 0, total = 0;
};

PbPlan pb_plan(const gee_pb *pb, int32_t K)
{
    PbPlan P;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align_up(off, 256);
        const size_t at = off;
        off += bytes;
        return at;
    };
    P.o_counts = take(8 * (size_t)(K + 1));
    P.o_inv = take(8 * (size_t)(K + 1));
    P.o_lab = take((size_t)pb->n);
    P.o_tab = take(align_up((size_t)pb->n_lds, 16));
    P.o_yv = take((size_t)pb->nnz + 48); // the gap before the tier and word reads past the end
    P.total = align_up(off, 256);
    return P;
}

} // namespace

extern "C" {

size_t gee_embed_pb_workspace(const gee_pb *pb, int32_t K)
{
    if (check_pb(pb) != GEE_OK || K < 1 || K > kPbMaxK) return 0;
    return pb_plan(pb, K).total;
}

int gee_embed_pb(const gee_pb *pb, const int32_t *labels, int32_t K, float *Z, void *ws, size_t ws_bytes,
                 int32_t *err, const gee_embed_opts *opts, hipStream_t stream)
{
    int rc;
    if ((rc = check_pb(pb)) != GEE_OK) return rc;
    if (K < 1 || K > kPbMaxK || !labels || !Z) return GEE_EINVAL;
    const PbPlan p = pb_plan(pb, K);
    if (!ws || !aligned(ws, 256) || ws_bytes < p.total) return GEE_EWORKSPACE;
    char *w = static_cast<char *>(ws);
    uint64_t *counts = reinterpret_cast<uint64_t *>(w + p.o_counts);
    double *inv = reinterpret_cast<double *>(w + p.o_inv);
    uint8_t *lab = reinterpret_cast<uint8_t *>(w + p.o_lab);
    uint8_t *tab = reinterpret_cast<uint8_t *>(w + p.o_tab);
    uint8_t *yv = reinterpret_cast<uint8_t *>(w + p.o_yv);
    if ((rc = hip_rc(launch_counts(labels, pb->n, K, counts, lab, Pack::U8, err, stream)))) return rc;
    if ((rc = hip_rc(launch_weights(counts, K, inv, stream)))) return rc;
    const bool timed = opts && opts->hot_begin && opts->hot_end;
    if (timed && (rc = hip_rc(hipEventRecord(opts->hot_begin, stream)))) return rc;
    const PbLayout L = pb_layout(pb->n, pb->n_lds);
    const int kind = pb->rsd ? 2 : (pb->val ? 1 : 0);
    if ((rc = hip_rc(launch_pb_gather(pb->n, pb->nnz, L, pb->n_lds, pb->cell_start, pb->cell_count, pb->col,
                                      pb->lds_ids, pb->meta, kind, lab, tab, yv, err, stream))))
        return rc;
    if ((rc = hip_rc(launch_pb_rows(pb->n, pb->nnz, K, L, pb->cell_start, pb->cell_count, pb->cell_word, pb->ul, yv,
                                    pb->val, pb->rb_flag, pb->rsd, pb->meta, pb->n_lds, inv, Z, err, stream))))
        return rc;
    if (timed && (rc = hip_rc(hipEventRecord(opts->hot_end, stream)))) return rc;
    return GEE_OK;
}

size_t gee_csr_workspace(int64_t n, int64_t s, int weighted, int64_t hot_budget)
{
    if (n < 1 || n > kMaxN || s < 0 || s > kMaxRecords || hot_budget < 0) return 0;
    return csr_build_layout(n, s, weighted != 0, hot_budget < n ? hot_budget : n, nullptr, nullptr);
}

int gee_csr_build(const gee_coo *g, int64_t hot_budget, int64_t *row_ptr, int32_t *col, float *val,
                  int32_t *hot_ids, void *ws, size_t ws_bytes, int32_t *err, hipStream_t stream)
{
    int rc = check_coo(g);
    if (rc != GEE_OK) return rc;
    if (hot_budget < 0) return GEE_EINVAL;
    const int64_t n_hot = hot_budget < g->n ? hot_budget : g->n;
    if (!row_ptr || (g->s > 0 && !col) || (g->w && g->s > 0 && !val) || (n_hot > 0 && !hot_ids)) return GEE_EINVAL;
    const size_t need = csr_build_layout(g->n, g->s, g->w != nullptr, n_hot, nullptr, nullptr);
    if (!ws || !aligned(ws, 256) || ws_bytes < need) return GEE_EWORKSPACE;
    CsrBuildWs w;
    csr_build_layout(g->n, g->s, g->w != nullptr, n_hot, static_cast<char *>(ws), &w);
    return hip_rc(
        launch_csr_build(g->n, g->s, g->src, g->dst, g->w, n_hot, row_ptr, col, val, hot_ids, w, err, stream));
}

int gee_argmax(const float *Z, int64_t n, int32_t K, int64_t ldz, const int32_t *prev, int32_t *labels,
               uint64_t *changed, hipStream_t stream)
{
    if (!Z || !labels || n < 1 || n > kMaxN || K < 1 || K > kMaxK || ldz < K) return GEE_EINVAL;
    if (prev == labels) return GEE_EINVAL;
    if ((uint64_t)n > (uint64_t)INT64_MAX / (uint64_t)ldz) return GEE_EOVERFLOW;
    return hip_rc(launch_argmax(n, K, ldz, Z, prev, labels, prev ? changed : nullptr, stream));
}

int gee_embed_batch_tune(const gee_csr *csr, const gee_batch *batch, const int32_t *seg_lens, int n_seg,
                         const int32_t *group_vectors, int n_group, int reps, void *ws, size_t ws_bytes, int32_t *err,
                         hipStream_t stream, int32_t *best_seg, int32_t *best_group, float *best_ms)
{
    if (!seg_lens || n_seg < 1 || reps < 1 || !best_seg || !best_group || !best_ms) return GEE_EINVAL;
    if (n_group < 0 || (n_group > 0 && !group_vectors)) return GEE_EINVAL;
    for (int i = 0; i < n_seg; ++i)
        if (seg_lens[i] < 0 || seg_lens[i] % 64 != 0 || seg_lens[i] > (1 << 22)) return GEE_EINVAL;
    for (int i = 0; i < n_group; ++i)
        if (group_vectors[i] < 0 || group_vectors[i] > kGroupMax) return GEE_EINVAL;
    const int32_t default_group = 0;
    const int32_t *groups = n_group > 0 ? group_vectors : &default_group;
    const int ng = n_group > 0 ? n_group : 1;
    int rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((rc = hip_rc(hipEventCreate(&e0)))) return rc;
    if ((rc = hip_rc(hipEventCreate(&e1)))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    float best_t = 0.f;
    int32_t best_l = -1, best_g = -1;
    for (int gi = 0; gi < ng && rc == GEE_OK; ++gi) {
        for (int i = 0; i < n_seg && rc == GEE_OK; ++i) {
            gee_embed_opts o = {};
            o.seg_len = seg_lens[i];
            o.group_vectors = groups[gi];
            if ((rc = gee_embed_batch(csr, batch, ws, ws_bytes, err, &o, stream))) break;
            if ((rc = hip_rc(hipEventRecord(e0, stream)))) break;
            for (int r = 0; r < reps && rc == GEE_OK; ++r)
                rc = gee_embed_batch(csr, batch, ws, ws_bytes, err, &o, stream);
            if (rc || (rc = hip_rc(hipEventRecord(e1, stream))) || (rc = hip_rc(hipEventSynchronize(e1)))) break;
            float ms = 0.f;
            if ((rc = hip_rc(hipEventElapsedTime(&ms, e0, e1)))) break;
            ms /= (float)reps;
            if (best_l < 0 || ms < best_t) {
                best_t = ms;
                best_l = seg_lens[i];
                best_g = groups[gi];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best_seg = best_l;
    *best_group = best_g;
    *best_ms = best_t;
    return GEE_OK;
}

} // extern "C"

struct gee_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

int gee_capture_begin(hipStream_t stream)
{
    if (!stream) return GEE_EINVAL;
    return hip_rc(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
}

int gee_capture_end(hipStream_t stream, gee_graph **graph)
{
    if (!stream || !graph) return GEE_EINVAL;
    *graph = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_rc(e);
    }
    hipGraphExec_t x = nullptr;
    if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_rc(e);
    }
    gee_graph *r = new (std::nothrow) gee_graph{g, x};
    if (!r) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return GEE_EHIP;
    }
    *graph = r;
    return GEE_OK;
}

int gee_graph_launch(const gee_graph *graph, hipStream_t stream)
{
    if (!graph) return GEE_EINVAL;
    return hip_rc(hipGraphLaunch(graph->exec, stream));
}

void gee_graph_destroy(gee_graph *graph)
{
    if (!graph) return;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
}

int gee_copy(void *dst, const void *src, size_t bytes, hipStream_t stream)
{
    if (!dst || !src || bytes % 16 || !aligned(dst, 16) || !aligned(src, 16)) return GEE_EINVAL;
    return hip_rc(launch_copy(dst, src, bytes, stream));
}

} // extern "C"
