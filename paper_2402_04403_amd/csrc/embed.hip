// GEE kernels for gfx950: class counts, projection weights, degrees, the
// edge-parallel push pass and the CSR-pull pass with its split-row merge.
//
// Algorithm 1 (Section II of the paper) builds W from the class counts and then
// adds W(v, Y(v)) * w into Z(u, Y(v)) and W(u, Y(u)) * w into Z(v, Y(u)) for every
// record. Here W is never materialised: W(v, k) = [Y(v) = k] * inv[k]. Both
// factors that are constant per output element, inv[k] and (Laplacian) the row's
// own d_u^-1/2, are taken out of the sums and applied once when a row is
// written; the sums themselves add raw weights (times d_v^-1/2 for the
// Laplacian). Unit-weight adjacency sums are therefore exact integers.

#include "common.h"
#include "launch.h"

namespace gee {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

inline int grid_for(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

template <typename T> __global__ void k_fill(T *__restrict__ p, int64_t count, T value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ------------------------------------------------------------------ counts --

constexpr int kHistBins = 4096;

// counts[k] += #{v : labels[v] = k}; invalid labels raise GEE_ELABEL, are not
// counted and pack as 0 (unknown). Block-private LDS histogram when K+1 fits.
template <typename P>
__global__ void __launch_bounds__(kBlock)
k_counts(const int32_t *__restrict__ labels, int64_t n, int32_t K, uint64_t *__restrict__ counts,
         P *__restrict__ packed, int32_t *err)
{
    __shared__ uint32_t hist[kHistBins];
    const bool lds = (K + 1) <= kHistBins;
    if (lds)
        for (int b = threadIdx.x; b <= K; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    bool bad = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t y = labels[v];
        const bool ok = (uint32_t)y <= (uint32_t)K;
        bad |= !ok;
        if (ok) {
            if (lds) atomicAdd(&hist[y], 1u);
            else atomicAdd((unsigned long long *)&counts[y], 1ull);
        }
        if (packed) packed[v] = (P)(ok ? y : 0);
    }
    if (bad) flag_error(err, GEE_ELABEL);
    __syncthreads();
    if (lds)
        for (int b = threadIdx.x; b <= K; b += blockDim.x)
            if (hist[b]) atomicAdd((unsigned long long *)&counts[b], (unsigned long long)hist[b]);
}

// inv[0] = 0; inv[k] = 1 / n_k (IEEE division), 0 for an empty class.
__global__ void k_weights(const uint64_t *__restrict__ counts, int32_t K, double *__restrict__ inv)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    const uint64_t c = counts[k];
    inv[k] = (k == 0 || c == 0) ? 0.0 : 1.0 / (double)c;
}

// ----------------------------------------------------------------- degrees --

template <bool W>
__global__ void __launch_bounds__(kBlock)
k_degrees_coo(int64_t n, int64_t ns, const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
              const float *__restrict__ w, double *__restrict__ deg, bool check_neg, int32_t *err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[i], v = dst[i];
        if ((uint32_t)u >= (uint64_t)n || (uint32_t)v >= (uint64_t)n) {
            flag_error(err, GEE_EVERTEX);
            continue;
        }
        const float x = W ? w[i] : 1.0f;
        if (W && check_neg && !(x >= 0.0f)) {
            flag_error(err, GEE_ENEGW);
            continue;
        }
        atomicAdd(&deg[u], (double)x);
        atomicAdd(&deg[v], (double)x);
    }
}

// One thread per row: sum the row's stored weights in order (deterministic).
template <bool W>
__global__ void __launch_bounds__(kBlock)
k_degrees_csr(int64_t n, const int64_t *__restrict__ row_ptr, const float *__restrict__ val, int64_t nnz,
              double *__restrict__ deg, bool check_neg, int32_t *err)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = row_ptr[u], e = row_ptr[u + 1];
        b = b < 0 ? 0 : (b > nnz ? nnz : b);
        e = e < b ? b : (e > nnz ? nnz : e);
        if (!W) {
            deg[u] = (double)(e - b);
            continue;
        }
        double d = 0.0;
        bool neg = false;
        for (int64_t j = b; j < e; ++j) {
            const float x = val[j];
            neg |= !(x >= 0.0f);
            d += (double)x;
        }
        if (check_neg && neg) flag_error(err, GEE_ENEGW);
        deg[u] = d;
    }
}

// Laplacian label records: class in the low word, d^-1/2 rounded to FP32 in the
// high word (0 for an isolated vertex).
__global__ void __launch_bounds__(kBlock)
k_pack_lap(const int32_t *__restrict__ labels, int64_t n, int32_t K, const double *__restrict__ deg,
           uint64_t *__restrict__ lab)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t y = labels[v];
        const uint32_t cls = (uint32_t)y <= (uint32_t)K ? (uint32_t)y : 0u;
        const double d = deg[v];
        const float r = d > 0.0 ? (float)(1.0 / sqrt(d)) : 0.0f;
        lab[v] = (uint64_t)cls | ((uint64_t)__float_as_uint(r) << 32);
    }
}

// -------------------------------------------------------- form (a): push --

// One thread per record (four records per thread, strided for coalescing):
// gather both endpoints' label records and add the raw contribution into Z
// with FP32 global atomics. Class weights and the row factor come later.
template <bool LAP, bool W, typename P>
__global__ void __launch_bounds__(kBlock)
k_push(int64_t n, int64_t ns, const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
       const float *__restrict__ w, const P *__restrict__ lab, int32_t K, float *__restrict__ Z, int32_t *err)
{
    constexpr int R = 4;
    const int64_t tile = (int64_t)blockIdx.x * (kBlock * R);
    int32_t u[R], v[R];
    float x[R];
    bool ok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = tile + r * kBlock + threadIdx.x;
        ok[r] = i < ns;
        u[r] = ok[r] ? src[i] : 0;
        v[r] = ok[r] ? dst[i] : 0;
        x[r] = (W && ok[r]) ? w[i] : 1.0f;
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (ok[r] && ((uint32_t)u[r] >= (uint64_t)n || (uint32_t)v[r] >= (uint64_t)n)) {
            bad = true;
            ok[r] = false;
        }
    }
    P pu[R], pv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        pu[r] = ok[r] ? lab[u[r]] : (P)0;
        pv[r] = ok[r] ? lab[v[r]] : (P)0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;
        const int yu = LabelRec<P>::cls(pu[r]), yv = LabelRec<P>::cls(pv[r]);
        if (yv > 0) {
            const float c = LAP ? x[r] * LabelRec<P>::rsd(pv[r]) : x[r];
            atomicAdd(&Z[(int64_t)u[r] * K + (yv - 1)], c);
        }
        if (yu > 0) {
            const float c = LAP ? x[r] * LabelRec<P>::rsd(pu[r]) : x[r];
            atomicAdd(&Z[(int64_t)v[r] * K + (yu - 1)], c);
        }
    }
    if (bad) flag_error(err, GEE_EVERTEX);
}

// Z[u, k] = fl32(Z[u, k] * inv[k+1] * (Laplacian ? d_u^-1/2 : 1)), in FP64.
template <bool LAP, typename P>
__global__ void __launch_bounds__(kBlock)
k_scale(int64_t total, int32_t K, uint64_t kmagic, const double *__restrict__ inv, const P *__restrict__ lab,
        float *__restrict__ Z)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t u = K == 1 ? (uint64_t)i : div_big((uint64_t)i, kmagic);
        const int k = (int)((uint64_t)i - u * (uint64_t)K);
        double sc = inv[k + 1];
        if (LAP) sc *= (double)LabelRec<P>::rsd(lab[u]);
        Z[i] = (float)((double)Z[i] * sc);
    }
}

// ---------------------------------------------------- form (b): CSR pull --

// Merge-path split of the (row ends, entries) sequence: segment t starts at
// diagonal d = t * L. Returns rows consumed i (rows < i are complete) and
// entries consumed e = d - i; the row end of row m is taken before entry x iff
// row_ptr[m + 1] <= x.
__global__ void __launch_bounds__(kBlock)
k_seg_bounds(int64_t n, int64_t nnz, const int64_t *__restrict__ row_ptr, int64_t L, int64_t nseg,
             int32_t *__restrict__ seg_i, int64_t *__restrict__ seg_e)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > nseg) return;
    const int64_t total = n + nnz;
    const int64_t d = t * L < total ? t * L : total;
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < n ? d : n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (row_ptr[mid + 1] <= d - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    seg_i[t] = (int32_t)lo;
    seg_e[t] = d - lo;
}

// What segment j holds, from its boundaries (shared by the pull and merge passes).
struct SegInfo {
    int64_t i0, i1, e0, e1;
    bool carried; // row i0 has entries before e0: its part here is a head partial
    bool tail;    // row i1 starts here, has entries here and continues past e1
    int64_t rend; // rows [i0, rend) have entries or ends in this segment
};

__device__ inline SegInfo seg_info(int64_t j, int64_t n, const int64_t *__restrict__ row_ptr,
                                   const int32_t *__restrict__ seg_i, const int64_t *__restrict__ seg_e)
{
    SegInfo s;
    s.i0 = seg_i[j];
    s.i1 = seg_i[j + 1];
    s.e0 = seg_e[j];
    s.e1 = seg_e[j + 1];
    s.carried = (s.i0 < n) && (row_ptr[s.i0] < s.e0);
    const bool i1_here = (s.i1 < n) && (s.e0 < s.e1) && (row_ptr[s.i1] < s.e1);
    s.tail = i1_here && !(s.i1 == s.i0 && s.carried);
    s.rend = s.i1 + (i1_here ? 1 : 0);
    return s;
}

template <typename B> __device__ inline void lds_add(B *p, B x);
template <> __device__ inline void lds_add<uint32_t>(uint32_t *p, uint32_t x) { atomicAdd(p, x); }
template <> __device__ inline void lds_add<double>(double *p, double x) { atomicAdd(p, x); }

// One wavefront per segment. The segment's rows are walked in windows of RW
// consecutive rows whose K bins live in this wavefront's LDS slice. Entries are
// read 64 at a time (coalesced), each lane finds its entry's row by binary
// search over the window's row starts, gathers the neighbour's label record and
// adds into bin (row, class) with an LDS atomic. A window's rows are then
// written to Z as one contiguous block (non-temporal stores); a row cut by a
// segment boundary goes to the FP64 partials instead (head: continues from an
// earlier segment; tail: continues into later ones).
template <typename B, bool LAP, bool W, typename P>
__global__ void __launch_bounds__(kBlock)
k_pull(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
       const float *__restrict__ val, const P *__restrict__ lab, const double *__restrict__ inv, int32_t K,
       uint64_t kmagic32, const int32_t *__restrict__ seg_i, const int64_t *__restrict__ seg_e, int64_t nseg,
       int RW, uint32_t wave_bytes, float *__restrict__ Z, double *__restrict__ part, int32_t *err)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (j >= nseg) return;
    B *bins = (B *)(smem + (size_t)wave * wave_bytes);
    int32_t *cs = (int32_t *)(smem + (size_t)wave * wave_bytes + align_up((size_t)RW * K * sizeof(B), 16));

    const SegInfo sg = seg_info(j, n, row_ptr, seg_i, seg_e);
    for (int b = lane; b < RW * K; b += kWave) bins[b] = (B)0;
    bool bad = false;

    for (int64_t r = sg.i0; r < sg.rend; r += RW) {
        const int nr = (int)((sg.rend - r) < RW ? (sg.rend - r) : RW);
        // clamped row starts of the window, relative to e0; cs[nr] ends the last row
        for (int l = lane; l <= nr; l += kWave) {
            int64_t p = row_ptr[r + l];
            p = p < sg.e0 ? sg.e0 : (p > sg.e1 ? sg.e1 : p);
            cs[l] = (int32_t)(p - sg.e0);
        }
        wave_sync();
        const int32_t ws = cs[0], we = cs[nr];
        constexpr int U = 4;
        for (int32_t q0 = ws; q0 < we; q0 += U * kWave) {
            int32_t q[U], c[U];
#pragma unroll
            for (int t = 0; t < U; ++t) {
                q[t] = q0 + t * kWave + lane;
                c[t] = q[t] < we ? col[sg.e0 + q[t]] : -1;
            }
            P pk[U];
            float x[U];
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const bool in = q[t] < we;
                const bool ok = in && (uint32_t)c[t] < (uint64_t)n;
                bad |= in && !ok;
                if (!ok) q[t] = -1;
                pk[t] = ok ? lab[c[t]] : (P)0;
                x[t] = (W && ok) ? val[sg.e0 + q[t]] : 1.0f;
            }
#pragma unroll
            for (int t = 0; t < U; ++t) {
                const int y = LabelRec<P>::cls(pk[t]);
                if (q[t] < 0 || y == 0) continue;
                int lo = 0, hi = nr; // cs[lo] <= q < cs[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (cs[mid] <= q[t]) lo = mid;
                    else hi = mid;
                }
                if (sizeof(B) == 4) {
                    lds_add<B>(&bins[lo * K + (y - 1)], (B)1);
                } else {
                    double cval = W ? (double)x[t] : 1.0;
                    if (LAP) cval *= (double)LabelRec<P>::rsd(pk[t]);
                    lds_add<B>(&bins[lo * K + (y - 1)], (B)cval);
                }
            }
        }
        wave_sync();
        const int total = nr * K;
        for (int idx = lane; idx < total; idx += kWave) {
            const int l = (int)div_small((uint32_t)idx, kmagic32);
            const int k = idx - l * K;
            const int64_t u = r + l;
            const B b = bins[idx];
            bins[idx] = (B)0;
            if (u == sg.i0 && sg.carried) {
                part[(2 * j) * K + k] = (double)b;
            } else if (u == sg.i1 && sg.tail) {
                part[(2 * j + 1) * K + k] = (double)b;
            } else {
                double sc = inv[k + 1];
                if (LAP) sc *= (double)LabelRec<P>::rsd(lab[u]);
                __builtin_nontemporal_store((float)((double)b * sc), &Z[u * K + k]);
            }
        }
        wave_sync();
    }
    if (bad) flag_error(err, GEE_EVERTEX);
}

// Rows cut by segment boundaries: add the tail partial of the segment the row
// starts in and the head partials of the following segments, in segment order,
// then scale and write the row once.
template <bool LAP, typename P>
__global__ void __launch_bounds__(kBlock)
k_merge(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ seg_i,
        const int64_t *__restrict__ seg_e, int64_t nseg, const P *__restrict__ lab, const double *__restrict__ inv,
        int32_t K, const double *__restrict__ part, float *__restrict__ Z)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (j >= nseg) return;
    const SegInfo sg = seg_info(j, n, row_ptr, seg_i, seg_e);
    if (!sg.tail) return;
    const int64_t u = sg.i1;
    const double ru = LAP ? (double)LabelRec<P>::rsd(lab[u]) : 1.0;
    for (int k = lane; k < K; k += kWave) {
        double acc = part[(2 * j + 1) * K + k];
        for (int64_t jj = j + 1; jj < nseg; ++jj) {
            acc += part[(2 * jj) * K + k];
            if (seg_i[jj + 1] > u) break;
        }
        Z[u * K + k] = (float)(acc * (inv[k + 1] * ru));
    }
}

// -------------------------------------------------------------- copy probe --

__global__ void __launch_bounds__(kBlock)
k_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n16)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

template <typename P> inline P *as(void *p) { return static_cast<P *>(p); }

} // namespace

// ================================================================ launchers ==

hipError_t launch_fill_u64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(count, kBlock, 65536)), dim3(kBlock), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t count, float value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(count, kBlock * 4, 65536)), dim3(kBlock), 0, s, p, count,
                       value);
    return hipGetLastError();
}

hipError_t launch_counts(const int32_t *labels, int64_t n, int32_t K, uint64_t *counts, void *packed, Pack pack,
                         int32_t *err, hipStream_t s)
{
    hipError_t e = launch_fill_u64(counts, (int64_t)K + 1, 0, s);
    if (e != hipSuccess) return e;
    const dim3 g(grid_for(n, kBlock * 16, 4096)), b(kBlock);
    if (pack == Pack::U16)
        hipLaunchKernelGGL(k_counts<uint16_t>, g, b, 0, s, labels, n, K, counts, as<uint16_t>(packed), err);
    else
        hipLaunchKernelGGL(k_counts<uint8_t>, g, b, 0, s, labels, n, K, counts,
                           pack == Pack::U8 ? as<uint8_t>(packed) : nullptr, err);
    return hipGetLastError();
}

hipError_t launch_weights(const uint64_t *counts, int32_t K, double *inv, hipStream_t s)
{
    hipLaunchKernelGGL(k_weights, dim3(grid_for((int64_t)K + 1, kBlock, 1 << 20)), dim3(kBlock), 0, s, counts, K,
                       inv);
    return hipGetLastError();
}

hipError_t launch_degrees_coo(int64_t n, int64_t ns, const int32_t *src, const int32_t *dst, const float *w,
                              double *deg, bool check_neg, int32_t *err, hipStream_t s)
{
    hipError_t e = launch_fill_u64(reinterpret_cast<uint64_t *>(deg), n, 0, s); // +0.0
    if (e != hipSuccess || ns == 0) return e;
    const dim3 g(grid_for(ns, kBlock * 8, 1 << 20)), b(kBlock);
    if (w) hipLaunchKernelGGL(k_degrees_coo<true>, g, b, 0, s, n, ns, src, dst, w, deg, check_neg, err);
    else hipLaunchKernelGGL(k_degrees_coo<false>, g, b, 0, s, n, ns, src, dst, w, deg, check_neg, err);
    return hipGetLastError();
}

hipError_t launch_degrees_csr(int64_t n, const int64_t *row_ptr, const float *val, int64_t nnz, double *deg,
                              bool check_neg, int32_t *err, hipStream_t s)
{
    const dim3 g(grid_for(n, kBlock, 1 << 20)), b(kBlock);
    if (val) hipLaunchKernelGGL(k_degrees_csr<true>, g, b, 0, s, n, row_ptr, val, nnz, deg, check_neg, err);
    else hipLaunchKernelGGL(k_degrees_csr<false>, g, b, 0, s, n, row_ptr, val, nnz, deg, check_neg, err);
    return hipGetLastError();
}

hipError_t launch_pack_lap(const int32_t *labels, int64_t n, int32_t K, const double *deg, uint64_t *lab,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_lap, dim3(grid_for(n, kBlock * 4, 1 << 20)), dim3(kBlock), 0, s, labels, n, K, deg,
                       lab);
    return hipGetLastError();
}

template <bool LAP, bool W, typename P>
static hipError_t push_t(const EmbedArgs &a, int64_t ns, const int32_t *src, const int32_t *dst, const float *w,
                         hipStream_t s)
{
    const int64_t blocks = (ns + kBlock * 4 - 1) / (kBlock * 4);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_push<LAP, W, P>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.n, ns, src, dst, w,
                       static_cast<const P *>(a.lab), a.K, a.Z, a.err);
    return hipGetLastError();
}

hipError_t launch_push(const EmbedArgs &a, int64_t ns, const int32_t *src, const int32_t *dst, const float *w,
                       hipStream_t s)
{
    if (a.laplacian) {
        return w ? push_t<true, true, uint64_t>(a, ns, src, dst, w, s)
                 : push_t<true, false, uint64_t>(a, ns, src, dst, w, s);
    }
    if (a.pack == Pack::U16)
        return w ? push_t<false, true, uint16_t>(a, ns, src, dst, w, s)
                 : push_t<false, false, uint16_t>(a, ns, src, dst, w, s);
    return w ? push_t<false, true, uint8_t>(a, ns, src, dst, w, s) : push_t<false, false, uint8_t>(a, ns, src, dst, w, s);
}

static uint64_t magic64(int32_t K) { return K <= 1 ? 0 : (uint64_t)(~0ull / (uint64_t)K) + 1; }
static uint64_t magic32(int32_t K) { return ((1ull << 32) + (uint64_t)K - 1) / (uint64_t)K; }

hipError_t launch_scale(const EmbedArgs &a, hipStream_t s)
{
    const int64_t total = a.n * a.K;
    const dim3 g(grid_for(total, kBlock * 8, 1 << 20)), b(kBlock);
    if (a.laplacian)
        hipLaunchKernelGGL((k_scale<true, uint64_t>), g, b, 0, s, total, a.K, magic64(a.K), a.inv,
                           static_cast<const uint64_t *>(a.lab), a.Z);
    else
        hipLaunchKernelGGL((k_scale<false, uint8_t>), g, b, 0, s, total, a.K, magic64(a.K), a.inv,
                           static_cast<const uint8_t *>(nullptr), a.Z);
    return hipGetLastError();
}

hipError_t launch_seg_bounds(int64_t n, int64_t nnz, const int64_t *row_ptr, int64_t L, int64_t nseg,
                             int32_t *seg_i, int64_t *seg_e, hipStream_t s)
{
    hipLaunchKernelGGL(k_seg_bounds, dim3(grid_for(nseg + 1, kBlock, 1 << 30)), dim3(kBlock), 0, s, n, nnz,
                       row_ptr, L, nseg, seg_i, seg_e);
    return hipGetLastError();
}

size_t pull_wave_bytes(int32_t K, bool wide_bins, int rw)
{
    return align_up((size_t)rw * K * (wide_bins ? 8 : 4), 16) + align_up((size_t)(rw + 1) * 4, 16);
}

template <typename B, bool LAP, bool W, typename P>
static hipError_t pull_t(const EmbedArgs &a, const int64_t *row_ptr, const int32_t *col, const float *val,
                         const int32_t *seg_i, const int64_t *seg_e, int64_t nseg, int rw, double *part,
                         hipStream_t s)
{
    const uint32_t wb = (uint32_t)pull_wave_bytes(a.K, sizeof(B) == 8, rw);
    int wpb = (int)(65536 / wb);
    wpb = wpb > kWavesPerBlock ? kWavesPerBlock : (wpb < 1 ? 1 : wpb);
    const int64_t blocks = (nseg + wpb - 1) / wpb;
    hipLaunchKernelGGL((k_pull<B, LAP, W, P>), dim3((unsigned)blocks), dim3(wpb * kWave), (size_t)wpb * wb, s, a.n,
                       row_ptr, col, val, static_cast<const P *>(a.lab), a.inv, a.K, magic32(a.K), seg_i, seg_e,
                       nseg, rw, wb, a.Z, part, a.err);
    return hipGetLastError();
}

hipError_t launch_pull(const EmbedArgs &a, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const float *val,
                       const int32_t *seg_i, const int64_t *seg_e, int64_t nseg, int rw, double *part, hipStream_t s)
{
    (void)nnz;
    if (a.laplacian)
        return val ? pull_t<double, true, true, uint64_t>(a, row_ptr, col, val, seg_i, seg_e, nseg, rw, part, s)
                   : pull_t<double, true, false, uint64_t>(a, row_ptr, col, val, seg_i, seg_e, nseg, rw, part, s);
    if (val)
        return a.pack == Pack::U16
                   ? pull_t<double, false, true, uint16_t>(a, row_ptr, col, val, seg_i, seg_e, nseg, rw, part, s)
                   : pull_t<double, false, true, uint8_t>(a, row_ptr, col, val, seg_i, seg_e, nseg, rw, part, s);
    return a.pack == Pack::U16
               ? pull_t<uint32_t, false, false, uint16_t>(a, row_ptr, col, val, seg_i, seg_e, nseg, rw, part, s)
               : pull_t<uint32_t, false, false, uint8_t>(a, row_ptr, col, val, seg_i, seg_e, nseg, rw, part, s);
}

hipError_t launch_merge(const EmbedArgs &a, const int64_t *row_ptr, const int32_t *seg_i, const int64_t *seg_e,
                        int64_t nseg, const double *part, hipStream_t s)
{
    const int64_t blocks = (nseg + kWavesPerBlock - 1) / kWavesPerBlock;
    if (a.laplacian)
        hipLaunchKernelGGL((k_merge<true, uint64_t>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.n, row_ptr,
                           seg_i, seg_e, nseg, static_cast<const uint64_t *>(a.lab), a.inv, a.K, part, a.Z);
    else
        hipLaunchKernelGGL((k_merge<false, uint8_t>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.n, row_ptr,
                           seg_i, seg_e, nseg, static_cast<const uint8_t *>(nullptr), a.inv, a.K, part, a.Z);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n16, kBlock * 8, 1 << 20)), dim3(kBlock), 0, s,
                       static_cast<uint4 *>(dst), static_cast<const uint4 *>(src), n16);
    return hipGetLastError();
}

} // namespace gee
