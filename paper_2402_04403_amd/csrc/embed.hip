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

#include <type_traits>

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
    // four labels per lane are loaded before any is added
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < n; v0 += 4 * stride) {
        int32_t y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t v = v0 + q * stride;
            y[q] = v < n ? labels[v] : -1; // -1: past the end
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t v = v0 + q * stride;
            if (v >= n) break;
            const bool ok = (uint32_t)y[q] <= (uint32_t)K;
            bad |= !ok;
            if (ok) {
                if (lds) atomicAdd(&hist[y[q]], 1u);
                else atomicAdd((unsigned long long *)&counts[y[q]], 1ull);
            }
            if (packed) packed[v] = (P)(ok ? y[q] : 0);
        }
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

// Class counts of every vector of a batch group in one launch: blockIdx.y picks the
// vector (labels at labels + vec * n, counts at inv_off), so a batch of many small
// vectors does not pay a launch per vector. Counts start at zero.
__global__ void __launch_bounds__(kBlock)
k_counts_group(const int32_t *__restrict__ labels, int64_t n, GroupDesc d, uint64_t *__restrict__ counts,
               int32_t *err)
{
    __shared__ uint32_t hist[kBatchMaxKT + 1];
    const int i = blockIdx.y;
    const int32_t K = d.K[i];
    const int32_t *__restrict__ lab = labels + (int64_t)d.vec[i] * n;
    for (int b = threadIdx.x; b <= K; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    // four labels per lane are loaded before any is added
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < n; v0 += 4 * stride) {
        int32_t y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t v = v0 + q * stride;
            y[q] = v < n ? lab[v] : -1; // -1: past the end (not counted, not an error)
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool ok = (uint32_t)y[q] <= (uint32_t)K;
            bad |= !ok && v0 + q * stride < n;
            if (ok) atomicAdd(&hist[y[q]], 1u);
        }
    }
    if (bad) flag_error(err, GEE_ELABEL);
    __syncthreads();
    uint64_t *__restrict__ cnt = counts + d.inv_off[i];
    for (int b = threadIdx.x; b <= K; b += blockDim.x)
        if (hist[b]) atomicAdd((unsigned long long *)&cnt[b], (unsigned long long)hist[b]);
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
// Row sums of a CSR: one row per lane, its weights added in stored order with 16-byte
// loads where the row is aligned for them (the lanes of a wavefront read 64 different
// rows, so wide loads cut the memory requests fourfold). A row of more than kDegLong
// entries is summed instead by the whole wavefront (lane l takes entries l, l + 64, ...
// in order, then a fixed butterfly adds the 64 partial sums), so one long row does not
// hold a lane for its whole length. Every sum is taken in a fixed order.
constexpr int64_t kDegLong = 4096;

template <bool W>
__global__ void __launch_bounds__(kBlock)
k_degrees_csr(int64_t n, const int64_t *__restrict__ row_ptr, const float *__restrict__ val, int64_t nnz,
              double *__restrict__ deg, bool check_neg, bool vec_ok, int32_t *err)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    bool neg = false;
    for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave; base < n;
         base += waves * kWave) {
        const int64_t u = base + lane;
        const bool act = u < n;
        int64_t b = act ? row_ptr[u] : 0, e = act ? row_ptr[u + 1] : 0;
        b = b < 0 ? 0 : (b > nnz ? nnz : b);
        e = e < b ? b : (e > nnz ? nnz : e);
        if (!W) {
            if (act) deg[u] = (double)(e - b);
            continue;
        }
        const bool longrow = act && e - b > kDegLong;
        if (act && !longrow) {
            double d = 0.0;
            int64_t q = b;
            if (vec_ok) {
                for (; q < e && (q & 3); ++q) {
                    const float x = val[q];
                    neg |= !(x >= 0.0f);
                    d += (double)x;
                }
                for (; q + 4 <= e; q += 4) {
                    const float4 x = *reinterpret_cast<const float4 *>(val + q);
                    neg |= !(x.x >= 0.0f) || !(x.y >= 0.0f) || !(x.z >= 0.0f) || !(x.w >= 0.0f);
                    d += (double)x.x;
                    d += (double)x.y;
                    d += (double)x.z;
                    d += (double)x.w;
                }
            }
            for (; q < e; ++q) {
                const float x = val[q];
                neg |= !(x >= 0.0f);
                d += (double)x;
            }
            deg[u] = d;
        }
        // the long rows of these 64, one at a time by the whole wavefront
        for (uint64_t longs = __ballot(longrow); longs; longs &= longs - 1) {
            const int l = __builtin_ctzll(longs);
            const int64_t lb = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l) & 0xffffffffll;
            const int64_t lb_hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
            const int64_t le_lo = __builtin_amdgcn_readlane((int)(e & 0xffffffff), l) & 0xffffffffll;
            const int64_t le_hi = __builtin_amdgcn_readlane((int)(e >> 32), l);
            const int64_t rb = (lb_hi << 32) | lb, re = (le_hi << 32) | le_lo;
            double d = 0.0;
            for (int64_t q = rb + lane; q < re; q += kWave) {
                const float x = val[q];
                neg |= !(x >= 0.0f);
                d += (double)x;
            }
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) d += __shfl_xor(d, o, kWave);
            if (lane == 0) deg[base + l] = d;
        }
    }
    if (check_neg && neg) flag_error(err, GEE_ENEGW);
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

// Compact label table of the hot vertices named by a CSR's hot slots.
template <typename P>
__global__ void __launch_bounds__(kBlock)
k_pack_hot(const P *__restrict__ lab, int64_t n, const int32_t *__restrict__ hot_ids, int64_t n_hot,
           P *__restrict__ hotlab, int32_t *err)
{
    for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n_hot; h += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = hot_ids[h];
        const bool ok = (uint32_t)v < (uint64_t)n;
        if (!ok) flag_error(err, GEE_EVERTEX);
        hotlab[h] = ok ? lab[v] : (P)0;
    }
}

// Hot label table packed at 6 bits per class, five slots per 32-bit word (K <= 63).
__global__ void __launch_bounds__(kBlock)
k_pack_hot6(const uint8_t *__restrict__ lab, int64_t n, const int32_t *__restrict__ hot_ids, int64_t n_hot,
            uint32_t *__restrict__ hot6, int32_t *err)
{
    const int64_t nw = (n_hot + 4) / 5;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t word = 0;
        for (int i = 0; i < 5; ++i) {
            const int64_t h = 5 * w + i;
            if (h >= n_hot) break;
            const int32_t v = hot_ids[h];
            const bool ok = (uint32_t)v < (uint64_t)n;
            if (!ok) flag_error(err, GEE_EVERTEX);
            word |= (ok ? (uint32_t)(lab[v] & 63u) : 0u) << (6 * i);
        }
        hot6[w] = word;
    }
}

// -------------------------------------------------------- form (a): push --

// One thread per record (four records per thread, strided for coalescing):
// gather both endpoints' label records and add the raw contribution into Z
// with FP32 global atomics. Class weights and the row factor come later.
// ATOMIC = false is the diagnostic of the paper's atomics-off run (Section IV):
// plain read-modify-write, so concurrent updates of one element can be lost.
template <bool LAP, bool W, typename P, bool ATOMIC>
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
            float *z = &Z[(int64_t)u[r] * K + (yv - 1)];
            if (ATOMIC) atomicAdd(z, c);
            else *z += c;
        }
        if (yu > 0) {
            const float c = LAP ? x[r] * LabelRec<P>::rsd(pu[r]) : x[r];
            float *z = &Z[(int64_t)v[r] * K + (yu - 1)];
            if (ATOMIC) atomicAdd(z, c);
            else *z += c;
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

// Wavefront inclusive max-scan of values >= -1 with DPP lane moves (no LDS
// traffic, so it never waits behind the LDS atomics in flight): shifts by 1, 2,
// 4, 8 within each 16-lane row, then row broadcasts of lanes 15 and 31.
__device__ inline int imax(int a, int b) { return a > b ? a : b; }
__device__ inline int wave_incl_max(int x)
{
    x = imax(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false)); // row_shr:1
    x = imax(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false)); // row_shr:2
    x = imax(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false)); // row_shr:4
    x = imax(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false)); // row_shr:8
    x = imax(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xa, 0xf, false)); // row_bcast:15
    x = imax(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xc, 0xf, false)); // row_bcast:31
    return x;
}
// Value of the previous lane (-1 for lane 0): DPP wave_shr:1.
__device__ inline int wave_shr1(int x) { return __builtin_amdgcn_update_dpp(-1, x, 0x138, 0xf, 0xf, false); }

// Bin storage of the pull pass, by kind:
//  0: one FP64 sum per class (weighted or Laplacian);
//  1: unit-weight counts, two classes per 32-bit word (16-bit counters; a segment
//     holds at most 65535 entries, so they cannot overflow);
//  2: unit-weight counts, one 32-bit counter per class;
//  3: one FP32 sum per class (weighted or Laplacian). A window whose rows all have at
//     most kF32Terms entries in the segment uses them: no bin then takes more than
//     kF32Terms terms, and for non-negative terms an FP32 sum of m terms in any order
//     is within (m - 1) 2^-24 of its exact value, relative. A window with a longer row
//     takes FP64 bins for half as many rows in the same LDS; a segment with a negative
//     weight is flagged and computed again with FP64 bins by a second launch.
template <int BK> struct Bins;
template <> struct Bins<0> {
    using word = double;
    __host__ __device__ static int words(int K) { return K; }
    __device__ static void add(word *row, int k, double x) { atomicAdd(&row[k], x); }
    __device__ static void add_masked(word *row, int k, double x, bool use) { atomicAdd(&row[k], use ? x : 0.0); }
    __device__ static double get(const word *row, int k) { return row[k]; }
};
template <> struct Bins<1> {
    using word = uint32_t;
    __host__ __device__ static int words(int K) { return (K + 1) / 2; }
    __device__ static void add(word *row, int k, double) { atomicAdd(&row[k >> 1], 1u << (16 * (k & 1))); }
    __device__ static void add_masked(word *row, int k, double, bool use)
    {
        atomicAdd(&row[k >> 1], use ? 1u << (16 * (k & 1)) : 0u);
    }
    __device__ static double get(const word *row, int k) { return (double)((row[k >> 1] >> (16 * (k & 1))) & 0xffffu); }
};
template <> struct Bins<2> {
    using word = uint32_t;
    __host__ __device__ static int words(int K) { return K; }
    __device__ static void add(word *row, int k, double) { atomicAdd(&row[k], 1u); }
    __device__ static void add_masked(word *row, int k, double, bool use) { atomicAdd(&row[k], use ? 1u : 0u); }
    __device__ static double get(const word *row, int k) { return (double)row[k]; }
};
template <> struct Bins<3> {
    using word = float;
    __host__ __device__ static int words(int K) { return K; }
    __device__ static void add(word *row, int k, double x) { atomicAdd(&row[k], (float)x); }
    __device__ static void add_masked(word *row, int k, double x, bool use)
    {
        atomicAdd(&row[k], use ? (float)x : 0.0f);
    }
    __device__ static double get(const word *row, int k) { return (double)row[k]; }
};
// Bin kind of the unit-weight adjacency variant, and of the others.
constexpr int kUnitBins = 1;
constexpr int kRealBins = 3;
constexpr int kF32Terms = 128; // terms per FP32 bin: (128 - 1) 2^-24 = 7.6e-6 relative at most

constexpr int kPass = 1024;              // entries whose row-start markers are mapped at once
constexpr int kChunk = 2 * 4 * kWave;    // entries per inner step (two 16-byte loads per lane)
constexpr int kFlatFlushMaxK = kWave;    // K up to this writes rows as flat aligned blocks
constexpr int kSinkBytes = kWave * 8;    // one word per lane for masked bin updates

// LDS of one wavefront: bins of RW rows, the row-start marker map of one pass,
// and the class weights (K <= 64).
__host__ __device__ inline size_t pull_bins_bytes(int32_t K, int bk, int rw)
{
    if (bk == 3) return align_up((size_t)((rw + 1) / 2) * K * 8, 16); // rw FP32 rows or (rw + 1) / 2 FP64 rows
    const size_t row = bk == 0 ? (size_t)K * 8 : (bk == 1 ? (size_t)(K + 1) / 2 * 4 : (size_t)K * 4);
    return align_up((size_t)rw * row, 16);
}
__host__ __device__ inline size_t pull_lds_bytes(int32_t K, int bk, int rw)
{
    return pull_bins_bytes(K, bk, rw) + kPass + kSinkBytes + (K <= kFlatFlushMaxK ? align_up((size_t)K * 8, 16) : 0);
}

// One wavefront per segment of seg_len work items (rows + entries).
//  - The segment's rows are walked in windows of RW consecutive rows whose K bins
//    live in this wavefront's LDS.
//  - A window's entries are taken in passes of kPass entries; in each pass the
//    rows starting inside it write their local index into a byte map at their
//    first entry. An entry's row is the running maximum of the markers up to it:
//    a max over the lane's own four entries plus a wavefront max-scan, carried
//    from step to step.
//  - Each step reads 512 entries (two 16-byte loads per lane). The neighbour label
//    records of step i are gathered before the column loads of step i+1 are
//    issued, so those loads stay in flight while step i adds into its bins with
//    LDS atomics. A column value with bit 31 set names a slot of the compact
//    hot-vertex label table instead of a vertex.
//  - The window's rows are written to Z with non-temporal stores: for K <= 64 as
//    one flat run of floats in aligned 64-float blocks (whole cache lines), else
//    row by row with lanes over classes. A row cut by a segment boundary goes to
//    the FP64 partials instead (head: continues from an earlier segment; tail:
//    continues into later ones).
//  - Real-valued bins (kind 3) are FP32 unless a row of the window has more than
//    kF32Terms entries in the segment; the weighted adjacency version flags a
//    segment with a negative weight in redo[j] (FP32 sums are only bounded relative
//    to their own value for terms of one sign), and a second launch with FP64 bins
//    (kind 0, redo given) recomputes exactly the flagged segments.
template <int BK, bool LAP, bool W, typename P, bool H6>
__global__ void __launch_bounds__(kBlock)
k_pull(int64_t n, int64_t nnz, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
       const float *__restrict__ val, const P *__restrict__ lab, const P *__restrict__ hotlab, int64_t n_hot,
       const double *__restrict__ inv, int32_t K, const int32_t *__restrict__ seg_i,
       const int64_t *__restrict__ seg_e, int64_t nseg, int RW, uint32_t wave_bytes, bool vec_ok,
       float *__restrict__ Z, double *__restrict__ part, uint8_t *__restrict__ redo, int32_t *err)
{
    constexpr bool REAL = BK == 0 || BK == 3;     // sums of weights (and d^-1/2), not counts
    constexpr bool FLAG_NEG = BK == 3 && W && !LAP; // flags segments with a negative weight
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (j >= nseg) return;
    if (BK == 0 && redo && !redo[j]) return; // the FP64 pass over flagged segments only
    unsigned char *my = smem + (size_t)wave * wave_bytes;
    const size_t bins_bytes = pull_bins_bytes(K, BK, RW);
    int8_t *mark = (int8_t *)(my + bins_bytes);
    unsigned char *sink_bytes = my + bins_bytes + kPass; // one 8-byte word per lane: target of masked adds
    double *invt = (double *)(my + bins_bytes + kPass + kSinkBytes);
    const bool flat = K <= kFlatFlushMaxK;

    const SegInfo sg = seg_info(j, n, row_ptr, seg_i, seg_e);
    for (int b = lane; b < (int)(bins_bytes / 4); b += kWave) ((uint32_t *)my)[b] = 0u;
    for (int b = lane; b < kPass / 4; b += kWave) ((int32_t *)mark)[b] = -1;
    if (flat && lane < K) invt[lane] = inv[lane + 1];
    bool bad = false, neg = false;
    // A segment whose last 16-byte column quad may pass the end of the array takes
    // the guarded loads; every other segment runs branch-free steps, so the loads
    // in flight can be counted statically and the next step's column loads stay
    // outstanding while this step's atomics issue.
    const bool tail_seg = !vec_ok || sg.e1 + 4 > nnz;

    // row_ptr[rr + lane], row_ptr[rr + lane + 1], clamped into the array; the next
    // window's pair is fetched when a window starts, so no window waits for it
    auto fetch_rows = [&](int64_t rr, int64_t &a0, int64_t &a1) {
        int64_t idx = rr + lane;
        idx = idx < n - 1 ? idx : n - 1;
        a0 = row_ptr[idx];
        a1 = row_ptr[idx + 1];
    };
    int64_t rp0, rp1;
    fetch_rows(sg.i0, rp0, rp1);
    for (int64_t r = sg.i0; r < sg.rend;) {
        int nr = (int)((sg.rend - r) < RW ? (sg.rend - r) : RW);
        int64_t p0 = rp0, p1 = rp1;
        // lane l < nr: clamped start and end of row r + l, relative to e0
        int32_t cs = 0, ce = 0;
        if (lane < nr) {
            p0 = p0 < sg.e0 ? sg.e0 : (p0 > sg.e1 ? sg.e1 : p0);
            p1 = p1 < sg.e0 ? sg.e0 : (p1 > sg.e1 ? sg.e1 : p1);
            cs = (int32_t)(p0 - sg.e0);
            ce = (int32_t)(p1 - sg.e0);
        }
        bool wide = false;
        if constexpr (BK == 3) {
            // FP32 bins unless one of the window's rows has more than kF32Terms entries here;
            // then FP64 bins for the first (RW + 1) / 2 rows
            wide = __ballot(ce - cs > kF32Terms) != 0ull;
            if (wide && nr > (RW + 1) / 2) {
                nr = (RW + 1) / 2;
                if (lane >= nr) cs = ce = 0;
            }
        }
        fetch_rows(r + nr, rp0, rp1);
        const int32_t ws = __builtin_amdgcn_readlane(cs, 0), we = __builtin_amdgcn_readlane(ce, nr - 1);
        // 4-aligned (in absolute entry index) start of the window's steps
        const int32_t base = (int32_t)(((sg.e0 + ws) & ~(int64_t)3) - sg.e0);
        const bool nonempty = lane < nr && cs < ce;

        auto window = [&](auto bins_tag) {
            using BT = typename decltype(bins_tag)::type;
            using word = typename BT::word;
            word *bins = (word *)my;
            word *sink = (word *)sink_bytes;
            const int KW = BT::words(K);
            int carry = -1;
            for (int32_t p0 = base; p0 < we; p0 += kPass) {
                const int32_t p1 = (p0 + kPass < we) ? p0 + kPass : we;
                const bool mine = nonempty && cs >= p0 && cs < p0 + kPass;
                if (mine) mark[cs - p0] = (int8_t)lane;
                wave_sync();

                auto pass = [&](auto tail_tag) {
                    constexpr bool TAIL = decltype(tail_tag)::value;
                    // column (and weight) quad of a half-step: lane owns entries q .. q+3
                    auto load = [&](int32_t q, int32_t (&c)[4], float (&x)[4]) {
                        const bool any = q < p1 && q + 3 >= ws;
                        if (TAIL) {
                            const int64_t a = sg.e0 + q;
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                const bool in = any && q + t >= ws && q + t < p1;
                                c[t] = in ? col[a + t] : 0;
                                if (W) x[t] = in ? val[a + t] : 0.0f;
                            }
                        } else {
                            // lanes outside the pass read the window's first quad (in bounds)
                            const int64_t a = sg.e0 + (any ? q : base);
                            const int4 cq = *reinterpret_cast<const int4 *>(col + a);
                            c[0] = cq.x, c[1] = cq.y, c[2] = cq.z, c[3] = cq.w;
                            if (W) {
                                const float4 vq = *reinterpret_cast<const float4 *>(val + a);
                                x[0] = vq.x, x[1] = vq.y, x[2] = vq.z, x[3] = vq.w;
                            }
                        }
                    };
                    // row-start marker word of a half-step (-1 outside the pass)
                    auto marks = [&](int32_t q) -> int32_t {
                        const bool any = q < p1 && q + 3 >= ws;
                        int32_t wi = (q - p0) >> 2;
                        wi = wi < 0 ? 0 : (wi >= kPass / 4 ? kPass / 4 - 1 : wi);
                        const int32_t mw = ((const int32_t *)mark)[wi];
                        return any ? mw : -1;
                    };
                    int32_t cc[2][4], cn[2][4] = {};
                    float xc[2][4] = {}, xn[2][4] = {};
                    int32_t mwc[2], mwn[2] = {-1, -1};
                    load(p0 + 4 * lane, cc[0], xc[0]);
                    load(p0 + 4 * kWave + 4 * lane, cc[1], xc[1]);
                    mwc[0] = marks(p0 + 4 * lane);
                    mwc[1] = marks(p0 + 4 * kWave + 4 * lane);
                    for (int32_t q0 = p0; q0 < p1; q0 += kChunk) {
                        int m[2][4];
                        bool in[2][4];
                        P pk[2][4];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int32_t q = q0 + h * 4 * kWave + 4 * lane;
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                m[h][t] = (int)(int8_t)(mwc[h] >> (8 * t));
                                in[h][t] = q + t >= ws && q + t < p1;
                            }
                            m[h][1] = imax(m[h][1], m[h][0]);
                            m[h][2] = imax(m[h][2], m[h][1]);
                            m[h][3] = imax(m[h][3], m[h][2]);
                            const int incl = wave_incl_max(m[h][3]);
                            const int excl = imax(wave_shr1(incl), carry);
                            carry = imax(carry, __builtin_amdgcn_readlane(incl, kWave - 1));
#pragma unroll
                            for (int t = 0; t < 4; ++t) m[h][t] = imax(m[h][t], excl);
                            // label records, one gather per entry (masked lanes read lab[0]);
                            // bit 31 of a column selects the hot table
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                const int32_t c = cc[h][t];
                                const bool hot = c < 0;
                                const uint32_t idx = (uint32_t)c & 0x7fffffffu;
                                const bool ok = in[h][t] && (hot ? (int64_t)idx < n_hot : (int64_t)idx < n);
                                bad |= in[h][t] && !ok;
                                in[h][t] = ok;
                                if (H6) {
                                    // one aligned 32-bit gather: a hot slot's 6-bit field in the
                                    // packed hot table, or the byte of a cold label in its word
                                    const uint32_t wq = __umulhi(idx, 0xCCCCCCCDu) >> 2; // idx / 5
                                    const uint32_t *src =
                                        !ok ? reinterpret_cast<const uint32_t *>(lab)
                                            : (hot ? reinterpret_cast<const uint32_t *>(hotlab) + wq
                                                   : reinterpret_cast<const uint32_t *>(lab + (idx & ~3u)));
                                    const uint32_t word32 = *src;
                                    const uint32_t sh = hot ? 6u * (idx - 5u * wq) : 8u * (idx & 3u);
                                    pk[h][t] = ok ? (P)((word32 >> sh) & (hot ? 63u : 255u)) : (P)0;
                                } else {
                                    const P *tab = (ok && hot) ? hotlab : lab;
                                    pk[h][t] = tab[ok ? idx : 0u];
                                }
                            }
                        }
                        // next step's columns (issued after this step's gathers) and markers
                        // (read before this step's atomics enter the LDS queue)
                        const int32_t qn = q0 + kChunk;
                        load(qn + 4 * lane, cn[0], xn[0]);
                        load(qn + 4 * kWave + 4 * lane, cn[1], xn[1]);
                        mwn[0] = marks(qn + 4 * lane);
                        mwn[1] = marks(qn + 4 * kWave + 4 * lane);
                        // bin updates; masked entries add nothing to this lane's sink word
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                const int y = LabelRec<P>::cls(pk[h][t]);
                                const bool use = in[h][t] && y > 0 && m[h][t] >= 0;
                                double add = 1.0;
                                if (REAL) {
                                    if (W) add = (double)xc[h][t];
                                    if (LAP) add *= (double)LabelRec<P>::rsd(pk[h][t]);
                                }
                                if (FLAG_NEG) neg |= use && xc[h][t] < 0.0f;
                                BT::add_masked(use ? &bins[m[h][t] * KW] : &sink[lane], use ? y - 1 : 0, add, use);
                            }
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            mwc[h] = mwn[h];
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                cc[h][t] = cn[h][t];
                                if (W) xc[h][t] = xn[h][t];
                            }
                        }
                    }
                };
                if (tail_seg) pass(std::true_type{});
                else pass(std::false_type{});
                wave_sync();
                if (mine) mark[cs - p0] = -1;
            }
            wave_sync();

            // ---- write the window's rows
            const bool head_here = sg.carried && r == sg.i0;
            const bool tail_here = sg.tail && sg.i1 >= r && sg.i1 < r + nr;
            if (head_here)
                for (int k = lane; k < K; k += kWave) part[(2 * j) * K + k] = BT::get(&bins[0], k);
            if (tail_here)
                for (int k = lane; k < K; k += kWave) part[(2 * j + 1) * K + k] = BT::get(&bins[(sg.i1 - r) * KW], k);
            if (flat) {
                // floats [r K, (r + nr) K) in 64-float blocks aligned to 256 bytes
                const int64_t f_lo = r * K, f_hi = (r + nr) * K;
                const int64_t f_start = f_lo & ~(int64_t)(kWave - 1);
                int64_t f = f_start + lane;
                const int rel = (int)(f - f_lo); // negative in the first block: floats of earlier rows
                int l = rel >= 0 ? rel / K : -((-rel + K - 1) / K);
                int k = rel - l * K;
                const int dl = kWave / K, dk = kWave % K;
                for (; f < f_hi; f += kWave) {
                    if (l >= 0) {
                        const int64_t u = r + l;
                        const bool skip = (head_here && l == 0) || (tail_here && u == sg.i1);
                        if (!skip) {
                            double sc = invt[k];
                            if (LAP) sc *= (double)LabelRec<P>::rsd(lab[u]);
                            __builtin_nontemporal_store((float)(BT::get(&bins[l * KW], k) * sc), &Z[f]);
                        }
                    }
                    l += dl;
                    k += dk;
                    if (k >= K) {
                        k -= K;
                        ++l;
                    }
                }
            } else {
                for (int l = 0; l < nr; ++l) {
                    const int64_t u = r + l;
                    if ((head_here && l == 0) || (tail_here && u == sg.i1)) continue;
                    const double ru = LAP ? (double)LabelRec<P>::rsd(lab[u]) : 1.0;
                    for (int k = lane; k < K; k += kWave)
                        __builtin_nontemporal_store((float)(BT::get(&bins[l * KW], k) * (inv[k + 1] * ru)),
                                                    &Z[u * K + k]);
                }
            }
            wave_sync();
            for (int b = lane; b < nr * KW; b += kWave) bins[b] = (word)0;
            wave_sync();
        };
        struct Own { using type = Bins<BK>; };
        if constexpr (BK == 3) {
            struct F64 { using type = Bins<0>; };
            if (wide) window(F64{});
            else window(Own{});
        } else {
            window(Own{});
        }
        r += nr;
    }
    if (FLAG_NEG) {
        const bool any_neg = __ballot(neg) != 0ull;
        if (lane == 0) redo[j] = any_neg ? 1 : 0;
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
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
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
    // 1,024 workgroups at most: each ends with K + 1 global adds into the same counts
    const dim3 g(grid_for(n, kBlock * 16, 1024)), b(kBlock);
    if (pack == Pack::U16)
        hipLaunchKernelGGL(k_counts<uint16_t>, g, b, 0, s, labels, n, K, counts, as<uint16_t>(packed), err);
    else
        hipLaunchKernelGGL(k_counts<uint8_t>, g, b, 0, s, labels, n, K, counts,
                           pack == Pack::U8 ? as<uint8_t>(packed) : nullptr, err);
    return hipGetLastError();
}

hipError_t launch_counts_group(const int32_t *labels, int64_t n, const GroupDesc &d, uint64_t *counts, int32_t *err,
                               hipStream_t s)
{
    if (d.G < 1 || d.G > kGroupMax) return hipErrorInvalidValue;
    // about 4,096 workgroups over the group: every workgroup ends with K + 1 global adds
    // into its vector's counts, and many workgroups per vector would queue on those words
    const dim3 g(grid_for(n, kBlock * 16, 4096 / d.G), d.G), b(kBlock);
    hipLaunchKernelGGL(k_counts_group, g, b, 0, s, labels, n, d, counts, err);
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
    const bool vec_ok = (uintptr_t)val % 16 == 0;
    if (val) hipLaunchKernelGGL(k_degrees_csr<true>, g, b, 0, s, n, row_ptr, val, nnz, deg, check_neg, vec_ok, err);
    else hipLaunchKernelGGL(k_degrees_csr<false>, g, b, 0, s, n, row_ptr, val, nnz, deg, check_neg, vec_ok, err);
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
    if (a.atomic_updates)
        hipLaunchKernelGGL((k_push<LAP, W, P, true>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.n, ns, src, dst, w,
                           static_cast<const P *>(a.lab), a.K, a.Z, a.err);
    else
        hipLaunchKernelGGL((k_push<LAP, W, P, false>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a.n, ns, src, dst,
                           w, static_cast<const P *>(a.lab), a.K, a.Z, a.err);
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

size_t pull_wave_bytes(int32_t K, bool wide_bins, int rw) { return pull_lds_bytes(K, wide_bins ? kRealBins : kUnitBins, rw); }

template <int BK, bool LAP, bool W, typename P, bool H6 = false>
static hipError_t pull_t(const EmbedArgs &a, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                         const float *val, const void *hotlab, int64_t n_hot, const int32_t *seg_i,
                         const int64_t *seg_e, int64_t nseg, int rw, double *part, uint8_t *redo, hipStream_t s)
{
    const uint32_t wb = (uint32_t)pull_lds_bytes(a.K, BK, rw);
    int wpb = (int)(65536 / wb);
    wpb = wpb > kWavesPerBlock ? kWavesPerBlock : (wpb < 1 ? 1 : wpb);
    const int64_t blocks = (nseg + wpb - 1) / wpb;
    const bool vec_ok = ((uintptr_t)col % 16 == 0) && (!val || (uintptr_t)val % 16 == 0);
    hipLaunchKernelGGL((k_pull<BK, LAP, W, P, H6>), dim3((unsigned)blocks), dim3(wpb * kWave), (size_t)wpb * wb, s,
                       a.n, nnz, row_ptr, col, val, static_cast<const P *>(a.lab), static_cast<const P *>(hotlab),
                       n_hot, a.inv, a.K, seg_i, seg_e, nseg, rw, wb, vec_ok, a.Z, part, redo, a.err);
    return hipGetLastError();
}

hipError_t launch_pull(const EmbedArgs &a, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const float *val,
                       const void *hotlab, int64_t n_hot, const int32_t *seg_i, const int64_t *seg_e, int64_t nseg,
                       int rw, double *part, uint8_t *redo, hipStream_t s)
{
#define GEE_PULL(PK, LAP, W, P) \
    pull_t<PK, LAP, W, P>(a, nnz, row_ptr, col, val, hotlab, n_hot, seg_i, seg_e, nseg, rw, part, nullptr, s)
    if (a.laplacian) return val ? GEE_PULL(kRealBins, true, true, uint64_t) : GEE_PULL(kRealBins, true, false, uint64_t);
    if (val) {
        // FP32 bins, then FP64 bins over the segments that hold a negative weight
        if (!redo) return hipErrorInvalidValue;
        hipError_t e = a.pack == Pack::U16
                           ? pull_t<kRealBins, false, true, uint16_t>(a, nnz, row_ptr, col, val, hotlab, n_hot, seg_i,
                                                                      seg_e, nseg, rw, part, redo, s)
                           : pull_t<kRealBins, false, true, uint8_t>(a, nnz, row_ptr, col, val, hotlab, n_hot, seg_i,
                                                                     seg_e, nseg, rw, part, redo, s);
        if (e != hipSuccess) return e;
        return a.pack == Pack::U16 ? pull_t<0, false, true, uint16_t>(a, nnz, row_ptr, col, val, hotlab, n_hot, seg_i,
                                                                      seg_e, nseg, rw, part, redo, s)
                                   : pull_t<0, false, true, uint8_t>(a, nnz, row_ptr, col, val, hotlab, n_hot, seg_i,
                                                                     seg_e, nseg, rw, part, redo, s);
    }
    if (a.pack == Pack::U16) return GEE_PULL(kUnitBins, false, false, uint16_t);
    return a.hot6 ? pull_t<kUnitBins, false, false, uint8_t, true>(a, nnz, row_ptr, col, val, hotlab, n_hot, seg_i,
                                                                  seg_e, nseg, rw, part, nullptr, s)
                  : GEE_PULL(kUnitBins, false, false, uint8_t);
#undef GEE_PULL
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

hipError_t launch_pack_hot(const EmbedArgs &a, const int32_t *hot_ids, int64_t n_hot, void *hotlab, hipStream_t s)
{
    if (n_hot <= 0) return hipSuccess;
    const dim3 g(grid_for(n_hot, kBlock, 1 << 20)), b(kBlock);
    if (a.hot6)
        hipLaunchKernelGGL(k_pack_hot6, dim3(grid_for((n_hot + 4) / 5, kBlock, 1 << 20)), b, 0, s,
                           static_cast<const uint8_t *>(a.lab), a.n, hot_ids, n_hot, static_cast<uint32_t *>(hotlab),
                           a.err);
    else if (a.pack == Pack::U8)
        hipLaunchKernelGGL(k_pack_hot<uint8_t>, g, b, 0, s, static_cast<const uint8_t *>(a.lab), a.n, hot_ids, n_hot,
                           static_cast<uint8_t *>(hotlab), a.err);
    else if (a.pack == Pack::U16)
        hipLaunchKernelGGL(k_pack_hot<uint16_t>, g, b, 0, s, static_cast<const uint16_t *>(a.lab), a.n, hot_ids,
                           n_hot, static_cast<uint16_t *>(hotlab), a.err);
    else
        hipLaunchKernelGGL(k_pack_hot<uint64_t>, g, b, 0, s, static_cast<const uint64_t *>(a.lab), a.n, hot_ids,
                           n_hot, static_cast<uint64_t *>(hotlab), a.err);
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
