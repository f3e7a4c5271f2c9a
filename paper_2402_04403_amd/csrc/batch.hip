// Batched GEE on gfx950: many label vectors embedded over one graph in one pass
// of the CSR.
//
// Algorithm 1 (Section II of the paper) is a single pass over the edges for one
// label vector. For B vectors on the same graph the pass is shared: the vectors
// of a group (up to 64, all adjacency or all Laplacian) are stored transposed, one
// row of 16-bit labels per vertex, so one gather of a neighbour's label row (one
// 128-byte line for 64 vectors) serves every vector of the group. A block of 256
// threads owns a segment of the merge-path split (rows + entries), accumulates the
// bins of a window of rows for all vectors of the group in LDS, and writes each
// row's group columns of Z once. Rows cut by segment boundaries are summed from
// FP64 partials in segment order, as in the single-vector pull pass.

#include "common.h"
#include "launch.h"

namespace gee {

namespace {

constexpr int kBT = 256;               // threads per block
constexpr int kMaxGroup = 64;          // vectors per group
constexpr size_t kBatchLds = 48 * 1024; // bins of a window (per block)

inline int grid_cap(int64_t items, int per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

// labmat[v * Gs + b] = label of vertex v in vector b of the group (0 for a label
// outside [0, K_b] and for the padding columns b >= G). A 64 x 64 tile goes
// through LDS so both the read (along v) and the write (along b) are coalesced.
__global__ void __launch_bounds__(kBT)
k_pack_group(const int32_t *__restrict__ labels, int64_t n, GroupDesc d, uint16_t *__restrict__ labmat, int32_t *err)
{
    __shared__ uint16_t tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    bool bad = false;
    for (int b = ty; b < d.Gs; b += kBT / 64) {
        const int64_t v = v0 + tx;
        uint16_t y = 0;
        if (v < n && b < d.G) {
            const int32_t x = labels[(int64_t)d.vec[b] * n + v];
            const bool ok = (uint32_t)x <= (uint32_t)d.K[b];
            bad |= !ok;
            y = ok ? (uint16_t)x : 0;
        }
        tile[tx][b] = y;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += kBT / 64) {
        const int64_t v = v0 + r;
        if (v < n && tx < d.Gs) labmat[v * d.Gs + tx] = tile[r][tx];
    }
    if (bad) flag_error(err, GEE_ELABEL);
}

// scale[coff_b + k] = 1 / n_{b,k+1} for the group's columns (inv tables of each vector).
__global__ void k_group_scale(const double *__restrict__ inv_all, GroupDesc d, double *__restrict__ scale)
{
    const int b = blockIdx.x;
    if (b >= d.G) return;
    for (int k = threadIdx.x; k < d.K[b]; k += blockDim.x) scale[d.coff[b] + k] = inv_all[d.inv_off[b] + k + 1];
}

struct BatchSeg {
    int64_t i0, i1, e0, e1;
    bool carried, tail;
    int64_t rend;
};

__device__ inline BatchSeg batch_seg(int64_t j, int64_t n, const int64_t *__restrict__ row_ptr,
                                     const int32_t *__restrict__ seg_i, const int64_t *__restrict__ seg_e)
{
    BatchSeg s;
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

template <bool WIDE> struct GBins;
template <> struct GBins<false> { // unit-weight adjacency: integer counts
    using word = uint32_t;
    __device__ static void add(word *p, double) { atomicAdd(p, 1u); }
};
template <> struct GBins<true> { // weighted or Laplacian: FP64 sums
    using word = double;
    __device__ static void add(word *p, double x) { atomicAdd(p, x); }
};

// One block per segment. The window's rows have bins [RW][KT] in LDS (KT = sum of
// K_b over the group). Each thread takes one entry at a time: it finds the entry's
// row by a binary search over the window's row starts, gathers the neighbour's
// label row (G 16-bit labels, 16 bytes per load) and adds 1 (or w, times the
// neighbour's d^-1/2 for a Laplacian group) into bin (row, col_off[b] + y_b - 1)
// for every vector b with y_b > 0.
template <bool WIDE, bool LAP, bool W>
__global__ void __launch_bounds__(kBT)
k_pull_group(int64_t n, int64_t nnz, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
             const float *__restrict__ val, const int32_t *__restrict__ hot_ids, int64_t n_hot,
             const uint16_t *__restrict__ labmat, GroupDesc d, const double *__restrict__ scale, const float *__restrict__ rsd, const int32_t *__restrict__ seg_i,
             const int64_t *__restrict__ seg_e, int64_t nseg, int RW, float *__restrict__ Z, int64_t ldz,
             int64_t zcol, double *__restrict__ part, int32_t *err)
{
    using word = typename GBins<WIDE>::word;
    extern __shared__ __align__(16) unsigned char smem[];
    word *bins = (word *)smem;
    const int KT = d.KT, G = d.G;
    int32_t *cs = (int32_t *)(smem + align_up((size_t)RW * KT * sizeof(word), 16));
    int32_t *coff = cs + (kMaxGroup + 2);
    const int t = threadIdx.x;
    const int64_t j = blockIdx.x;
    if (j >= nseg) return;
    const BatchSeg sg = batch_seg(j, n, row_ptr, seg_i, seg_e);
    for (int b = t; b < G; b += kBT) coff[b] = d.coff[b];
    for (int i = t; i < RW * KT; i += kBT) bins[i] = (word)0;
    __syncthreads();
    bool bad = false;

    for (int64_t r = sg.i0; r < sg.rend; r += RW) {
        const int nr = (int)((sg.rend - r) < RW ? (sg.rend - r) : RW);
        if (t <= nr) {
            int64_t p = row_ptr[r + t];
            p = p < sg.e0 ? sg.e0 : (p > sg.e1 ? sg.e1 : p);
            cs[t] = (int32_t)(p - sg.e0);
        }
        __syncthreads();
        const int32_t ws = cs[0], we = cs[nr];
        for (int32_t q = ws + t; q < we; q += kBT) {
            int lo = 0, hi = nr; // cs[lo] <= q < cs[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (cs[mid] <= q) lo = mid;
                else hi = mid;
            }
            const int64_t e = sg.e0 + q;
            int32_t c = col[e];
            if (c < 0) {
                const int64_t slot = (int64_t)((uint32_t)c & 0x7fffffffu);
                c = slot < n_hot ? hot_ids[slot] : -1;
            }
            if ((uint32_t)c >= (uint64_t)n) {
                bad = true;
                continue;
            }
            double inc = W ? (double)val[e] : 1.0;
            if (LAP) inc *= (double)rsd[c];
            word *rowbins = bins + (size_t)lo * KT;
            const uint16_t *lr = labmat + (int64_t)c * d.Gs;
            for (int b0 = 0; b0 < G; b0 += 8) {
                // eight 16-bit labels per 16-byte load (rows padded to a multiple of 8 labels)
                const uint4 q4 = *reinterpret_cast<const uint4 *>(lr + b0);
                const uint32_t wv[4] = {q4.x, q4.y, q4.z, q4.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int b = b0 + i;
                    const uint32_t y = (wv[i >> 1] >> (16 * (i & 1))) & 0xffffu;
                    if (b < G && y > 0) GBins<WIDE>::add(&rowbins[coff[b] + (int)y - 1], inc);
                }
            }
        }
        __syncthreads();
        // write the window's rows: group columns [zcol, zcol + KT) of each row
        const bool head_here = sg.carried && r == sg.i0;
        const bool tail_here = sg.tail && sg.i1 >= r && sg.i1 < r + nr;
        for (int l = 0; l < nr; ++l) {
            const int64_t u = r + l;
            const bool head = head_here && l == 0, tail = tail_here && u == sg.i1;
            const double ru = LAP ? (double)rsd[u] : 1.0;
            for (int f = t; f < KT; f += kBT) {
                const double x = (double)bins[(size_t)l * KT + f];
                if (head) part[(2 * j) * KT + f] = x;
                else if (tail) part[(2 * j + 1) * KT + f] = x;
                else __builtin_nontemporal_store((float)(x * (scale[f] * ru)), &Z[u * ldz + zcol + f]);
            }
        }
        __syncthreads();
        for (int i = t; i < nr * KT; i += kBT) bins[i] = (word)0;
        __syncthreads();
    }
    if (bad) flag_error(err, GEE_EVERTEX);
}

// Rows cut by segment boundaries: tail partial of the start segment plus the head
// partials of the following segments, in segment order; scaled and written once.
template <bool LAP>
__global__ void __launch_bounds__(kBT)
k_merge_group(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ seg_i,
              const int64_t *__restrict__ seg_e, int64_t nseg, int KT, const double *__restrict__ scale,
              const float *__restrict__ rsd, const double *__restrict__ part, float *__restrict__ Z, int64_t ldz,
              int64_t zcol)
{
    const int64_t j = blockIdx.x;
    if (j >= nseg) return;
    const BatchSeg sg = batch_seg(j, n, row_ptr, seg_i, seg_e);
    if (!sg.tail) return;
    const int64_t u = sg.i1;
    const double ru = LAP ? (double)rsd[u] : 1.0;
    for (int f = threadIdx.x; f < KT; f += blockDim.x) {
        double acc = part[(2 * j + 1) * KT + f];
        for (int64_t jj = j + 1; jj < nseg; ++jj) {
            acc += part[(2 * jj) * KT + f];
            if (seg_i[jj + 1] > u) break;
        }
        Z[u * ldz + zcol + f] = (float)(acc * (scale[f] * ru));
    }
}

__global__ void k_rsd(const double *__restrict__ deg, int64_t n, float *__restrict__ rsd)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const double d = deg[v];
        rsd[v] = d > 0.0 ? (float)(1.0 / sqrt(d)) : 0.0f;
    }
}

} // namespace

size_t batch_window_bytes(int KT, bool wide, int rw)
{
    return align_up((size_t)rw * KT * (wide ? 8 : 4), 16) + (size_t)(2 * kMaxGroup + 4) * 4;
}

int batch_rows_per_window(int KT, bool wide)
{
    int rw = 64;
    while (rw > 1 && batch_window_bytes(KT, wide, rw) > kBatchLds) --rw;
    return batch_window_bytes(KT, wide, rw) <= 65536 ? rw : 0;
}

hipError_t launch_pack_group(const int32_t *labels, int64_t n, const GroupDesc &d, uint16_t *labmat, int32_t *err,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_group, dim3((unsigned)((n + 63) / 64)), dim3(kBT), 0, s, labels, n, d, labmat, err);
    return hipGetLastError();
}

hipError_t launch_group_scale(const double *inv_all, const GroupDesc &d, double *scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_group_scale, dim3(d.G), dim3(256), 0, s, inv_all, d, scale);
    return hipGetLastError();
}

hipError_t launch_rsd(const double *deg, int64_t n, float *rsd, hipStream_t s)
{
    hipLaunchKernelGGL(k_rsd, dim3(grid_cap(n, 256 * 4)), dim3(256), 0, s, deg, n, rsd);
    return hipGetLastError();
}

hipError_t launch_pull_group(const GroupArgs &g, hipStream_t s)
{
    const bool wide = g.lap || g.val;
    const size_t lds = batch_window_bytes(g.d.KT, wide, g.rw);
#define GEE_GROUP(WIDE, LAP, W)                                                                                      \
    hipLaunchKernelGGL((k_pull_group<WIDE, LAP, W>), dim3((unsigned)g.nseg), dim3(kBT), lds, s, g.n, g.nnz, g.row_ptr, \
                       g.col, g.val, g.hot_ids, g.n_hot, g.labmat, g.d, g.scale, g.rsd, g.seg_i, g.seg_e, g.nseg,    \
                       g.rw, g.Z, g.ldz, g.zcol, g.part, g.err)
    if (g.lap) {
        if (g.val) GEE_GROUP(true, true, true);
        else GEE_GROUP(true, true, false);
    } else {
        if (g.val) GEE_GROUP(true, false, true);
        else GEE_GROUP(false, false, false);
    }
#undef GEE_GROUP
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.lap)
        hipLaunchKernelGGL(k_merge_group<true>, dim3((unsigned)g.nseg), dim3(kBT), 0, s, g.n, g.row_ptr, g.seg_i,
                           g.seg_e, g.nseg, g.d.KT, g.scale, g.rsd, g.part, g.Z, g.ldz, g.zcol);
    else
        hipLaunchKernelGGL(k_merge_group<false>, dim3((unsigned)g.nseg), dim3(kBT), 0, s, g.n, g.row_ptr, g.seg_i,
                           g.seg_e, g.nseg, g.d.KT, g.scale, g.rsd, g.part, g.Z, g.ldz, g.zcol);
    return hipGetLastError();
}

} // namespace gee
