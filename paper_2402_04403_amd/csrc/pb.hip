// Propagation-blocked pull pass for unit-weight adjacency embeddings, gfx950.
//
// Algorithm 1 (Section II) with unit weights adds, for every entry (u, v) of the
// symmetric adjacency, one count into Z(u, Y(v)); the class weights are applied
// once per element. The plain pull pass reads Y(v) at a random address for every
// entry, and on graphs whose label table is far larger than L2 most of those reads
// fill a 128-byte line for one byte. Here the gather and the accumulation are two
// streaming passes over a per-graph re-layout of the CSR entries:
//
//   layout (per graph): the entries sorted stably by column block (2^21 vertices),
//     so within a block they stay in (row, column) order. A cell is the run of one
//     column block's entries that belong to one block of 256 rows. Stored: the
//     column of every entry, its row within the 256-row block (8 bits), and for each
//     (row block, column block) the cell's start and length.
//   gather (per call): walk the entries in that order and write the 8-bit label of
//     each entry's column; one column block's labels are 2 MB, so consecutive work
//     reads them from L2.
//   rows (per call): one workgroup per 256-row block reads the block's cells (one
//     run per column block), counts (row, class) in LDS bins and writes its rows of Z
//     once, count * 1/n_k.
//
// Counts are integers, so the result is independent of order and bit-identical to
// the pull pass.

#include "common.h"
#include "launch.h"

namespace gee {

namespace {

constexpr int kT = 256;
constexpr int64_t kPbRows = (int64_t)1 << kPbRowBits;

inline int grid_cap(int64_t items, int per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

// mark[row_ptr[u]] = u for every row with entries (mark zero-filled before); an
// inclusive max-scan then gives every entry its row.
__global__ void __launch_bounds__(kT) k_pb_mark(int64_t n, const int64_t *__restrict__ row_ptr, int64_t *mark)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = row_ptr[u];
        if (a < row_ptr[u + 1]) mark[a] = u;
    }
}

// keys[e] = (column << 32) | row, in place over the rows; hot-slot columns decoded.
__global__ void __launch_bounds__(kT)
k_pb_key(int64_t nnz, int64_t n, const int32_t *__restrict__ col, const int32_t *__restrict__ hot_ids, int64_t n_hot,
         uint64_t *keys, int32_t *err)
{
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = col[e];
        if (c < 0) {
            const int64_t slot = (int64_t)((uint32_t)c & 0x7fffffffu);
            c = slot < n_hot ? hot_ids[slot] : -1;
        }
        if ((uint64_t)c >= (uint64_t)n) {
            bad = true;
            c = 0;
        }
        keys[e] = ((uint64_t)c << 32) | (keys[e] & 0xffffffffull);
    }
    if (bad) flag_error(err, GEE_EVERTEX);
}

__device__ inline int64_t pb_cell(uint64_t key, int64_t n_rb)
{
    return (int64_t)(key >> (32 + kPbColBits)) * n_rb + (int64_t)((key & 0xffffffffull) >> kPbRowBits);
}

// colc / ul from the sorted keys; celllast[cell] = index + 1 of the cell's last entry.
__global__ void __launch_bounds__(kT)
k_pb_finalize(const uint64_t *__restrict__ keys, int64_t nnz, int64_t n_rb, int32_t *__restrict__ colc,
              uint8_t *__restrict__ ul, int64_t *__restrict__ celllast)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        colc[i] = (int32_t)(k >> 32);
        ul[i] = (uint8_t)(k & (kPbRows - 1));
        const int64_t cell = pb_cell(k, n_rb);
        if (i + 1 == nnz || pb_cell(keys[i + 1], n_rb) != cell) celllast[cell] = i + 1;
    }
}

// Row-block-major table: cell (rb, cb) starts where cell (cb, rb) - 1 of the sorted
// (column-block-major) order ends.
__global__ void __launch_bounds__(kT)
k_pb_table(int64_t n_rb, int32_t n_cb, const int64_t *__restrict__ cellend, int64_t *__restrict__ cell_start,
           uint32_t *__restrict__ cell_count)
{
    const int64_t cells = n_rb * n_cb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rb = i / n_cb, cb = i - rb * n_cb;
        const int64_t c = cb * n_rb + rb;
        const int64_t a = c == 0 ? 0 : cellend[c - 1];
        cell_start[i] = a;
        cell_count[i] = (uint32_t)(cellend[c] - a);
    }
}

// yv[i] = lab[colc[i]], 16 entries per thread with 16-byte loads of columns and one
// 16-byte store of labels.
__global__ void __launch_bounds__(kT)
k_pb_gather(int64_t nnz, const int32_t *__restrict__ colc, const uint8_t *__restrict__ lab, uint8_t *__restrict__ yv)
{
    const int64_t nvec = nnz / 16;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += (int64_t)gridDim.x * blockDim.x) {
        const int4 *cp = reinterpret_cast<const int4 *>(colc + v * 16);
        int4 c4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c4[q] = cp[q];
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[q] = (uint32_t)lab[c4[q].x] | ((uint32_t)lab[c4[q].y] << 8) | ((uint32_t)lab[c4[q].z] << 16) |
                   ((uint32_t)lab[c4[q].w] << 24);
        *reinterpret_cast<uint4 *>(yv + v * 16) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    for (int64_t i = nvec * 16 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
         i += (int64_t)gridDim.x * blockDim.x)
        yv[i] = lab[colc[i]];
}

constexpr int kPbCells = 4;    // cells a wavefront reads at once

// One workgroup per 256-row block. Wavefront w takes the block's cells w, w + 4,
// ..., four at a time: its lanes cover the cells' entries (row within the block and
// label, both coalesced) so the loads of four cells are in flight together. One
// count per entry into LDS bins [row][class], then the rows of Z are written once
// (count * 1/n_k).
__global__ void __launch_bounds__(kT)
k_pb_rows(int64_t n, int32_t K, uint64_t magicK, int32_t n_cb, const int64_t *__restrict__ cell_start,
          const uint32_t *__restrict__ cell_count, const uint8_t *__restrict__ ul, const uint8_t *__restrict__ yv,
          const double *__restrict__ inv, float *__restrict__ Z)
{
    // LDS: bins [kPbRows * K] uint32, inv [K] double, cell starts [n_cb] int64, counts [n_cb]
    extern __shared__ __align__(16) uint32_t bins[];
    double *invs = reinterpret_cast<double *>(bins + align_up((size_t)kPbRows * K, 2));
    int64_t *cst = reinterpret_cast<int64_t *>(invs + K);
    uint32_t *ccn = reinterpret_cast<uint32_t *>(cst + n_cb);
    const int64_t rb = blockIdx.x;
    const int64_t r0 = rb * kPbRows;
    const int nr = (int)((n - r0) < kPbRows ? (n - r0) : kPbRows);
    const int t = threadIdx.x, lane = t % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(t / kWave);
    constexpr int kWaves = kT / kWave;
    for (int i = t; i < kPbRows * K; i += kT) bins[i] = 0;
    for (int k = t; k < K; k += kT) invs[k] = inv[k + 1];
    for (int c = t; c < n_cb; c += kT) {
        cst[c] = cell_start[rb * n_cb + c];
        ccn[c] = cell_count[rb * n_cb + c];
    }
    __syncthreads();
    for (int c0 = wave; c0 < n_cb; c0 += kWaves * kPbCells) {
        int64_t a[kPbCells];
        uint32_t m[kPbCells], mmax = 0;
#pragma unroll
        for (int j = 0; j < kPbCells; ++j) {
            const int c = c0 + j * kWaves;
            a[j] = c < n_cb ? cst[c] : 0;
            m[j] = c < n_cb ? ccn[c] : 0u;
            mmax = m[j] > mmax ? m[j] : mmax;
        }
        for (uint32_t q = lane; q < mmax; q += kWave) {
            uint32_t u[kPbCells], y[kPbCells];
#pragma unroll
            for (int j = 0; j < kPbCells; ++j) {
                const bool ok = q < m[j];
                u[j] = ok ? ul[a[j] + q] : 0u;
                y[j] = ok ? yv[a[j] + q] : 0u;
            }
#pragma unroll
            for (int j = 0; j < kPbCells; ++j)
                if (y[j] != 0) atomicAdd(&bins[u[j] * (uint32_t)K + (y[j] - 1)], 1u);
        }
    }
    __syncthreads();
    float *zb = Z + r0 * K;
    const uint32_t total = (uint32_t)nr * (uint32_t)K;
    for (uint32_t f = t; f < total; f += kT) {
        const uint32_t row = div_small(f, magicK);
        const uint32_t k = f - row * (uint32_t)K;
        __builtin_nontemporal_store((float)((double)bins[f] * invs[k]), zb + f);
    }
}

} // namespace

PbLayout pb_layout(int64_t n)
{
    PbLayout L;
    L.n_rb = (n + kPbRows - 1) / kPbRows;
    L.n_cb = (int32_t)((n + ((int64_t)1 << kPbColBits) - 1) >> kPbColBits);
    if (L.n_cb < 1) L.n_cb = 1;
    L.cells = L.n_rb * L.n_cb;
    return L;
}

// Build scratch: two key buffers [nnz], radix histograms, scan partials, two cell arrays.
size_t pb_build_scratch(int64_t n, int64_t nnz)
{
    const PbLayout L = pb_layout(n);
    size_t hb, ob, pbytes;
    radix_scratch_bytes(nnz, nnz > L.cells ? nnz : L.cells, &hb, &ob, &pbytes);
    size_t off = 0;
    auto take = [&](size_t b) {
        off = align_up(off, 256);
        off += b;
    };
    take((size_t)nnz * 8);
    take((size_t)nnz * 8);
    take(hb);
    take(ob);
    take(pbytes);
    take((size_t)L.cells * 8);
    take((size_t)L.cells * 8);
    return align_up(off, 256);
}

hipError_t launch_pb_build(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const int32_t *hot_ids,
                           int64_t n_hot, int32_t *colc, uint8_t *ul, int64_t *cell_start, uint32_t *cell_count,
                           void *ws, int32_t *err, hipStream_t s)
{
    const PbLayout L = pb_layout(n);
    size_t hb, ob, pbytes;
    radix_scratch_bytes(nnz, nnz > L.cells ? nnz : L.cells, &hb, &ob, &pbytes);
    char *base = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t b) {
        off = align_up(off, 256);
        char *p = base + off;
        off += b;
        return p;
    };
    uint64_t *k0 = (uint64_t *)take((size_t)nnz * 8);
    uint64_t *k1 = (uint64_t *)take((size_t)nnz * 8);
    uint32_t *hist = (uint32_t *)take(hb);
    int64_t *offs = (int64_t *)take(ob);
    int64_t *part = (int64_t *)take(pbytes);
    int64_t *celllast = (int64_t *)take((size_t)L.cells * 8);
    int64_t *cellend = (int64_t *)take((size_t)L.cells * 8);
    hipError_t e;
    const dim3 b(kT);
    if (nnz > 0) {
        // row of every entry, then (column << 32) | row
        if ((e = launch_fill_i64(reinterpret_cast<int64_t *>(k1), nnz, 0, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_pb_mark, dim3(grid_cap(n, kT * 4)), b, 0, s, n, row_ptr, reinterpret_cast<int64_t *>(k1));
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = max_scan_i64(reinterpret_cast<const int64_t *>(k1), nnz, reinterpret_cast<int64_t *>(k0), part, s)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_pb_key, dim3(grid_cap(nnz, kT * 4)), b, 0, s, nnz, n, col, hot_ids, n_hot, k0, err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // stable sort on the column-block bits (the entries are in row order already)
        uint64_t *sorted = k0;
        if (L.n_cb > 1) {
            int hi = 32 + kPbColBits;
            while (hi < 64 && ((int64_t)1 << (hi - 32 - kPbColBits)) < L.n_cb) ++hi;
            if ((e = radix_sort_bits(k0, k1, nnz, 32 + kPbColBits, hi, hist, offs, part, &sorted, s)) != hipSuccess)
                return e;
        }
        if ((e = launch_fill_i64(celllast, L.cells, 0, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_pb_finalize, dim3(grid_cap(nnz, kT * 4)), b, 0, s, sorted, nnz, L.n_rb, colc, ul,
                           celllast);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        if ((e = launch_fill_i64(celllast, L.cells, 0, s)) != hipSuccess) return e;
    }
    if ((e = max_scan_i64(celllast, L.cells, cellend, part, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pb_table, dim3(grid_cap(L.cells, kT * 4)), b, 0, s, L.n_rb, L.n_cb, cellend, cell_start,
                       cell_count);
    return hipGetLastError();
}

hipError_t launch_pb_gather(int64_t nnz, const int32_t *colc, const uint8_t *lab, uint8_t *yv, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pb_gather, dim3(grid_cap(nnz, kT * 16)), dim3(kT), 0, s, nnz, colc, lab, yv);
    return hipGetLastError();
}

hipError_t launch_pb_rows(int64_t n, int32_t K, const PbLayout &L, const int64_t *cell_start,
                          const uint32_t *cell_count, const uint8_t *ul, const uint8_t *yv, const double *inv, float *Z,
                          hipStream_t s)
{
    const size_t lds = align_up((size_t)kPbRows * K, 2) * 4 + (size_t)K * 8 + (size_t)L.n_cb * 12;
    const uint64_t magic = ((1ull << 32) + (uint64_t)K - 1) / (uint64_t)K;
    hipLaunchKernelGGL(k_pb_rows, dim3((unsigned)L.n_rb), dim3(kT), lds, s, n, K, magic, L.n_cb, cell_start,
                       cell_count, ul, yv, inv, Z);
    return hipGetLastError();
}

} // namespace gee
