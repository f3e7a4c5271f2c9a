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
//     so within a block they stay in (row, column) order. Entries whose column is one
//     of the first n_lds hot slots of the CSR (its highest-degree vertices) go to
//     extra column blocks after the vertex blocks, one per "tier slice" of 2^17 slots,
//     and keep their slot within the slice instead of the vertex. A cell is the run of
//     one column block's entries that belong to one block of 256 rows. Stored: the
//     column of every vertex-block entry (32 bits), the slot of every tier entry (17
//     bits: 16 in place, the 17th in a bit array), its row within the 256-row block (8
//     bits), and for each (row
//     block, column block) the cell's start and length. The tier entries start at H0,
//     the first multiple of 16 at or after the last vertex-block entry; the gap of
//     fewer than 16 entries before it belongs to no cell (its columns are 0).
//   gather (per call): walk the entries in that order and write the 8-bit label of
//     each entry's column. One vertex column block's labels are 2 MB, so consecutive
//     work reads them from L2, one L2 request per entry. The tier's entries are read
//     against one slice's labels (128 KB) held in LDS by the workgroup, so on a
//     power-law graph most entries cost no L2 request at all.
//   rows (per call): one workgroup per 256-row block reads the block's cells as one
//     flattened run of 32-bit words (four entries a word, each lane its own words),
//     counts (row, class) in LDS bins and writes its rows of Z once, count * 1/n_k.
//
// Counts are integers, so the result is independent of order and bit-identical to
// the pull pass.

#include <limits.h>

#include "common.h"
#include "launch.h"

namespace gee {

namespace {

constexpr int kT = 256;
constexpr int kRowsT = 512;    // rows kernel: 8 wavefronts per 256-row block (16 when its LDS allows two)
constexpr int kRowsU = 4;      // words per lane in flight in the rows kernel
constexpr int kLdsT = 1024;    // LDS-tier gather: 16 wavefronts share one label table
constexpr uint32_t kXcds = 8;  // accelerator dies, each with its own L2
constexpr int64_t kPbRows = (int64_t)1 << kPbRowBits;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

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

// keys[e] = (column << 32) | row, in place over the rows. Hot slot q below n_lds gets
// the key column ((n_vcb + q / 2^17) << 21) | (q mod 2^17): column block n_vcb + slice;
// other hot slots are decoded.
__global__ void __launch_bounds__(kT)
k_pb_key(int64_t nnz, int64_t n, const int32_t *__restrict__ col, const int32_t *__restrict__ hot_ids, int64_t n_hot,
         int64_t n_lds, int32_t n_vcb, uint64_t *keys, int32_t *err)
{
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c0 = col[e];
        uint64_t kc;
        if (c0 < 0) {
            const int64_t slot = (int64_t)((uint32_t)c0 & 0x7fffffffu);
            if (slot < n_lds) {
                kc = ((uint64_t)(n_vcb + (slot >> kPbSliceBits)) << kPbColBits) | (uint64_t)(slot & (kPbSlice - 1));
            } else {
                const int64_t c = slot < n_hot ? hot_ids[slot] : -1;
                if ((uint64_t)c >= (uint64_t)n) bad = true;
                kc = (uint64_t)c < (uint64_t)n ? (uint64_t)c : 0;
            }
        } else {
            if (c0 >= n) bad = true;
            kc = c0 < n ? (uint64_t)c0 : 0;
        }
        keys[e] = (kc << 32) | (keys[e] & 0xffffffffull);
    }
    if (bad) flag_error(err, GEE_EVERTEX);
}

__device__ inline int64_t pb_cell(uint64_t key, int64_t n_rb)
{
    return (int64_t)(key >> (32 + kPbColBits)) * n_rb + (int64_t)((key & 0xffffffffull) >> kPbRowBits);
}

// tier[0] = h0, the number of vertex-block entries (the first sorted key whose column
// block is a tier slice, by binary search); tier[1] = H0, h0 rounded up to 16.
__global__ void k_pb_tier_start(const uint64_t *__restrict__ keys, int64_t nnz, int32_t n_vcb, int64_t *tier)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((keys[mid] >> (32 + kPbColBits)) >= (uint64_t)n_vcb) hi = mid;
        else lo = mid + 1;
    }
    tier[0] = lo;
    tier[1] = (lo + 15) & ~(int64_t)15;
}

// Layout arrays from the sorted keys. Sorted index i goes to o = i before h0 and to
// i + (H0 - h0) from h0 on. A vertex-block entry stores its column in colc[o]; a tier
// entry stores the low 16 bits of its slot within the slice at colb[4 H0 + 2 (o - H0)]
// (16-bit, little-endian; the 17th bit is written by k_pb_tier_hi). ul[o]
// is the row within its block; celllast[cell] = o + 1 for a cell's last entry. The gap
// [h0, H0) gets column 0 and row 0. tier = {h0, H0} (null: no tier, h0 = H0 = nnz).
__global__ void __launch_bounds__(kT)
k_pb_finalize(const uint64_t *__restrict__ keys, const float *__restrict__ sval, int64_t nnz, int64_t n_rb,
              int32_t n_vcb, const int64_t *__restrict__ tier, int32_t *__restrict__ colc, uint8_t *__restrict__ colb,
              uint8_t *__restrict__ ul, float *__restrict__ vl, int64_t *__restrict__ celllast)
{
    const int64_t h0 = tier ? tier[0] : nnz, H0 = tier ? tier[1] : nnz;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gs = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gt; i < nnz; i += gs) {
        const uint64_t k = keys[i];
        const uint64_t c = k >> 32;
        const int64_t o = i < h0 ? i : i + (H0 - h0);
        if (vl) vl[o] = sval[i];
        if (i < h0) {
            colc[o] = (int32_t)c;
        } else {
            // the slot's low 16 bits (its 17th bit goes to the tier's bit array, k_pb_tier_hi)
            reinterpret_cast<uint16_t *>(colb + 4 * H0)[o - H0] = (uint16_t)c;
        }
        ul[o] = (uint8_t)(k & (kPbRows - 1));
        const int64_t cell = pb_cell(k, n_rb);
        if (i + 1 == nnz || pb_cell(keys[i + 1], n_rb) != cell) celllast[cell] = o + 1;
    }
    for (int64_t i = h0 + gt; i < H0; i += gs) {
        colc[i] = 0;
        ul[i] = 0;
        if (vl) vl[i] = 0.0f;
    }
}

// The tier's bit array: bit r of it is the 17th bit of tier entry H0 + r's slot. The
// tier's NT = nnz - h0 entries are padded to NTp, a multiple of 64; their low halves take
// bytes [4 H0, 4 H0 + 2 NTp) of col and the bit array follows (8-byte aligned), NTp / 64
// words of 64 bits (padding bits 0). One entry per lane, one word per wavefront (ballot).
__global__ void __launch_bounds__(kT)
k_pb_tier_hi(const uint64_t *__restrict__ keys, int64_t nnz, const int64_t *__restrict__ tier, uint8_t *colb)
{
    const int64_t h0 = tier[0], H0 = tier[1];
    const int64_t NT = nnz - h0, NTp = (NT + 63) & ~(int64_t)63;
    uint64_t *bits = reinterpret_cast<uint64_t *>(colb + 4 * H0 + 2 * NTp);
    const int lane = threadIdx.x % kWave;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t ws = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t q = w0; q < NTp / 64; q += ws) { // uniform per wavefront
        const int64_t r = 64 * q + lane;
        const bool bit = r < NT && ((keys[h0 + (r < NT ? r : 0)] >> (32 + 16)) & 1u) != 0;
        const uint64_t m = __ballot(bit);
        if (lane == 0) bits[q] = m;
    }
}

// rb_flag[rb] = 1 when a row of 256-row block rb has more than kPbF32Terms entries or
// a weight that is not >= 0 (NaN included): such a block sums in FP64. One workgroup
// per block: thread t checks row 256 rb + t, then the block's entries are scanned with
// coalesced reads.
__global__ void __launch_bounds__(kT)
k_pb_rbflag(int64_t n, int64_t n_rb, const int64_t *__restrict__ row_ptr, const float *__restrict__ val,
            uint8_t *__restrict__ rb_flag)
{
    for (int64_t rb = blockIdx.x; rb < n_rb; rb += gridDim.x) {
        const int64_t r0 = rb * kPbRows, r1 = r0 + kPbRows < n ? r0 + kPbRows : n;
        const int64_t u = r0 + threadIdx.x;
        bool f = u < r1 && row_ptr[u + 1] - row_ptr[u] > kPbF32Terms;
        if (val)
            for (int64_t e = row_ptr[r0] + threadIdx.x; e < row_ptr[r1]; e += kT) f |= !(val[e] >= 0.0f);
        f = __syncthreads_or(f) != 0;
        if (threadIdx.x == 0) rb_flag[rb] = f ? 1 : 0;
        __syncthreads();
    }
}

// The layout's fingerprint: n, nnz, n_lds, weighted; meta[4] (the weights' grid) is
// filled in by k_pb_grid_final for a weighted layout.
__global__ void k_pb_meta(int64_t *meta, int64_t n, int64_t nnz, int64_t n_lds, int64_t weighted)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        meta[0] = n;
        meta[1] = nnz;
        meta[2] = n_lds;
        meta[3] = weighted;
        meta[4] = kPbNoGrid;
        meta[5] = meta[6] = meta[7] = 0;
    }
}

// The Laplacian layout's term of every CSR entry, in CSR order: w d_u^-1/2 d_v^-1/2 for its
// row u (the low half of its key) and column v (a hot-slot column decoded through
// hot_ids): the product of the FP32 weight and the two FP32 factors, taken in FP64 and
// rounded once to FP32. A column outside [0, n) gives 0 (k_pb_key flags it).
__global__ void __launch_bounds__(kT)
k_pb_lapw(int64_t nnz, int64_t n, const int32_t *__restrict__ col, const float *__restrict__ val,
          const int32_t *__restrict__ hot_ids, int64_t n_hot, const uint64_t *__restrict__ keys,
          const float *__restrict__ rsd, float *__restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c0 = col[e];
        int64_t v = c0;
        if (c0 < 0) {
            const int64_t slot = (int64_t)((uint32_t)c0 & 0x7fffffffu);
            v = slot < n_hot ? hot_ids[slot] : -1;
        }
        const int64_t u = (int64_t)(keys[e] & 0xffffffffull);
        const double rv = (uint64_t)v < (uint64_t)n ? (double)rsd[v] : 0.0;
        const double ru = (uint64_t)u < (uint64_t)n ? (double)rsd[u] : 0.0;
        out[e] = (float)((val ? (double)val[e] : 1.0) * ru * rv);
    }
}

__global__ void k_pb_grid_init(int32_t *ex)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ex[0] = INT_MAX;
        ex[1] = INT_MIN;
    }
}

// The binary exponents of the lowest and the highest set bit over the positive finite
// weights: ex[0] = min, ex[1] = max (ex starts at {INT_MAX, INT_MIN}).
__global__ void __launch_bounds__(kT)
k_pb_grid_bits(int64_t nnz, const float *__restrict__ val, int32_t *ex)
{
    int lo = INT_MAX, hi = INT_MIN;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const float w = val[e];
        if (!(w > 0.0f) || !(w < INFINITY)) continue; // zero, negative or not finite: not on the grid's path
        const uint32_t b = __float_as_uint(w), ef = b >> 23, m = b & 0x7fffffu;
        const uint32_t sig = ef ? (m | 0x800000u) : m;       // significand as an integer
        const int e0 = ef ? (int)ef - 150 : -149;            // its unit's exponent
        lo = min(lo, e0 + __builtin_ctz(sig));
        hi = max(hi, e0 + 31 - __builtin_clz(sig));
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        lo = min(lo, __shfl_down(lo, o, kWave));
        hi = max(hi, __shfl_down(hi, o, kWave));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMin(&ex[0], lo);
        atomicMax(&ex[1], hi);
    }
}

// meta[4] = g when every positive weight is a multiple of 2^-g and a sum of kPbF32Terms of
// them stays below 2^32 once scaled by 2^g (the row sums of an unflagged block then add
// exactly in 32-bit integers), else kPbNoGrid.
__global__ void k_pb_grid_final(const int32_t *ex, int64_t *meta)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int lo = ex[0], hi = ex[1];
    if (lo == INT_MAX) { // no positive weight: every sum is zero
        meta[4] = 0;
        return;
    }
    const int g = -lo; // scale 2^g: the lowest bit becomes bit 0
    const bool fits = g >= -126 && g <= 126 && hi + g + 8 <= 32; // (2^(hi+1) - 1) 2^g 2^7 < 2^32
    meta[4] = fits ? g : kPbNoGrid;
}

// Row-block-major table: cell (rb, cb) starts where cell (cb, rb) - 1 of the sorted
// (column-block-major) order ends, a tier cell no earlier than H0 (past the gap).
__global__ void __launch_bounds__(kT)
k_pb_table(int64_t n_rb, int32_t n_cb, int32_t n_vcb, const int64_t *__restrict__ tier,
           const int64_t *__restrict__ cellend, int64_t *__restrict__ cell_start, uint32_t *__restrict__ cell_count)
{
    const int64_t H0 = tier ? tier[1] : 0;
    const int64_t cells = n_rb * n_cb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rb = i / n_cb, cb = i - rb * n_cb;
        const int64_t c = cb * n_rb + rb;
        int64_t a = c == 0 ? 0 : cellend[c - 1];
        if (cb >= n_vcb && a < H0) a = H0;
        const int64_t e = cellend[c];
        cell_start[i] = a;
        cell_count[i] = (uint32_t)(e > a ? e - a : 0);
    }
}

// slice_entries[j] = entries whose column is one of hot slots [j 2^17, (j + 1) 2^17) (the
// row lengths of those vertices, the CSR being symmetric); one workgroup per slice.
__global__ void __launch_bounds__(kT)
k_pb_slice_entries(int64_t n_slots, const int32_t *__restrict__ hot_ids, const int64_t *__restrict__ row_ptr,
                   int64_t *__restrict__ slice_entries)
{
    __shared__ int64_t part[kT / kWave];
    const int64_t j = blockIdx.x;
    const int64_t a = j * kPbSlice, b = (j + 1) * kPbSlice < n_slots ? (j + 1) * kPbSlice : n_slots;
    int64_t sum = 0;
    for (int64_t q = a + threadIdx.x; q < b; q += kT) {
        const int64_t v = hot_ids[q];
        sum += row_ptr[v + 1] - row_ptr[v];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) sum += __shfl_down(sum, o, kWave);
    if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int w = 0; w < kT / kWave; ++w) tot += part[w];
        slice_entries[j] = tot;
    }
}

// cell_word[rb n_cb + c] = the first 32-bit word of cell c in row block rb's run of words
// (its cells one after another, each covering ceil(((start mod 4) + count) / 4) words,
// none when empty): one thread per row block.
__global__ void __launch_bounds__(kT)
k_pb_words(int64_t n_rb, int32_t n_cb, const int64_t *__restrict__ cell_start, const uint32_t *__restrict__ cell_count,
           uint32_t *__restrict__ cell_word)
{
    for (int64_t rb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; rb < n_rb; rb += (int64_t)gridDim.x * blockDim.x) {
        uint32_t run = 0;
        for (int32_t c = 0; c < n_cb; ++c) {
            const int64_t i = rb * n_cb + c;
            const uint32_t m = cell_count[i];
            cell_word[i] = run;
            run += m != 0u ? ((uint32_t)(cell_start[i] & 3) + m + 3u) >> 2 : 0u;
        }
    }
}

__device__ inline int64_t clamp_index(int64_t h, int64_t nnz) { return h < 0 ? 0 : (h > nnz ? nnz : h); }

// The layout's fingerprint (written by its build) against the fields of the gee_pb it
// came with. A layout built for another graph fails this, and every pass then skips its
// work and raises GEE_EVERTEX: its columns need not lie in [0, n) of these labels.
__device__ inline bool layout_matches(const int64_t *__restrict__ meta, int64_t n, int64_t nnz, int64_t n_lds,
                                      int kind, int32_t *err)
{
    const bool ok = meta[0] == n && meta[1] == nnz && meta[2] == n_lds && meta[3] == kind;
    if (!ok && threadIdx.x == 0 && blockIdx.x == 0) flag_error(err, GEE_EVERTEX);
    return ok;
}

// yv[i] = lab[colc[i]] over the entries with vertex columns [0, h0), 32 entries per
// thread: eight 16-byte loads of columns, their 32 label reads in flight together, and
// two 16-byte stores of labels (32 entries measured faster than 16 or 64). h0 is the
// first tier entry (*tier_start), or nnz without a tier (tier_start null). The columns
// are the layout's own, all in [0, n) once its fingerprint matches.
__global__ void __launch_bounds__(kT)
k_pb_gather(int64_t nnz, int64_t n, int64_t n_lds, int kind, const int64_t *__restrict__ meta,
            const int64_t *__restrict__ tier_start, const int32_t *__restrict__ colc, const uint8_t *__restrict__ lab,
            uint8_t *__restrict__ yv, int32_t *err)
{
    if (!layout_matches(meta, n, nnz, n_lds, kind, err)) return;
    const int64_t h0 = tier_start ? clamp_index(*tier_start, nnz) : nnz;
    const int64_t nvec = h0 / 32;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += (int64_t)gridDim.x * blockDim.x) {
        const int4 *cp = reinterpret_cast<const int4 *>(colc + v * 32);
        int4 c4[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) c4[q] = cp[q];
        uint32_t w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            w[q] = (uint32_t)lab[c4[q].x] | ((uint32_t)lab[c4[q].y] << 8) | ((uint32_t)lab[c4[q].z] << 16) |
                   ((uint32_t)lab[c4[q].w] << 24);
        uint4 *out = reinterpret_cast<uint4 *>(yv + v * 32);
        out[0] = make_uint4(w[0], w[1], w[2], w[3]);
        out[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
    for (int64_t i = nvec * 32 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < h0;
         i += (int64_t)gridDim.x * blockDim.x)
        yv[i] = lab[colc[i]];
}

// tab[q] = lab[lds_ids[q]] for the n_lds tier slots, zero-padded to a multiple of 16; a
// slot whose vertex is outside [0, n) gets label 0 and raises GEE_EVERTEX.
__global__ void __launch_bounds__(kT)
k_pb_tier_labels(int64_t n_lds, int64_t n, int64_t nnz, int kind, const int64_t *__restrict__ meta,
                 const int32_t *__restrict__ lds_ids, const uint8_t *__restrict__ lab, uint8_t *__restrict__ tab,
                 int32_t *err)
{
    if (!layout_matches(meta, n, nnz, n_lds, kind, err)) return;
    const int64_t padded = (n_lds + 15) / 16 * 16;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < padded; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = i < n_lds ? lds_ids[i] : 0;
        const bool ok = (uint64_t)(uint32_t)v < (uint64_t)n;
        bad |= !ok;
        tab[i] = (i < n_lds && ok) ? lab[v] : 0;
    }
    if (bad) flag_error(err, GEE_EVERTEX);
}

// The slot of tier entry i: its low 16 bits at colb[4 H0 + 2 (i - H0)], its 17th bit in
// the bit array at colb[hb] (bit i - H0).
__device__ inline uint32_t tier_slot(const uint8_t *colb, int64_t H0, const uint8_t *hb, int64_t i)
{
    const int64_t r = i - H0;
    return (uint32_t)reinterpret_cast<const uint16_t *>(colb + 4 * H0)[r] | ((uint32_t)((hb[r >> 3] >> (r & 7)) & 1u) << 16);
}

// yv[i] = (labels of slice j)[slot of i] over the tier entries [H0, E), where slice j's
// entries start at sl_start[j] (cell (0, n_vcb + j); sl_start[0] = H0, a multiple of 16)
// and E = cell_start + cell_count of the last cell. The range is cut into one chunk per
// workgroup (16-aligned); for every slice its chunk meets, the workgroup copies that
// slice's labels (at most kPbSlice bytes) into an LDS table of kPbSlice bytes and reads
// them there. Sixteen entries' slots are two 16-byte loads and one 2-byte load. Slots are
// masked to the table, so no LDS read leaves it.
__global__ void __launch_bounds__(kLdsT)
k_pb_gather_tier(int64_t nnz, int64_t n, int kind, const int64_t *__restrict__ meta, int32_t n_sl, int64_t n_lds,
                 const int64_t *__restrict__ sl_start, const int64_t *__restrict__ last_start,
                 const uint32_t *__restrict__ last_count, const uint8_t *__restrict__ colb,
                 const uint8_t *__restrict__ tab, uint8_t *__restrict__ yv, int32_t *err)
{
    extern __shared__ __align__(16) uint8_t stab[];
    if (!layout_matches(meta, n, nnz, n_lds, kind, err)) return;
    __shared__ int64_t bnd[kPbMaxSlices + 1];
    const int t = threadIdx.x;
    const int64_t lim = nnz + 16; // entries of the layout, gap included, are at most nnz + 15
    const int64_t E = clamp_index(*last_start + (int64_t)*last_count, lim);
    if (t <= n_sl) bnd[t] = t < n_sl ? clamp_index(sl_start[t], E) : E;
    __syncthreads();
    const int64_t H0 = bnd[0] & ~(int64_t)15; // a multiple of 16 by construction
    // the bit array after the low halves of the tier's E - H0 entries, padded to 64 (every
    // read stays below 4 (nnz + 16) + 200 bytes, inside col's nnz + 64 words)
    const uint8_t *hb = colb + 4 * H0 + 2 * ((E - H0 + 63) & ~(int64_t)63);
    const int64_t per = ((E - H0 + gridDim.x - 1) / gridDim.x + 15) & ~(int64_t)15;
    int64_t lo = H0 + (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < E ? lo + per : E;
    lo = lo > bnd[0] ? lo : bnd[0];
    if (lo >= hi) return; // the whole workgroup
    const uint32_t mask = (uint32_t)kPbSlice - 1;
    for (int j = 0; j < n_sl; ++j) {
        const int64_t a = lo > bnd[j] ? lo : bnd[j];
        const int64_t b = hi < bnd[j + 1] ? hi : bnd[j + 1];
        if (a >= b) continue; // the whole workgroup
        __syncthreads(); // the previous slice's reads are done
        const int64_t nj = n_lds - (int64_t)j * kPbSlice < kPbSlice ? n_lds - (int64_t)j * kPbSlice : kPbSlice;
        const uint4 *src = reinterpret_cast<const uint4 *>(tab + (int64_t)j * kPbSlice);
        for (int i = t; i < (int)((nj + 15) / 16); i += kLdsT) reinterpret_cast<uint4 *>(stab)[i] = src[i];
        __syncthreads();
        const int64_t v0 = (a + 15) / 16, v1 = b / 16;
        // entries 16 v .. 16 v + 15: their low halves, 32 bytes at 4 H0 + 2 (16 v - H0)
        // (16-byte aligned), and their 17th bits, 2 bytes at hb + 2 (v - H0 / 16). The slots
        // of a lane's next 16 entries are loaded before its current ones are looked up, so
        // two loads per lane are in flight while the LDS reads run.
        auto slots = [&](int64_t v, uint4 (&q)[2], uint32_t &h) {
            const int64_t g = v - H0 / 16;
            const uint4 *cp = reinterpret_cast<const uint4 *>(colb + 4 * H0) + 2 * g;
            q[0] = cp[0];
            q[1] = cp[1];
            h = reinterpret_cast<const uint16_t *>(hb)[g];
        };
        int64_t v = v0 + t;
        uint4 cur[2] = {};
        uint32_t ch = 0u;
        if (v < v1) slots(v, cur, ch);
        while (v < v1) {
            const int64_t vn = v + kLdsT;
            uint4 nxt[2] = {};
            uint32_t nh = 0u;
            if (vn < v1) slots(vn, nxt, nh);
            const uint32_t x[8] = {cur[0].x, cur[0].y, cur[0].z, cur[0].w, cur[1].x, cur[1].y, cur[1].z, cur[1].w};
            uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t slot = ((x[e / 2] >> (16 * (e % 2))) & 0xffffu) | (((ch >> e) & 1u) << 16);
                w[e / 4] |= (uint32_t)stab[slot & mask] << (8 * (e % 4));
            }
            *reinterpret_cast<uint4 *>(yv + v * 16) = make_uint4(w[0], w[1], w[2], w[3]);
#pragma unroll
            for (int i = 0; i < 2; ++i) cur[i] = nxt[i];
            ch = nh;
            v = vn;
        }
        // entries outside the 16-aligned run: the head [a, 16 v0) and the tail [16 v1, b)
        const int64_t head_end = v0 * 16 < b ? v0 * 16 : b;
        for (int64_t i = a + t; i < head_end; i += kLdsT) yv[i] = stab[tier_slot(colb, H0, hb, i) & mask];
        const int64_t tail_begin = v1 * 16 > head_end ? v1 * 16 : head_end;
        for (int64_t i = tail_begin + t; i < b; i += kLdsT) yv[i] = stab[tier_slot(colb, H0, hb, i) & mask];
    }
}

// One workgroup of NT threads (512, or 1024 when fewer than three of 512 fit in a CU's
// LDS) per 256-row block. The block's cells (one run per column block) are read as one
// flattened sequence of 32-bit words of ul and yv: word f of the sequence is found by a
// binary search over the cells' word prefix in LDS, and lane i of a wavefront takes words
// i, i + 64, ... so loads stay coalesced and kRowsU of them per array are in flight per
// lane. The bytes of a word that lie outside its cell (the cells do not start on word
// boundaries) are masked. One count per entry into LDS bins [row][class] (unit weights:
// without a branch, an entry outside its cell or without a class adding 0); then the rows
// of Z are written once (count * 1/n_k), four floats at a time when Z is 16-byte aligned
// (VEC). The word prefix of the cells comes with the layout (cell_word).
//
// HALF (many classes): the bins take half the LDS, so more workgroups share a CU. A
// unit-weight block of at most 4 * 16383 entries counts into 16-bit halves of 32-bit
// words (no count can reach 2^16, so none carries into its neighbour); a larger block
// is counted in two passes over its words, rows 0-127 and then rows 128-255, each into
// 32-bit bins.
//
// WT (weighted layout): the bins hold sums of the entries' weights (a Laplacian layout's
// entries carry w d_u^-1/2 d_v^-1/2). A block whose flag is 0 (rows of at most
// kPbF32Terms entries, no negative weight) sums in 32-bit integers when the layout's
// weights lie on a grid 2^-g (meta[4] = g; the sums are then exact); other blocks sum in
// FP64. The bins' LDS holds R rows of either (R = 256 or 128 for the integers, half that
// for FP64), and the block's rows are taken R at a time, one pass over its words each.
template <bool VEC, bool HALF, bool WT, int NT>
__global__ void __launch_bounds__(NT)
k_pb_rows(int64_t n, int64_t nnz, int64_t n_lds, const int64_t *__restrict__ meta, int64_t lim, int32_t K,
          uint64_t magicK, int32_t n_cb, int32_t top, int32_t strideq, const int64_t *__restrict__ cell_start,
          const uint32_t *__restrict__ cell_count, const uint32_t *__restrict__ cell_word,
          const uint32_t *__restrict__ ul4, const uint32_t *__restrict__ yv4, const f32x4 *__restrict__ vl4,
          const uint8_t *__restrict__ rb_flag, const float *__restrict__ rsd, const double *__restrict__ inv,
          float *__restrict__ Z, int32_t *err)
{
    // LDS: bins [nb] uint32 (nb = 256 K, or 128 K for HALF, rounded up to 4), invx
    // [K + 3] double (invx[i] = 1/n_(i mod K) + 1), per cell: first entry [n_cb] (its
    // word and its byte offset in that word), word prefix [n_cb + 1], entry count [n_cb].
    extern __shared__ __align__(16) uint32_t bins[];
    if (!layout_matches(meta, n, nnz, n_lds, rsd ? 2 : (WT ? 1 : 0), err)) return;
    const uint32_t nb = (uint32_t)align_up((size_t)(HALF ? kPbRows / 2 : kPbRows) * K, 4);
    double *invx = reinterpret_cast<double *>(bins + nb);
    uint32_t *ca = reinterpret_cast<uint32_t *>(invx + K + 3);
    uint32_t *pre = ca + n_cb;
    uint32_t *cm = pre + n_cb + 1;
    // Workgroups are dealt to the 8 XCDs in turn (i -> XCD i mod 8). Neighbouring row
    // blocks' cells share cache lines (a vertex block's cells are small and adjacent),
    // so each XCD takes one contiguous run of row blocks and the lines are fetched into
    // one L2 only.
    const uint32_t per = gridDim.x / kXcds, rem = gridDim.x % kXcds;
    const uint32_t xcd = blockIdx.x % kXcds, bk = blockIdx.x / kXcds;
    const int64_t rb = (int64_t)(xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + bk;
    const int64_t r0 = rb * kPbRows;
    const int nr = (int)((n - r0) < kPbRows ? (n - r0) : kPbRows);
    const int t = threadIdx.x, lane = t % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(t / kWave);
    // the block's global reads first (its first NT cells and the class factors; K + 3 <=
    // NT), then the bins are zeroed while they are in flight
    int64_t a1 = 0;
    uint32_t m1 = 0u, p1 = 0u;
    double v1 = 0.0;
    if (t < n_cb) {
        a1 = cell_start[rb * n_cb + t];
        m1 = cell_count[rb * n_cb + t];
        p1 = cell_word[rb * n_cb + t];
    }
    if (t < K + 3) v1 = inv[1 + t % K];
    for (uint32_t i = t; i < nb / 4; i += NT) reinterpret_cast<u32x4 *>(bins)[i] = u32x4{0u, 0u, 0u, 0u};
    if (t < K + 3) invx[t] = v1;
    for (int c = t; c < n_cb; c += NT) {
        const bool first = c == t;
        int64_t a = first ? a1 : cell_start[rb * n_cb + c];
        uint32_t m = first ? m1 : cell_count[rb * n_cb + c];
        const uint32_t p = first ? p1 : cell_word[rb * n_cb + c];
        // a cell must lie inside the layout's entries [0, lim): one that does not (a layout
        // that is not what it claims) is read as empty and raises GEE_EVERTEX
        if (a < 0 || a > lim || (int64_t)m > lim - a) {
            flag_error(err, GEE_EVERTEX);
            a = 0;
            m = 0u;
        }
        ca[c] = (uint32_t)a; // below 2^32: the layout holds fewer than 2^32 entries
        cm[c] = m;
        pre[c] = p;
        if (c == n_cb - 1) pre[n_cb] = p + (m != 0u ? ((uint32_t)(a & 3) + m + 3u) >> 2 : 0u);
    }
    __syncthreads();
    const uint32_t T = pre[n_cb];
    const int64_t wlim = (lim + 3) / 4; // the last word holding layout entries

    // every entry (ub, yb) of the block's cells with a known class, to add(ub, yb, weight)
    // (the weight is 1 for a unit-weight layout)
    auto count = [&](auto add) __attribute__((always_inline)) {
        for (uint32_t f0 = (uint32_t)(wave * kWave + lane); f0 < T; f0 += kRowsU * NT) {
            uint32_t u[kRowsU], y[kRowsU], rel[kRowsU], m[kRowsU];
            f32x4 wq[kRowsU];
            // the cells of the kRowsU words, by binary searches run in step: each step reads
            // pre[] once per word (an index past the last cell reads pre[n_cb] = T, which
            // no word reaches), so the reads of one step are in flight together
            int cs[kRowsU];
#pragma unroll
            for (int j = 0; j < kRowsU; ++j) cs[j] = 0;
            for (int st = top; st > 0; st >>= 1) {
                uint32_t p[kRowsU];
#pragma unroll
                for (int j = 0; j < kRowsU; ++j) {
                    const int nc = cs[j] + st;
                    p[j] = pre[nc < n_cb ? nc : n_cb];
                }
#pragma unroll
                for (int j = 0; j < kRowsU; ++j)
                    cs[j] = p[j] <= f0 + (uint32_t)j * NT ? cs[j] + st : cs[j];
            }
#pragma unroll
            for (int j = 0; j < kRowsU; ++j) {
                const uint32_t f = f0 + (uint32_t)j * NT;
                u[j] = 0u;
                y[j] = 0u;
                rel[j] = 0u;
                m[j] = 0u;
                wq[j] = f32x4{1.0f, 1.0f, 1.0f, 1.0f};
                if (f < T) {
                    const int c = cs[j];
                    const uint32_t k = f - pre[c];
                    // the word prefix comes with the layout: a word index it would carry past
                    // the layout's words (an inconsistent prefix) is clamped into them, and
                    // the entries it then reads lie outside the cell's count, so none is added
                    const uint32_t a = ca[c];
                    int64_t w = (int64_t)(a >> 2) + k;
                    w = w < wlim ? w : wlim;
                    u[j] = ul4[w];
                    y[j] = yv4[w];
                    if (WT) wq[j] = vl4[w];
                    rel[j] = 4u * k - (a & 3u); // entry index within the cell of the word's byte 0 (mod 2^32)
                    m[j] = cm[c];
                }
            }
#pragma unroll
            for (int j = 0; j < kRowsU; ++j) {
                if (f0 + (uint32_t)j * NT < T) {
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const uint32_t yb = (y[j] >> (8 * b)) & 0xffu;
                        const uint32_t ub = (u[j] >> (8 * b)) & 0xffu;
                        add(ub, yb, wq[j][b], yb != 0u && rel[j] + (uint32_t)b < m[j]);
                    }
                }
            }
        }
    };
    // rows [lo, hi) of the block to Z from the bins, get4(g) giving the four sums of flat
    // elements g .. g + 3 (g a multiple of 4) and get1(g) one, g counted from row lo, each
    // times 1/n_k of its class k (a Laplacian layout's entries carry both d^-1/2 factors).
    // With 16-byte stores (VEC: Z 16-byte aligned, lo K a multiple of 4) the quads a thread
    // takes are strideq apart, a multiple of K elements, so all of them start at one class
    // and its four factors stay in registers.
    auto write = [&](int lo, int hi, auto get4, auto get1) __attribute__((always_inline)) {
        float *zb = Z + (r0 + lo) * K;
        const uint32_t total = (uint32_t)(hi - lo) * (uint32_t)K;
        uint32_t done = 0;
        if (VEC && strideq > 0) {
            const uint32_t nv = total / 4;
            if (t < strideq) {
                const uint32_t k = (4u * (uint32_t)t) % (uint32_t)K;
                const double i0 = invx[k], i1 = invx[k + 1], i2 = invx[k + 2], i3 = invx[k + 3];
                for (uint32_t v = t; v < nv; v += (uint32_t)strideq) {
                    const auto c = get4(4u * v);
                    const f32x4 o = {(float)((double)c.x * i0), (float)((double)c.y * i1), (float)((double)c.z * i2),
                                     (float)((double)c.w * i3)};
                    __builtin_nontemporal_store(o, reinterpret_cast<f32x4 *>(zb) + v);
                }
            }
            done = nv * 4;
        }
        for (uint32_t f = done + t; f < total; f += NT) {
            const uint32_t k = f - div_small(f, magicK) * (uint32_t)K;
            __builtin_nontemporal_store((float)((double)get1(f) * invx[k]), zb + f);
        }
    };
    auto zero = [&]() __attribute__((always_inline)) {
        __syncthreads(); // the previous rows are written
        for (uint32_t i = t; i < nb / 4; i += NT) reinterpret_cast<u32x4 *>(bins)[i] = u32x4{0u, 0u, 0u, 0u};
        __syncthreads();
    };
    if constexpr (WT) {
        double *db = reinterpret_cast<double *>(bins);
        // exact 32-bit integer sums for a block of grid weights whose flag is 0; FP64 sums
        // otherwise (FP64 LDS adds measured faster than FP32 ones on MI355X, even with the
        // block's rows taken in two passes)
        const int64_t grid = meta[4];
        const bool wide = rb_flag[rb] != 0 || grid == kPbNoGrid;
        int R = (int)(nb / (uint32_t)(wide ? 2 * K : K));
        R = R < kPbRows ? R : kPbRows;
        for (int lo = 0; lo < nr; lo += R) {
            if (lo > 0) zero();
            const int hi = nr < lo + R ? nr : lo + R;
            if (wide) {
                count([&](uint32_t ub, uint32_t yb, float w, bool ok) {
                    if (ok && ub - (uint32_t)lo < (uint32_t)R)
                        atomicAdd(&db[(ub - (uint32_t)lo) * (uint32_t)K + (yb - 1u)], (double)w);
                });
                __syncthreads();
                auto g4 = [&](uint32_t f) {
                    const double2 a = reinterpret_cast<const double2 *>(db)[f / 2];
                    const double2 b = reinterpret_cast<const double2 *>(db)[f / 2 + 1];
                    return f64x4{a.x, a.y, b.x, b.y};
                };
                auto g1 = [&](uint32_t f) { return db[f]; };
                write(lo, hi, g4, g1);
            } else {
                // every weight is an integer multiple of 2^-grid: 32-bit integer sums of the
                // scaled weights are exact (the build checked that they stay below 2^32), and
                // the row is written from the exact value, as from FP64 sums
                const float up = ldexpf(1.0f, (int)grid);
                const double down = ldexp(1.0, -(int)grid);
                count([&](uint32_t ub, uint32_t yb, float w, bool ok) {
                    if (ok && ub - (uint32_t)lo < (uint32_t)R)
                        atomicAdd(&bins[(ub - (uint32_t)lo) * (uint32_t)K + (yb - 1u)], (uint32_t)(w * up));
                });
                __syncthreads();
                auto g4 = [&](uint32_t f) {
                    const u32x4 c = reinterpret_cast<const u32x4 *>(bins)[f / 4];
                    return f64x4{(double)c.x * down, (double)c.y * down, (double)c.z * down, (double)c.w * down};
                };
                auto g1 = [&](uint32_t f) { return (double)bins[f] * down; };
                write(lo, hi, g4, g1);
            }
        }
        return;
    }
    auto get4_32 = [&](uint32_t f) { return reinterpret_cast<const u32x4 *>(bins)[f / 4]; };
    auto get1_32 = [&](uint32_t f) { return bins[f]; };
    if (!HALF) {
        // branch-free: an entry outside its cell or without a class adds 0 at a valid bin
        count([&](uint32_t ub, uint32_t yb, float, bool ok) {
            atomicAdd(&bins[__umul24(ub, (uint32_t)K) + (yb != 0u ? yb - 1u : 0u)], ok ? 1u : 0u);
        });
        __syncthreads();
        write(0, nr, get4_32, get1_32);
        return;
    }
    if (T <= 16383u) {
        // at most 65532 entries: 16-bit counts, element f in half (f & 1) of word f / 2
        count([&](uint32_t ub, uint32_t yb, float, bool ok) {
            if (!ok) return;
            const uint32_t f = ub * (uint32_t)K + (yb - 1u);
            atomicAdd(&bins[f >> 1], 1u << (16u * (f & 1u)));
        });
        __syncthreads();
        write(
            0, nr,
            [&](uint32_t f) {
                const uint2 w = reinterpret_cast<const uint2 *>(bins)[f / 4];
                return u32x4{w.x & 0xffffu, w.x >> 16, w.y & 0xffffu, w.y >> 16};
            },
            [&](uint32_t f) { return (bins[f >> 1] >> (16u * (f & 1u))) & 0xffffu; });
        return;
    }
    for (int h = 0; h < 2 && h * (kPbRows / 2) < nr; ++h) {
        if (h == 1) zero();
        count([&](uint32_t ub, uint32_t yb, float, bool ok) {
            if (ok && (ub >> 7) == (uint32_t)h) atomicAdd(&bins[(ub & 127u) * (uint32_t)K + (yb - 1u)], 1u);
        });
        __syncthreads();
        const int lo = h * (kPbRows / 2), hi = nr < lo + kPbRows / 2 ? nr : lo + kPbRows / 2;
        write(lo, hi, get4_32, get1_32);
    }
}

} // namespace

PbLayout pb_layout(int64_t n, int64_t n_lds)
{
    PbLayout L;
    L.n_rb = (n + kPbRows - 1) / kPbRows;
    L.n_vcb = (int32_t)((n + ((int64_t)1 << kPbColBits) - 1) >> kPbColBits);
    L.n_sl = (int32_t)((n_lds + kPbSlice - 1) >> kPbSliceBits);
    L.n_cb = L.n_vcb + L.n_sl;
    L.cells = L.n_rb * L.n_cb;
    return L;
}

// Build scratch: two key buffers [nnz], radix histograms, scan partials, two cell arrays.
size_t pb_build_scratch(int64_t n, int64_t nnz, int64_t n_lds, bool weighted, bool laplacian)
{
    const PbLayout L = pb_layout(n, n_lds);
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
    take(16);
    take(16);
    if (weighted || laplacian) {
        take((size_t)nnz * 4);
        take((size_t)nnz * 4);
    }
    if (laplacian) take((size_t)n * 8);
    return align_up(off, 256);
}

hipError_t launch_pb_build(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col, const float *val,
                           bool laplacian, const int32_t *hot_ids, int64_t n_hot, int64_t n_lds, int32_t *colc,
                           uint8_t *ul, int64_t *cell_start, uint32_t *cell_count, uint32_t *cell_word,
                           int32_t *lds_ids, float *vl, uint8_t *rb_flag, float *rsd, int64_t *meta, void *ws,
                           int32_t *err, hipStream_t s)
{
    const PbLayout L = pb_layout(n, n_lds);
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
    int64_t *tier_buf = (int64_t *)take(16);
    int64_t *tier = L.n_sl > 0 ? tier_buf : nullptr; // {h0, H0}
    int32_t *ex = (int32_t *)take(16);                // lowest and highest weight bit (weighted)
    const bool carried = val != nullptr || laplacian; // a value per entry goes with the sort
    float *v0 = carried ? (float *)take((size_t)nnz * 4) : nullptr;
    float *v1 = carried ? (float *)take((size_t)nnz * 4) : nullptr;
    double *deg = laplacian ? (double *)take((size_t)n * 8) : nullptr;
    float *sval = nullptr; // values in sorted order
    hipError_t e;
    const dim3 b(kT);
    const int64_t kind = laplacian ? 2 : (val ? 1 : 0);
    hipLaunchKernelGGL(k_pb_meta, dim3(1), dim3(kWave), 0, s, meta, n, nnz, n_lds, kind);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (carried) {
        hipLaunchKernelGGL(k_pb_rbflag, dim3(grid_cap(L.n_rb, 1)), b, 0, s, n, L.n_rb, row_ptr, val, rb_flag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (laplacian) {
            // the graph's degrees and d^-1/2 (the terms follow once every entry has its row)
            if ((e = launch_degrees_csr(n, row_ptr, val, nnz, deg, true, err, s)) != hipSuccess) return e;
            if ((e = launch_rsd(deg, n, rsd, s)) != hipSuccess) return e;
        } else if (nnz > 0 && (e = hipMemcpyAsync(v0, val, (size_t)nnz * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) {
            return e;
        }
    }
    if (n_lds > 0 && (e = hipMemcpyAsync(lds_ids, hot_ids, (size_t)n_lds * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return e;
    if (nnz > 0) {
        // row of every entry, then (column << 32) | row
        if ((e = launch_fill_i64(reinterpret_cast<int64_t *>(k1), nnz, 0, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_pb_mark, dim3(grid_cap(n, kT * 4)), b, 0, s, n, row_ptr, reinterpret_cast<int64_t *>(k1));
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = max_scan_i64(reinterpret_cast<const int64_t *>(k1), nnz, reinterpret_cast<int64_t *>(k0), part, s)) !=
            hipSuccess)
            return e;
        hipLaunchKernelGGL(k_pb_key, dim3(grid_cap(nnz, kT * 4)), b, 0, s, nnz, n, col, hot_ids, n_hot, n_lds, L.n_vcb,
                           k0, err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (laplacian) {
            // every entry's term w d_u^-1/2 d_v^-1/2 (its row u in the key's low half)
            hipLaunchKernelGGL(k_pb_lapw, dim3(grid_cap(nnz, kT * 4)), b, 0, s, nnz, n, col, val, hot_ids, n_hot, k0,
                               rsd, v0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (carried) {
            // the weights' grid (meta[4]), from the values the layout will hold
            hipLaunchKernelGGL(k_pb_grid_init, dim3(1), dim3(kWave), 0, s, ex);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_pb_grid_bits, dim3(grid_cap(nnz, kT * 16)), b, 0, s, nnz, v0, ex);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_pb_grid_final, dim3(1), dim3(kWave), 0, s, ex, meta);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            sval = v0;
        }
        // stable sort on the column-block bits (the entries are in row order already)
        uint64_t *sorted = k0;
        if (L.n_cb > 1) {
            int hi = 32 + kPbColBits;
            while (hi < 64 && ((int64_t)1 << (hi - 32 - kPbColBits)) < L.n_cb) ++hi;
            if (carried) {
                if ((e = radix_sort_bits_kv(k0, k1, v0, v1, nnz, 32 + kPbColBits, hi, hist, offs, part, &sorted, &sval,
                                            s)) != hipSuccess)
                    return e;
            } else if ((e = radix_sort_bits(k0, k1, nnz, 32 + kPbColBits, hi, hist, offs, part, &sorted, s)) !=
                       hipSuccess) {
                return e;
            }
        }
        if ((e = launch_fill_i64(celllast, L.cells, 0, s)) != hipSuccess) return e;
        if (tier) {
            hipLaunchKernelGGL(k_pb_tier_start, dim3(1), dim3(kWave), 0, s, sorted, nnz, L.n_vcb, tier);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_pb_finalize, dim3(grid_cap(nnz, kT * 4)), b, 0, s, sorted, sval, nnz, L.n_rb, L.n_vcb,
                           tier, colc, reinterpret_cast<uint8_t *>(colc), ul, vl, celllast);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (tier) {
            hipLaunchKernelGGL(k_pb_tier_hi, dim3(grid_cap(nnz + 64, kT)), b, 0, s, sorted, nnz, tier,
                               reinterpret_cast<uint8_t *>(colc));
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    } else {
        if ((e = launch_fill_i64(celllast, L.cells, 0, s)) != hipSuccess) return e;
        if (tier && (e = launch_fill_i64(tier, 2, 0, s)) != hipSuccess) return e;
        if (carried) { // no weights: any grid holds them
            hipLaunchKernelGGL(k_pb_grid_init, dim3(1), dim3(kWave), 0, s, ex);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(k_pb_grid_final, dim3(1), dim3(kWave), 0, s, ex, meta);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if ((e = max_scan_i64(celllast, L.cells, cellend, part, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pb_table, dim3(grid_cap(L.cells, kT * 4)), b, 0, s, L.n_rb, L.n_cb, L.n_vcb, tier, cellend,
                       cell_start, cell_count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pb_words, dim3(grid_cap(L.n_rb, kT)), b, 0, s, L.n_rb, L.n_cb, cell_start, cell_count,
                       cell_word);
    return hipGetLastError();
}

hipError_t launch_pb_gather(int64_t n, int64_t nnz, const PbLayout &L, int64_t n_lds, const int64_t *cell_start,
                            const uint32_t *cell_count, const int32_t *colc, const int32_t *lds_ids,
                            const int64_t *meta, int kind, const uint8_t *lab, uint8_t *tab, uint8_t *yv,
                            int32_t *err, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    const int64_t *sl_start = L.n_sl > 0 ? cell_start + L.n_vcb : nullptr; // cells (0, n_vcb + j)
    // vertex blocks: one workgroup per 8,192 entries, dispatched in order, so the entries
    // in flight stay within one or two column blocks (their labels in L2)
    hipLaunchKernelGGL(k_pb_gather, dim3(grid_cap(nnz, kT * 32)), dim3(kT), 0, s, nnz, n, n_lds, kind, meta,
                       sl_start, colc, lab, yv, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || L.n_sl == 0) return e;
    hipLaunchKernelGGL(k_pb_tier_labels, dim3(grid_cap(n_lds, kT * 4)), dim3(kT), 0, s, n_lds, n, nnz, kind, meta,
                       lds_ids, lab, tab, err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    // one workgroup per CU (the table takes 128 KB of LDS), at least 64K entries each
    int64_t grid = nnz / 65536;
    if (grid > cus) grid = cus;
    if (grid < 1) grid = 1;
    const int64_t last = L.cells - 1; // the last cell of the column-block-major order
    hipLaunchKernelGGL(k_pb_gather_tier, dim3((unsigned)grid), dim3(kLdsT), (size_t)kPbSlice, s, nnz, n, kind,
                       meta, L.n_sl, n_lds, sl_start, cell_start + last, cell_count + last,
                       reinterpret_cast<const uint8_t *>(colc), tab, yv, err);
    return hipGetLastError();
}

hipError_t launch_pb_slice_entries(int64_t n_slots, const int32_t *hot_ids, const int64_t *row_ptr,
                                  int64_t *slice_entries, hipStream_t s)
{
    const int64_t n_sl = (n_slots + kPbSlice - 1) >> kPbSliceBits;
    if (n_sl <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pb_slice_entries, dim3((unsigned)n_sl), dim3(kT), 0, s, n_slots, hot_ids, row_ptr,
                       slice_entries);
    return hipGetLastError();
}

size_t pb_rows_lds_bytes(int32_t K, int32_t n_cb, bool half)
{
    return align_up((size_t)(half ? kPbRows / 2 : kPbRows) * K, 4) * 4 + (size_t)(K + 3) * 8 +
           (size_t)(3 * n_cb + 1) * 4;
}

// LDS that three 512-thread workgroups of the rows pass can share on one CU: measured,
// three of 53,548 bytes run together and three of 53,948 bytes do not (less than the
// 160 KB the device reports), so a bound between the two.
constexpr size_t kRowsCuLds = 161280;

// 16-bit (HALF) bins when 32-bit bins would leave fewer than three workgroups per CU,
// as they do from about 51 classes up.
bool pb_rows_half(int32_t K, int32_t n_cb) { return 3 * pb_rows_lds_bytes(K, n_cb, false) > kRowsCuLds; }

hipError_t launch_pb_rows(int64_t n, int64_t nnz, int32_t K, const PbLayout &L, const int64_t *cell_start,
                          const uint32_t *cell_count, const uint32_t *cell_word, const uint8_t *ul, const uint8_t *yv,
                          const float *vl, const uint8_t *rb_flag, const float *rsd, const int64_t *meta,
                          int64_t n_lds, const double *inv, float *Z, int32_t *err, hipStream_t s)
{
    const int64_t lim = nnz + 15; // layout entries, the gap before the tier included
    const bool half = pb_rows_half(K, L.n_cb);
    const size_t lds = pb_rows_lds_bytes(K, L.n_cb, half);
    const uint64_t magic = ((1ull << 32) + (uint64_t)K - 1) / (uint64_t)K;
    int top = 1;
    while (top * 2 <= L.n_cb - 1) top *= 2;
    // 1024-thread workgroups when fewer than three of 512 fit in a CU's LDS (two then
    // still do, with twice the wavefronts per row block)
    const bool wide_wg = 3 * lds > kRowsCuLds;
    const int nt = wide_wg ? 2 * kRowsT : kRowsT;
    // quad stride of the fixed-class write: the largest multiple of K / gcd(K, 4) up to nt
    const int kq = K / (K % 4 == 0 ? 4 : (K % 2 == 0 ? 2 : 1));
    const int strideq = kq <= nt ? (nt / kq) * kq : 0;
    const uint32_t *ul4 = reinterpret_cast<const uint32_t *>(ul);
    const uint32_t *yv4 = reinterpret_cast<const uint32_t *>(yv);
    const f32x4 *vl4 = reinterpret_cast<const f32x4 *>(vl);
    const bool vec = (reinterpret_cast<uintptr_t>(Z) & 15) == 0;
#define GEE_ROWS_NT(V, H, W, N)                                                                                      \
    hipLaunchKernelGGL((k_pb_rows<V, H, W, N>), dim3((unsigned)L.n_rb), dim3(N), lds, s, n, nnz, n_lds, meta, lim,   \
                       K, magic, L.n_cb, top, strideq, cell_start, cell_count, cell_word, ul4, yv4, vl4, rb_flag, rsd,  \
                       inv, Z, err)
#define GEE_ROWS(V, H, W)                                                                                            \
    do {                                                                                                             \
        if (wide_wg) GEE_ROWS_NT(V, H, W, 2 * kRowsT);                                                               \
        else GEE_ROWS_NT(V, H, W, kRowsT);                                                                           \
    } while (0)
    if (vl) {
        if (half) {
            if (vec) GEE_ROWS(true, true, true);
            else GEE_ROWS(false, true, true);
        } else {
            if (vec) GEE_ROWS(true, false, true);
            else GEE_ROWS(false, false, true);
        }
    } else if (half) {
        if (vec) GEE_ROWS(true, true, false);
        else GEE_ROWS(false, true, false);
    } else {
        if (vec) GEE_ROWS(true, false, false);
        else GEE_ROWS(false, false, false);
    }
#undef GEE_ROWS
#undef GEE_ROWS_NT
    return hipGetLastError();
}

} // namespace gee
