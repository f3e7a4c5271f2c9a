// Batched GEE on gfx950: many label vectors embedded over one graph in one pass
// of the CSR.
//
// Algorithm 1 (Section II of the paper) is a single pass over the edges for one
// label vector. For B vectors on the same graph the pass is shared. The vectors of
// a group (up to 64, any mix of adjacency and Laplacian) are stored transposed: one
// row of labels per vertex (8-bit when every vector of the group has K <= 255, else
// 16-bit), so one 64- or 128-byte piece holds a vertex's labels in all 64 vectors. Hot vertices (the CSR's hot slots) get a compact copy of their
// rows, addressed by slot, so an entry whose column is a slot needs no id lookup.
//
// One wavefront owns a segment of the merge-path split (rows + entries). Lane b is
// vector b: for every entry (u, v) of a row the wave reads v's label row with one
// coalesced load and lane b adds the entry's weight into its own bin
// (u, coff_b + Y_b(v) - 1) in LDS. The bins of different lanes are disjoint, so the
// adds need no atomicity, and every bin receives its terms in CSR order: the FP64
// sums are deterministic. A finished row is scaled and written to Z once. Rows cut
// by segment boundaries are summed from FP64 partials in segment order.

#include <algorithm>
#include <type_traits>

#include "common.h"
#include "launch.h"

namespace gee {

namespace {

constexpr int kBT = 256;      // threads per block of the helper kernels
constexpr int kCW = 48;       // entries per chunk (a chunk never spans two rows; measured faster than 32 and 64)
constexpr int kMaxWavesPerBlock = 8;
constexpr uint32_t kNoVec = 0xffffffffu;
typedef __attribute__((address_space(1))) const uint16_t global_u16;
typedef __attribute__((address_space(1))) const uint8_t global_u8;

inline int grid_cap(int64_t items, int per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

// labmat[v * Gs + b] = label of vertex v in vector b of the group (0 for a label
// outside [0, K_b] and for the padding columns b >= G); row n is all zeros and is
// where invalid column ids point. Labels are 8-bit (L = uint8_t) when every vector
// of the group has K <= 255, else 16-bit. A tile of 256 vertices x Gs vectors goes
// through LDS so both the read (along v) and the write (along b, four labels per
// thread) are coalesced.
template <typename L>
__global__ void __launch_bounds__(kBT)
k_pack_group(const int32_t *__restrict__ labels, int64_t n, GroupDesc d, L *__restrict__ labmat, int32_t *err)
{
    // 256 vertices x 64 vectors; 136-byte rows, so four labels are one aligned 8-byte read
    __shared__ __align__(16) uint16_t tile[kBT][68];
    const int64_t v0 = (int64_t)blockIdx.x * kBT;
    const int t = threadIdx.x;
    const int64_t v = v0 + t;
    bool bad = false;
    // 1 KB of each vector per block, coalesced along v; 16 vectors' loads in flight at once
    for (int b0 = 0; b0 < d.Gs; b0 += 16) {
        int32_t x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int b = b0 + i;
            x[i] = v < n && b < d.G ? labels[(int64_t)d.vec[b] * n + v] : 0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int b = b0 + i;
            if (b < d.Gs) {
                const bool ok = b >= d.G || (uint32_t)x[i] <= (uint32_t)d.K[b];
                bad |= !ok;
                tile[t][b] = ok ? (uint16_t)x[i] : 0;
            }
        }
    }
    __syncthreads();
    // Gs is a multiple of 8, so a row holds Gs / 4 quads, each 4- (8-bit) or 8-byte
    // (16-bit) aligned
    const int qpr = d.Gs / 4;
    for (int i = t; i < kBT * qpr; i += kBT) {
        const int r = i / qpr, q = i - r * qpr;
        const int64_t u = v0 + r;
        if (u < n) {
            const uint2 w = *reinterpret_cast<const uint2 *>(&tile[r][4 * q]);
            if (sizeof(L) == 1)
                reinterpret_cast<uint32_t *>(labmat + u * d.Gs)[q] =
                    (w.x & 0xffu) | ((w.x >> 8) & 0xff00u) | ((w.y & 0xffu) << 16) | ((w.y >> 16) << 24);
            else
                reinterpret_cast<uint2 *>(labmat + u * d.Gs)[q] = w;
        }
    }
    if (blockIdx.x == 0 && t < d.Gs) labmat[n * d.Gs + t] = (L)0;
    if (bad) flag_error(err, GEE_ELABEL);
}

// Hot rows in slot order: labhot[s] = labmat[hot_ids[s]] (rows of rb bytes, copied in
// pieces of sizeof(P) bytes), and for a group with Laplacian vectors rsdhot[s] =
// d^-1/2 of that vertex.
template <typename P>
__global__ void __launch_bounds__(kBT)
k_pack_group_hot(const int32_t *__restrict__ hot_ids, int64_t n_hot, int64_t n, int rb,
                 const uint8_t *__restrict__ labmat, uint8_t *__restrict__ labhot, const float *__restrict__ rsd,
                 float *__restrict__ rsdhot, int32_t *err)
{
    const int pieces = rb / (int)sizeof(P);
    const int64_t total = n_hot * pieces;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = i / pieces;
        const int p = (int)(i - s * pieces);
        int64_t v = hot_ids[s];
        if ((uint64_t)v >= (uint64_t)n) {
            bad = true;
            v = n; // the zero row
        }
        const P q = *reinterpret_cast<const P *>(labmat + v * rb + p * (int)sizeof(P));
        *reinterpret_cast<P *>(labhot + s * rb + p * (int)sizeof(P)) = q;
        if (rsdhot && p == 0) rsdhot[s] = v < n ? rsd[v] : 0.0f;
    }
    if (bad) flag_error(err, GEE_EVERTEX);
}

// Per column f of the group: cscale[f] = 1 / n_{b,k+1} (IEEE division of the class
// count, 0 for an empty class), negated (sign bit set, also for a zero) when vector b is
// a Laplacian one. Per lane: vmeta[b] = coff_b | (Laplacian << 31), kNoVec for the
// lanes b >= G. counts_all holds each vector's K_b + 1 counts at its inv_off.
__global__ void k_group_cols(const uint64_t *__restrict__ counts_all, GroupDesc d, double *__restrict__ cscale,
                             uint32_t *__restrict__ vmeta)
{
    const int b = blockIdx.x;
    if (b == d.G) {
        for (int t = d.G + threadIdx.x; t < kGroupMax; t += blockDim.x) vmeta[t] = kNoVec;
        return;
    }
    const bool lap = d.lap[b] != 0;
    for (int k = threadIdx.x; k < d.K[b]; k += blockDim.x) {
        const uint64_t c = counts_all[d.inv_off[b] + k + 1];
        const double inv = c == 0 ? 0.0 : 1.0 / (double)c;
        cscale[d.coff[b] + k] = lap ? -inv : inv;
    }
    if (threadIdx.x == 0) vmeta[b] = (uint32_t)d.coff[b] | (lap ? 0x80000000u : 0u);
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

__device__ inline int64_t readlane64(int64_t x, int l)
{
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)x >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline float readlanef(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Factor of a bin in Z: 1 / n_k, times the row's d^-1/2 for a Laplacian column
// (sign bit of the stored scale). Same expression, x * (inv * r_u), as the
// single-vector pass, with r_u = 1 for adjacency columns.
__device__ inline double column_scale(double s, double ru)
{
    return __double_as_longlong(s) < 0 ? (-s) * ru : s * 1.0;
}

// The chunk iterator and the row window are scalar (wave-uniform) state.
struct Chunk {
    int64_t u = 0, e = 0; // row, first entry
    int m = 0;            // entries (1..kCW)
    bool last = false;    // the chunk ends the row's entries in this segment
};

// One wavefront per segment. Lane b accumulates vector b's bins of the current row
// (bins[coff_b .. coff_b + K_b), FP64, private to the lane). Entries are taken in
// chunks of up to kCW entries of one row; the labels of chunk k+1 and the column
// ids of chunk k+2 are in flight while chunk k is added and its row written. The
// row writes read nothing from global memory (column scales sit in LDS, shared by
// the block's wavefronts; row ends and d^-1/2 in a 64-row register window), so they
// never wait on those loads. L is the label type of the group's rows (8- or 16-bit).
template <bool W, bool LAP, typename L>
__global__ void __launch_bounds__(kWave * kMaxWavesPerBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_pull(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
             const float *__restrict__ val, int64_t n_hot, const L *__restrict__ labmat,
             const L *__restrict__ labhot, int Gs, const float *__restrict__ rsd,
             const float *__restrict__ rsdhot, const uint32_t *__restrict__ vmeta, const double *__restrict__ cscale,
             int KT, const int32_t *__restrict__ seg_i, const int64_t *__restrict__ seg_e, int64_t nseg,
             float *__restrict__ Z, int64_t ldz, int64_t zcol, double *__restrict__ part, int32_t *err,
             const uint8_t *__restrict__ lbase, uint32_t mat_off, uint32_t hot_off)
{
    extern __shared__ __align__(16) double smem_d[];
    const int KTp = (KT + 1) & ~1; // even, so 16-byte LDS accesses of column pairs stay aligned
    double *tab = smem_d; // [KT] column scales
    const int nw = blockDim.x / kWave;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); // uniform per wavefront
    const int lane = threadIdx.x % kWave;
    // per wavefront: KTp bins, then one sink bin per lane (target of unknown labels)
    double *bins = smem_d + (size_t)KTp + (size_t)(KTp + kWave) * wid;
    for (int f = threadIdx.x; f < KT; f += blockDim.x) tab[f] = cscale[f];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * nw + wid;
    if (j >= nseg) return;
    const BatchSeg sg = batch_seg(j, n, row_ptr, seg_i, seg_e);
    const uint32_t vm = vmeta[lane];
    const bool vvalid = vm != kNoVec;
    const int boff = (int)(vm & 0x7fffffffu) - 1; // bin of class y is boff + y
    const bool vlap = LAP && vvalid && (vm >> 31) != 0;
    // a lane without a vector reads a zero padding column (label rows are wider than the
    // group when it has fewer than 64 vectors), so its terms go to its sink
    const int lsrc = lane < Gs ? lane : Gs - 1;
    for (int f = lane; f < KTp + kWave; f += kWave) bins[f] = 0.0;
    const int sink = KTp + lane;
    bool bad = false;
    // label rows through one buffer resource when both arrays lie within 4 GiB of lbase
    // (one readlane per entry for its 32-bit offset), else by 64-bit addresses. The
    // resource is raw (stride 0, no record limit; word 3 0x20000: 32-bit data, no
    // swizzle), so its bounds are the caller's check of the span.
    const bool lbuf = lbase != nullptr;
    const __amdgpu_buffer_rsrc_t lres = __builtin_amdgcn_make_buffer_rsrc((void *)lbase, (short)0, -1, 0x00020000);
    const uint32_t rowb = (uint32_t)Gs * (uint32_t)sizeof(L), lbyte = (uint32_t)lsrc * (uint32_t)sizeof(L);

    // row window: lane i holds the end of row wb + i
    int64_t cu = sg.i0, ce = sg.e0, wb = sg.i0;
    int64_t win;
    auto load_window = [&]() __attribute__((always_inline)) {
        const int64_t r = wb + lane + 1;
        win = row_ptr[r < n ? r : n];
    };
    load_window();
    auto next_chunk = [&](Chunk &c) __attribute__((always_inline)) -> bool {
        while (cu < sg.rend) {
            if (cu - wb >= kWave) {
                wb = cu;
                load_window();
            }
            int64_t re = readlane64(win, (int)(cu - wb));
            re = re < sg.e1 ? re : sg.e1;
            if (ce < re) {
                const int64_t left = re - ce;
                c.u = cu;
                c.e = ce;
                c.m = (int)(left < kCW ? left : kCW);
                c.last = c.m == left;
                ce += c.m;
                return true;
            }
            ++cu;
        }
        return false;
    };
    // column id (and weight) of entry c.e + lane, lanes past the chunk repeating its
    // last entry; before them (Laplacian) the d^-1/2 of the chunk's row
    // (the row factor is a vector load: a scalar load would make every later LDS read
    // wait for it, since scalar loads complete out of order on the same counter)
    int32_t vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    auto load_cols = [&](const Chunk &c, int32_t &cv, float &wv, float &rq) __attribute__((always_inline)) {
        if (LAP) rq = rsd[c.u + vzero];
        const int64_t e = c.e + (lane < c.m ? lane : c.m - 1);
        cv = col[e];
        if (W) wv = val[e];
    };
    // label row of every entry of the chunk (lane b: vector b); per entry (lane j) its
    // weight and the neighbour's d^-1/2
    auto issue_labels = [&](int32_t cv, int m, float wv, float rq, uint16_t (&lab)[kCW], float &ia, float &rv,
                            float &ru) __attribute__((always_inline)) {
        if (W) ia = wv;
        if (LAP) ru = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(rq)));
        // lanes past the chunk (and invalid ids, flagged) read the zero row n: their terms
        // go to the sinks, so the adds of a group of 8 need no per-entry test
        const bool real = lane < m;
        const bool hot = cv < 0;
        const int64_t slot = (int64_t)((uint32_t)cv & 0x7fffffffu);
        const bool ok = hot ? slot < n_hot : cv < n;
        bad |= real && !ok;
        const bool use = real && ok;
        const int32_t c = use && !hot ? cv : (int32_t)n; // the zero row
        if (LAP) {
            const float *rp = use && hot ? rsdhot + slot : rsd + (use ? c : 0); // one load on every path
            const float r = *rp;
            rv = use ? r : 0.0f;
        }
        // row offset (or address) per entry (lane j), then per entry one coalesced load; in
        // groups of 8 under a wave-uniform guard (all of them are complete by the time the
        // next step's wait for its column ids returns)
        const L *rowp = use && hot ? labhot + slot * Gs : labmat + (int64_t)c * Gs;
        const uint32_t off = use && hot ? hot_off + (uint32_t)slot * rowb : mat_off + (uint32_t)c * rowb;
        const uint32_t ralo = (uint32_t)(uintptr_t)rowp, rahi = (uint32_t)((uintptr_t)rowp >> 32);
#pragma unroll
        for (int q0 = 0; q0 < kCW; q0 += 8) {
            if (q0 < m && lbuf) {
#pragma unroll
                for (int q = q0; q < q0 + 8; ++q) {
                    const uint32_t so = __builtin_amdgcn_readlane(off, q);
                    if (sizeof(L) == 1) lab[q] = __builtin_amdgcn_raw_buffer_load_b8(lres, lbyte, so, 0);
                    else lab[q] = __builtin_amdgcn_raw_buffer_load_b16(lres, lbyte, so, 0);
                }
            } else if (q0 < m) {
#pragma unroll
                for (int q = q0; q < q0 + 8; ++q) {
                    const uint64_t sa = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(rahi, q) << 32) |
                                        (uint64_t)(uint32_t)__builtin_amdgcn_readlane(ralo, q);
                    using GL = typename std::conditional<sizeof(L) == 1, global_u8, global_u16>::type;
                    lab[q] = reinterpret_cast<const GL *>(sa)[lsrc]; // global, not flat
                }
            } else {
#pragma unroll
                for (int q = q0; q < q0 + 8; ++q) lab[q] = 0;
            }
        }
    };
    // adds in groups of 8 under one wave-uniform test each: within a group no branch, so
    // the scheduler interleaves the entries (entries past the chunk carry label 0)
    auto consume = [&](const Chunk &c, const uint16_t (&lab)[kCW], float ia, float rv) __attribute__((always_inline)) {
#pragma unroll
        for (int q0 = 0; q0 < kCW; q0 += 8) {
            if (q0 < c.m) {
#pragma unroll
                for (int q = q0; q < q0 + 8; ++q) {
                    double inc = 1.0;
                    if (W) inc = (double)readlanef(ia, q);
                    if (LAP) {
                        const double il = inc * (double)readlanef(rv, q);
                        inc = vlap ? il : inc;
                    }
                    const uint32_t y = lab[q];
                    const int at = y != 0 ? boff + (int)y : sink; // no branch, no exec change
                    atomicAdd(&bins[at], inc);
                }
            }
        }
    };
    // row u's bins scaled by 1 / n_k (and, Laplacian columns, the row's d^-1/2 ru);
    // rows without entries hold zeros and take ru = 1
    auto flush = [&](int64_t u, double ru) __attribute__((always_inline)) {
        const bool head = sg.carried && u == sg.i0;
        const bool tail = sg.tail && u == sg.i1;
        if (head || tail) { // a split row: its FP64 partial, merged later in segment order
            double *pr = part + (2 * j + (tail ? 1 : 0)) * KT;
            for (int f = lane; f < KT; f += kWave) {
                pr[f] = bins[f];
                bins[f] = 0.0;
            }
            return;
        }
        float *zr = Z + u * ldz + zcol;
        // lane l takes column pairs (2l, 2l + 1) + 128 i: one 16-byte LDS read of bins,
        // one of scales and one 16-byte zeroing write per pair
        int f0 = 2 * lane;
        for (; f0 + 1 + kWave * 2 < KT; f0 += 2 * kWave * 2) {
            double2 x[2], t[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                x[i] = *reinterpret_cast<const double2 *>(bins + f0 + i * 2 * kWave);
                t[i] = *reinterpret_cast<const double2 *>(tab + f0 + i * 2 * kWave);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int f = f0 + i * 2 * kWave;
                *reinterpret_cast<double2 *>(bins + f) = make_double2(0.0, 0.0);
                __builtin_nontemporal_store((float)(x[i].x * column_scale(t[i].x, ru)), zr + f);
                __builtin_nontemporal_store((float)(x[i].y * column_scale(t[i].y, ru)), zr + f + 1);
            }
        }
        for (; f0 < KT; f0 += 2 * kWave) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int f = f0 + i;
                if (f < KT) {
                    const double x = bins[f];
                    bins[f] = 0.0;
                    __builtin_nontemporal_store((float)(x * column_scale(tab[f], ru)), zr + f);
                }
            }
        }
    };
    // a row with no entries in this segment: zeros, without touching its bins
    auto flush_empty = [&](int64_t u) __attribute__((always_inline)) {
        const bool head = sg.carried && u == sg.i0;
        const bool tail = sg.tail && u == sg.i1;
        if (head || tail) {
            flush(u, 1.0);
            return;
        }
        float *zr = Z + u * ldz + zcol;
        int f = lane;
        for (; f + 3 * kWave < KT; f += 4 * kWave) {
#pragma unroll
            for (int i = 0; i < 4; ++i) __builtin_nontemporal_store(0.0f, zr + f + i * kWave);
        }
        for (; f < KT; f += kWave) __builtin_nontemporal_store(0.0f, zr + f);
    };

    int64_t fr = sg.i0; // next row to write
    Chunk ck;
    bool have = next_chunk(ck);
    // Loads are issued unconditionally (a missing next chunk repeats the current
    // one) so the number of loads in flight is the same on every path, and loaded
    // registers are never copied (a copy would wait for the load): the two register
    // slots alternate between chunk k (being added) and chunk k + 1 (in flight).
    Chunk cn = ck;
    bool haven = have && next_chunk(cn);
    int32_t cv[2];
    float wv[2] = {0.f, 0.f}, rq[2] = {0.f, 0.f}, ia[2] = {0.f, 0.f}, rv[2] = {0.f, 0.f}, ru[2] = {1.f, 1.f};
    uint16_t lab[2][kCW];
    if (have) {
        load_cols(ck, cv[0], wv[0], rq[0]);
        issue_labels(cv[0], ck.m, wv[0], rq[0], lab[0], ia[0], rv[0], ru[0]);
        load_cols(cn, cv[1], wv[1], rq[1]);
    }
    // Chunk k sits in slot S (labels in lab[S]), chunk k + 1's column ids in cv[T]:
    // issue chunk k + 1's labels, then chunk k + 2's column ids into the free slot,
    // then add chunk k and write finished rows while both are in flight.
    auto step = [&](auto slot) __attribute__((always_inline)) {
        constexpr int S = decltype(slot)::value, T = 1 - S;
        issue_labels(cv[T], cn.m, wv[T], rq[T], lab[T], ia[T], rv[T], ru[T]);
        Chunk cnn = cn;
        const bool havenn = haven && next_chunk(cnn);
        load_cols(cnn, cv[S], wv[S], rq[S]); // chunk k + 2
        for (; fr < ck.u; ++fr) flush_empty(fr); // rows without entries in this segment
        consume(ck, lab[S], ia[S], rv[S]);
        if (ck.last) {
            flush(ck.u, (double)ru[S]);
            fr = ck.u + 1;
        }
        ck = cn;
        have = haven;
        cn = cnn;
        haven = havenn;
    };
    while (have) {
        step(std::integral_constant<int, 0>());
        if (!have) break;
        step(std::integral_constant<int, 1>());
    }
    for (; fr < sg.rend; ++fr) flush_empty(fr);
    if (bad) flag_error(err, GEE_EVERTEX);
}

// Rows cut by segment boundaries: tail partial of the start segment plus the head
// partials of the following segments, in segment order; scaled and written once.
template <bool LAP>
__global__ void __launch_bounds__(kBT)
k_merge_group(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ seg_i,
              const int64_t *__restrict__ seg_e, int64_t nseg, int KT, const double *__restrict__ cscale,
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
        Z[u * ldz + zcol + f] = (float)(acc * column_scale(cscale[f], ru));
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

int batch_waves_per_block(int KT)
{
    // one scale table, then bins + one sink per lane for each wavefront (KT rounded up to even)
    const size_t KTp = (size_t)((KT + 1) & ~1);
    const int fit = (int)((kBatchLdsBytes / sizeof(double) - KTp) / (KTp + kWave));
    return fit < 1 ? 0 : (fit < kMaxWavesPerBlock ? fit : kMaxWavesPerBlock);
}

size_t batch_lds_bytes(int KT, int nw)
{
    const size_t KTp = (size_t)((KT + 1) & ~1);
    return sizeof(double) * (KTp + (KTp + kWave) * (size_t)nw);
}

hipError_t launch_pack_group(const int32_t *labels, int64_t n, const GroupDesc &d, void *labmat, bool u8,
                             int32_t *err, hipStream_t s)
{
    const dim3 g((unsigned)((n + kBT - 1) / kBT)), b(kBT);
    if (u8)
        hipLaunchKernelGGL(k_pack_group<uint8_t>, g, b, 0, s, labels, n, d, static_cast<uint8_t *>(labmat), err);
    else
        hipLaunchKernelGGL(k_pack_group<uint16_t>, g, b, 0, s, labels, n, d, static_cast<uint16_t *>(labmat), err);
    return hipGetLastError();
}

hipError_t launch_pack_group_hot(const int32_t *hot_ids, int64_t n_hot, int64_t n, int row_bytes, const void *labmat,
                                 void *labhot, const float *rsd, float *rsdhot, int32_t *err, hipStream_t s)
{
    if (n_hot == 0) return hipSuccess;
    if (row_bytes <= 0 || row_bytes % 8 != 0) return hipErrorInvalidValue;
    const uint8_t *src = static_cast<const uint8_t *>(labmat);
    uint8_t *dst = static_cast<uint8_t *>(labhot);
    if (row_bytes % 16 == 0)
        hipLaunchKernelGGL(k_pack_group_hot<uint4>, dim3(grid_cap(n_hot * (row_bytes / 16), kBT * 4)), dim3(kBT), 0,
                           s, hot_ids, n_hot, n, row_bytes, src, dst, rsd, rsdhot, err);
    else
        hipLaunchKernelGGL(k_pack_group_hot<uint2>, dim3(grid_cap(n_hot * (row_bytes / 8), kBT * 4)), dim3(kBT), 0,
                           s, hot_ids, n_hot, n, row_bytes, src, dst, rsd, rsdhot, err);
    return hipGetLastError();
}

hipError_t launch_group_cols(const uint64_t *counts_all, const GroupDesc &d, double *cscale, uint32_t *vmeta,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_group_cols, dim3(d.G + 1), dim3(256), 0, s, counts_all, d, cscale, vmeta);
    return hipGetLastError();
}

hipError_t launch_rsd(const double *deg, int64_t n, float *rsd, hipStream_t s)
{
    hipLaunchKernelGGL(k_rsd, dim3(grid_cap(n, 256 * 4)), dim3(256), 0, s, deg, n, rsd);
    return hipGetLastError();
}

hipError_t launch_pull_group(const GroupArgs &g, hipStream_t s)
{
    const int nw = batch_waves_per_block(g.KT);
    if (nw < 1) return hipErrorInvalidValue;
    // both label arrays through one buffer resource: 32-bit byte offsets from the lower
    // of the two, when they span less than 4 GiB (else 64-bit addresses per entry)
    const size_t lb = g.u8 ? 1 : 2;
    const uintptr_t pm = (uintptr_t)g.labmat, ph = (uintptr_t)g.labhot;
    const uintptr_t lo = g.n_hot > 0 && ph < pm ? ph : pm;
    const uintptr_t hi = std::max(pm + (size_t)(g.n + 1) * (size_t)g.Gs * lb,
                                  g.n_hot > 0 ? ph + (size_t)g.n_hot * (size_t)g.Gs * lb : pm);
    const bool span_ok = hi - lo < ((uint64_t)1 << 32) - 64;
    const uint8_t *lbase = span_ok ? reinterpret_cast<const uint8_t *>(lo) : nullptr;
    const uint32_t mat_off = span_ok ? (uint32_t)(pm - lo) : 0u;
    const uint32_t hot_off = span_ok && g.n_hot > 0 ? (uint32_t)(ph - lo) : 0u;
    const size_t lds = batch_lds_bytes(g.KT, nw);
    const unsigned blocks = (unsigned)((g.nseg + nw - 1) / nw);
#define GEE_GROUP(W, LAP, L)                                                                                         \
    hipLaunchKernelGGL((k_batch_pull<W, LAP, L>), dim3(blocks), dim3(kWave * nw), lds, s, g.n, g.row_ptr, g.col,     \
                       g.val, g.n_hot, static_cast<const L *>(g.labmat), static_cast<const L *>(g.labhot), g.Gs,     \
                       g.rsd, g.rsdhot, g.vmeta, g.cscale, g.KT, g.seg_i, g.seg_e, g.nseg, g.Z, g.ldz, g.zcol,       \
                       g.part, g.err, lbase, mat_off, hot_off)
#define GEE_GROUP_L(W, LAP)                                                                                          \
    do {                                                                                                             \
        if (g.u8) GEE_GROUP(W, LAP, uint8_t);                                                                        \
        else GEE_GROUP(W, LAP, uint16_t);                                                                            \
    } while (0)
    if (g.lap) {
        if (g.val) GEE_GROUP_L(true, true);
        else GEE_GROUP_L(false, true);
    } else {
        if (g.val) GEE_GROUP_L(true, false);
        else GEE_GROUP_L(false, false);
    }
#undef GEE_GROUP_L
#undef GEE_GROUP
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.lap)
        hipLaunchKernelGGL(k_merge_group<true>, dim3((unsigned)g.nseg), dim3(kBT), 0, s, g.n, g.row_ptr, g.seg_i,
                           g.seg_e, g.nseg, g.KT, g.cscale, g.rsd, g.part, g.Z, g.ldz, g.zcol);
    else
        hipLaunchKernelGGL(k_merge_group<false>, dim3((unsigned)g.nseg), dim3(kBT), 0, s, g.n, g.row_ptr, g.seg_i,
                           g.seg_e, g.nseg, g.KT, g.cscale, g.rsd, g.part, g.Z, g.ldz, g.zcol);
    return hipGetLastError();
}

} // namespace gee
