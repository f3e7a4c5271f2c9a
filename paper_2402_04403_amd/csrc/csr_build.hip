// Canonical symmetric CSR build on gfx950.
//
// Each record (u, v, w) becomes two directed entries, (u -> v, w) and (v -> u, w),
// keyed by (row, column) packed into the low 2b bits of a 64-bit word (b = bits
// of n - 1). A stable LSD radix sort (8-bit digits) orders the 2s entries by the
// bit pattern of w first (weighted graphs only) and then by the key, so rows come
// out sorted by (column, w bits) and the layout depends only on the multiset of
// records. A final pass splits keys into col and derives row_ptr from the last
// entry of each row with an inclusive max-scan (empty rows inherit the end of
// the row before them).
//
// Each radix pass is three kernels: per-tile digit histograms, an exclusive scan
// of the digit-major histogram table, and a scatter that ranks items stably
// inside the tile (wavefront ballots), reorders the tile in LDS and writes runs
// of equal digits contiguously.

#include "common.h"
#include "launch.h"

namespace gee {

namespace {

constexpr int kT = 256;           // threads per block
constexpr int kItems = 16;        // items per thread
constexpr int kTile = kT * kItems; // 4096 items per tile
constexpr int kWaveItems = kTile / (kT / kWave);

inline int64_t tiles(int64_t N) { return (N + kTile - 1) / kTile; }

__device__ inline uint32_t digit_of(uint64_t key, float v, int shift, bool from_val)
{
    return from_val ? ((__float_as_uint(v) >> shift) & 0xffu) : (uint32_t)((key >> shift) & 0xffu);
}

// ------------------------------------------------------------ expand ----

template <bool W>
__global__ void __launch_bounds__(kT)
k_expand(int64_t n, int64_t ns, const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
         const float *__restrict__ w, int nb, uint64_t *__restrict__ keys, float *__restrict__ vals, int32_t *err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t u = (uint32_t)src[i], v = (uint32_t)dst[i];
        if (u >= (uint64_t)n || v >= (uint64_t)n) {
            flag_error(err, GEE_EVERTEX);
            u = v = 0; // keeps every later index in range; the output is unspecified now
        }
        keys[2 * i] = (u << nb) | v;
        keys[2 * i + 1] = (v << nb) | u;
        if (W) {
            const float x = w[i];
            vals[2 * i] = x;
            vals[2 * i + 1] = x;
        }
    }
}

// ------------------------------------------------------------- radix ----

template <bool HV>
__device__ inline void load_tile(const uint64_t *__restrict__ kin, const float *__restrict__ vin, int64_t N,
                                 int64_t tile0, int wave, int lane, uint64_t (&key)[kItems], float (&val)[kItems],
                                 bool (&valid)[kItems])
{
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int64_t idx = tile0 + (int64_t)wave * kWaveItems + i * kWave + lane;
        valid[i] = idx < N;
        key[i] = valid[i] ? kin[idx] : 0;
        val[i] = (HV && valid[i]) ? vin[idx] : 0.0f;
    }
}

// Digit histogram of one tile, written digit-major: hist[d * ntiles + tile].
template <bool HV>
__global__ void __launch_bounds__(kT)
k_radix_hist(const uint64_t *__restrict__ kin, const float *__restrict__ vin, int64_t N, int shift, bool from_val,
             uint32_t *__restrict__ hist, int64_t ntiles)
{
    __shared__ uint32_t h[256];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    h[t] = 0;
    __syncthreads();
    uint64_t key[kItems];
    float val[kItems];
    bool valid[kItems];
    load_tile<HV>(kin, vin, N, (int64_t)blockIdx.x * kTile, wave, lane, key, val, valid);
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const uint32_t d = digit_of(key[i], val[i], shift, from_val);
        const uint64_t peers = match8(d, __ballot(valid[i]));
        if (valid[i] && (peers & lanemask_lt(lane)) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)t * ntiles + blockIdx.x] = h[t];
}

// Block-wide exclusive sum of one uint32 per thread (256 threads).
__device__ inline uint32_t block_excl_sum_u32(uint32_t x, uint32_t *scratch /* >= 4 */)
{
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) scratch[wave] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += scratch[w];
    __syncthreads();
    return base + inc - x;
}

template <bool HV>
__global__ void __launch_bounds__(kT)
k_radix_scatter(const uint64_t *__restrict__ kin, const float *__restrict__ vin, uint64_t *__restrict__ kout,
                float *__restrict__ vout, int64_t N, int shift, bool from_val, const int64_t *__restrict__ offs,
                int64_t ntiles)
{
    __shared__ uint64_t tk[kTile];
    __shared__ float tv[HV ? kTile : 1];
    __shared__ uint32_t cnt[kT / kWave][256];
    __shared__ uint32_t dstart[256];
    __shared__ int64_t gofs[256];
    __shared__ uint32_t scratch[4];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t tile0 = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int w = 0; w < kT / kWave; ++w) cnt[w][t] = 0;
    gofs[t] = offs[(int64_t)t * ntiles + blockIdx.x];
    __syncthreads();

    uint64_t key[kItems];
    float val[kItems];
    bool valid[kItems];
    uint32_t rank[kItems];
    uint32_t dig[kItems];
    load_tile<HV>(kin, vin, N, tile0, wave, lane, key, val, valid);
    // stable rank within the wavefront's 1024 items, taken in (i, lane) order
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const uint32_t d = digit_of(key[i], val[i], shift, from_val);
        const uint64_t peers = match8(d, __ballot(valid[i]));
        const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt(lane));
        const uint32_t base = valid[i] ? cnt[wave][d] : 0u;
        wave_sync();
        if (valid[i] && below == 0) cnt[wave][d] = base + (uint32_t)__popcll(peers);
        wave_sync();
        rank[i] = base + below;
        dig[i] = d;
    }
    __syncthreads();
    // thread t owns digit t: tile-local start of the digit and of each wavefront's run
    const uint32_t c0 = cnt[0][t], c1 = cnt[1][t], c2 = cnt[2][t], c3 = cnt[3][t];
    const uint32_t start = block_excl_sum_u32(c0 + c1 + c2 + c3, scratch);
    dstart[t] = start;
    cnt[0][t] = start;
    cnt[1][t] = start + c0;
    cnt[2][t] = start + c0 + c1;
    cnt[3][t] = start + c0 + c1 + c2;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (!valid[i]) continue;
        const uint32_t pos = cnt[wave][dig[i]] + rank[i];
        if (pos >= (uint32_t)kTile) continue; // cannot happen when the ranks are consistent
        tk[pos] = key[i];
        if (HV) tv[pos] = val[i];
    }
    __syncthreads();
    const int64_t left = N - tile0;
    const int nvalid = left < kTile ? (int)left : kTile;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int p = i * kT + t;
        if (p >= nvalid) continue;
        const uint64_t k = tk[p];
        const float v = HV ? tv[p] : 0.0f;
        const uint32_t d = digit_of(k, v, shift, from_val);
        const int64_t o = gofs[d] + (p - (int64_t)dstart[d]);
        if (o < 0 || o >= N) continue; // cannot happen when histogram and scatter agree
        kout[o] = k;
        if (HV) vout[o] = v;
    }
}

// --------------------------------------------------------------- scan ----

struct SumOp {
    __device__ int64_t operator()(int64_t a, int64_t b) const { return a + b; }
    static constexpr int64_t identity = 0;
};
struct MaxOp {
    __device__ int64_t operator()(int64_t a, int64_t b) const { return a > b ? a : b; }
    static constexpr int64_t identity = INT64_MIN;
};

template <typename Op> __device__ inline int64_t wave_incl_scan(int64_t x, Op op)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x = op(x, y);
    }
    return x;
}

// Exclusive scan of one value per thread over the block; returns (exclusive, total).
template <typename Op> __device__ inline int64_t block_excl_scan(int64_t x, Op op, int64_t *sh, int64_t &total)
{
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t inc = wave_incl_scan(x, op);
    if (lane == kWave - 1) sh[wave] = inc;
    __syncthreads();
    int64_t base = Op::identity;
    for (int w = 0; w < wave; ++w) base = op(base, sh[w]);
    total = Op::identity;
    for (int w = 0; w < kT / kWave; ++w) total = op(total, sh[w]);
    __syncthreads();
    const int64_t prev = __shfl_up(inc, 1);
    const int64_t excl_in_wave = lane == 0 ? Op::identity : prev;
    return op(base, excl_in_wave);
}

template <typename In, typename Op>
__global__ void __launch_bounds__(kT) k_scan_reduce(const In *__restrict__ in, int64_t N, int64_t *__restrict__ part, Op op)
{
    __shared__ int64_t sh[kT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int64_t acc = Op::identity;
    for (int i = 0; i < kItems; ++i)
        if (base + i < N) acc = op(acc, (int64_t)in[base + i]);
    int64_t total;
    block_excl_scan(acc, op, sh, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Exclusive scan of the block partials in place, one block walking all chunks.
template <typename Op> __global__ void __launch_bounds__(kT) k_scan_top(int64_t *__restrict__ part, int64_t np, Op op)
{
    __shared__ int64_t sh[kT / kWave];
    int64_t carry = Op::identity;
    for (int64_t c0 = 0; c0 < np; c0 += kT) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t x = i < np ? part[i] : Op::identity;
        int64_t total;
        const int64_t ex = block_excl_scan(x, op, sh, total);
        if (i < np) part[i] = op(carry, ex);
        carry = op(carry, total);
    }
}

template <typename In, typename Op>
__global__ void __launch_bounds__(kT)
k_scan_apply(const In *__restrict__ in, int64_t N, const int64_t *__restrict__ part, int64_t *__restrict__ out, Op op,
             bool inclusive)
{
    __shared__ int64_t sh[kT / kWave];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    int64_t acc = Op::identity;
    for (int i = 0; i < kItems; ++i)
        if (base + i < N) acc = op(acc, (int64_t)in[base + i]);
    int64_t total;
    int64_t run = op(part[blockIdx.x], block_excl_scan(acc, op, sh, total));
    for (int i = 0; i < kItems; ++i) {
        if (base + i >= N) break;
        const int64_t x = (int64_t)in[base + i];
        if (inclusive) {
            run = op(run, x);
            out[base + i] = run;
        } else {
            out[base + i] = run;
            run = op(run, x);
        }
    }
}

template <typename In, typename Op>
hipError_t scan(const In *in, int64_t N, int64_t *out, int64_t *part, Op op, bool inclusive, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    const int64_t nt = tiles(N);
    hipLaunchKernelGGL((k_scan_reduce<In, Op>), dim3((unsigned)nt), dim3(kT), 0, s, in, N, part, op);
    hipLaunchKernelGGL((k_scan_top<Op>), dim3(1), dim3(kT), 0, s, part, nt, op);
    hipLaunchKernelGGL((k_scan_apply<In, Op>), dim3((unsigned)nt), dim3(kT), 0, s, in, N, part, out, op, inclusive);
    return hipGetLastError();
}

// ----------------------------------------------------------- finalize ----

// col[j] = low b bits of key j (and val[j]); rowlast[row] = j + 1 when j is the
// last entry of its row.
template <bool HV>
__global__ void __launch_bounds__(kT)
k_finalize(const uint64_t *__restrict__ keys, const float *__restrict__ vin, int64_t N, int64_t n, int nb,
           int32_t *__restrict__ col, float *__restrict__ vout, int64_t *__restrict__ rowlast)
{
    const uint64_t mask = (nb >= 64) ? ~0ull : ((1ull << nb) - 1ull);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[j];
        col[j] = (int32_t)(k & mask);
        if (HV) vout[j] = vin[j];
        const uint64_t row = k >> nb;
        if (row < (uint64_t)n && (j + 1 == N || (keys[j + 1] >> nb) != row)) rowlast[row] = j + 1;
    }
}

// -------------------------------------------------- hot-vertex selection ----
//
// The n_hot vertices of highest degree (ties broken by smaller id) get slots
// 0..n_hot-1 in id order, and every CSR column naming one of them is rewritten
// as (slot | 2^31). The pull pass then gathers these labels from a compact table
// of n_hot records, small enough to stay in L2, instead of from the n-entry
// label array. Degrees above kDegBins - 1 share the top bucket.

constexpr int kDegBins = 4096;

__device__ inline int deg_bucket(const int64_t *__restrict__ row_ptr, int64_t v)
{
    const int64_t d = row_ptr[v + 1] - row_ptr[v];
    return d <= 0 ? 0 : (d >= kDegBins - 1 ? kDegBins - 1 : (int)d);
}

__global__ void __launch_bounds__(kT) k_deg_hist(int64_t n, const int64_t *__restrict__ row_ptr, int64_t *hist)
{
    __shared__ uint32_t h[kDegBins];
    for (int b = threadIdx.x; b < kDegBins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[deg_bucket(row_ptr, v)], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < kDegBins; b += blockDim.x)
        if (h[b]) atomicAdd((unsigned long long *)&hist[b], (unsigned long long)h[b]);
}

// par[0] = bucket T with #(bucket >= T) >= H > #(bucket > T); par[1] = how many
// bucket-T vertices (the lowest ids) join the hot set.
__global__ void k_hot_threshold(const int64_t *__restrict__ hist, int64_t H, int64_t *par)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t above = 0;
    int T = 0;
    int64_t quota = H;
    for (int b = kDegBins - 1; b >= 0; --b) {
        if (above + hist[b] >= H) {
            T = b;
            quota = H - above;
            break;
        }
        above += hist[b];
    }
    par[0] = T;
    par[1] = quota;
}

__global__ void __launch_bounds__(kT)
k_hot_eq(int64_t n, const int64_t *__restrict__ row_ptr, const int64_t *__restrict__ par, int64_t *__restrict__ eq)
{
    const int T = (int)par[0];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        eq[v] = deg_bucket(row_ptr, v) == T;
}

__global__ void __launch_bounds__(kT)
k_hot_flag(int64_t n, const int64_t *__restrict__ row_ptr, const int64_t *__restrict__ par,
           const int64_t *__restrict__ eqrank, int64_t *__restrict__ hot)
{
    const int T = (int)par[0];
    const int64_t quota = par[1];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int b = deg_bucket(row_ptr, v);
        hot[v] = b > T || (b == T && eqrank[v] < quota);
    }
}

// Hot vertices in id order: hkeys[pos[v]] = ((kDegBins - 1 - bucket) << 32) | v, so
// that a stable sort on the upper word orders them by degree bucket, highest first,
// ties by id. The flag array becomes the slot map, reset to -1 here.
__global__ void __launch_bounds__(kT)
k_hot_compact(int64_t n, const int64_t *__restrict__ row_ptr, int64_t *__restrict__ flag_to_map,
              const int64_t *__restrict__ pos, int64_t n_hot, uint64_t *__restrict__ hkeys)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool hot = flag_to_map[v] != 0;
        const int64_t p = pos[v];
        if (hot && p < n_hot)
            hkeys[p] = ((uint64_t)(kDegBins - 1 - deg_bucket(row_ptr, v)) << 32) | (uint64_t)(uint32_t)v;
        flag_to_map[v] = -1;
    }
}

// Slot = rank in (degree bucket desc, id asc): the hottest labels share the first
// cache lines of the hot table.
__global__ void __launch_bounds__(kT)
k_hot_ids(int64_t n, int64_t n_hot, const uint64_t *__restrict__ hkeys, int64_t *__restrict__ map,
          int32_t *__restrict__ hot_ids)
{
    for (int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sl < n_hot; sl += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)hkeys[sl];
        hot_ids[sl] = (int32_t)v;
        if ((uint64_t)v < (uint64_t)n) map[v] = sl;
    }
}

__global__ void __launch_bounds__(kT)
k_col_encode(int64_t N, int64_t n, int32_t *__restrict__ col, const int64_t *__restrict__ map)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = col[j];
        if ((uint32_t)c >= (uint64_t)n) continue;
        const int64_t sl = map[c];
        if (sl >= 0) col[j] = (int32_t)((uint32_t)sl | 0x80000000u);
    }
}

__global__ void k_fill_i64(int64_t *__restrict__ p, int64_t count, int64_t value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

inline int grid_cap(int64_t items, int per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (1 << 20)) g = 1 << 20;
    return (int)g;
}

int key_bits(int64_t n)
{
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < n) ++b;
    return b < 1 ? 1 : b;
}

} // namespace

size_t csr_build_layout(int64_t n, int64_t s, bool weighted, int64_t n_hot, char *base, CsrBuildWs *out)
{
    const int64_t N = 2 * s;
    const int64_t nt = tiles(N > 0 ? N : 1);
    const int64_t nt_hot = tiles(n_hot > 0 ? n_hot : 1);
    const int64_t hist_len = 256 * (nt > nt_hot ? nt : nt_hot);
    const int64_t scan_len = (hist_len > n ? hist_len : n);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = align_up(off, 256);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    CsrBuildWs w{};
    w.keys[0] = (uint64_t *)take((size_t)N * 8);
    w.keys[1] = (uint64_t *)take((size_t)N * 8);
    w.vals[0] = weighted ? (float *)take((size_t)N * 4) : nullptr;
    w.vals[1] = weighted ? (float *)take((size_t)N * 4) : nullptr;
    w.hist = (uint32_t *)take((size_t)hist_len * 4);
    w.offs = (int64_t *)take((size_t)hist_len * 8);
    w.scan_part = (int64_t *)take((size_t)tiles(scan_len) * 8 + 8);
    w.rowlast = (int64_t *)take((size_t)n * 8);
    if (n_hot > 0) {
        w.vtmp[0] = (int64_t *)take((size_t)n * 8);
        w.vtmp[1] = (int64_t *)take((size_t)n * 8);
        w.hkeys[0] = (uint64_t *)take((size_t)n_hot * 8);
        w.hkeys[1] = (uint64_t *)take((size_t)n_hot * 8);
        w.hot_hist = (int64_t *)take((size_t)kDegBins * 8);
        w.hot_par = (int64_t *)take(2 * 8);
    }
    if (out) *out = w;
    return align_up(off, 256);
}

size_t radix_scratch_bytes(int64_t N, int64_t scan_n, size_t *hist_bytes, size_t *offs_bytes, size_t *part_bytes)
{
    const int64_t nt = tiles(N > 0 ? N : 1);
    const int64_t hist_len = 256 * nt;
    const int64_t scan_len = hist_len > scan_n ? hist_len : scan_n;
    *hist_bytes = (size_t)hist_len * 4;
    *offs_bytes = (size_t)hist_len * 8;
    *part_bytes = (size_t)tiles(scan_len) * 8 + 8;
    return *hist_bytes + *offs_bytes + *part_bytes;
}

hipError_t radix_sort_bits_kv(uint64_t *keys0, uint64_t *keys1, float *vals0, float *vals1, int64_t N, int lo, int hi,
                              uint32_t *hist, int64_t *offs, int64_t *scan_part, uint64_t **rkeys, float **rvals,
                              hipStream_t s)
{
    uint64_t *kb[2] = {keys0, keys1};
    float *vb[2] = {vals0, vals1};
    int cur = 0;
    const int64_t nt = tiles(N);
    hipError_t e;
    for (int sh = lo; N > 0 && sh < hi; sh += 8) {
        hipLaunchKernelGGL(k_radix_hist<true>, dim3((unsigned)nt), dim3(kT), 0, s, kb[cur], vb[cur], N, sh, false, hist,
                           nt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan(hist, 256 * nt, offs, scan_part, SumOp{}, false, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nt), dim3(kT), 0, s, kb[cur], vb[cur], kb[cur ^ 1],
                           vb[cur ^ 1], N, sh, false, offs, nt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        cur ^= 1;
    }
    *rkeys = kb[cur];
    *rvals = vb[cur];
    return hipSuccess;
}

hipError_t radix_sort_bits(uint64_t *keys0, uint64_t *keys1, int64_t N, int lo, int hi, uint32_t *hist,
                           int64_t *offs, int64_t *scan_part, uint64_t **result, hipStream_t s)
{
    uint64_t *buf[2] = {keys0, keys1};
    int cur = 0;
    const int64_t nt = tiles(N);
    hipError_t e;
    for (int sh = lo; N > 0 && sh < hi; sh += 8) {
        hipLaunchKernelGGL(k_radix_hist<false>, dim3((unsigned)nt), dim3(kT), 0, s, buf[cur], (const float *)nullptr,
                           N, sh, false, hist, nt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan(hist, 256 * nt, offs, scan_part, SumOp{}, false, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nt), dim3(kT), 0, s, buf[cur], (const float *)nullptr,
                           buf[cur ^ 1], (float *)nullptr, N, sh, false, offs, nt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        cur ^= 1;
    }
    *result = buf[cur];
    return hipSuccess;
}

hipError_t max_scan_i64(const int64_t *in, int64_t N, int64_t *out, int64_t *scan_part, hipStream_t s)
{
    return scan(in, N, out, scan_part, MaxOp{}, true, s);
}

hipError_t launch_fill_i64(int64_t *p, int64_t count, int64_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_cap(count, kT * 4)), dim3(kT), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_csr_build(int64_t n, int64_t ns, const int32_t *src, const int32_t *dst, const float *w,
                            int64_t n_hot, int64_t *row_ptr, int32_t *col, float *val, int32_t *hot_ids,
                            const CsrBuildWs &ws, int32_t *err, hipStream_t s)
{
    const int64_t N = 2 * ns;
    const bool HV = w != nullptr;
    const int nb = key_bits(n);
    hipError_t e;
    if (N > 0) {
        if (HV)
            hipLaunchKernelGGL(k_expand<true>, dim3(grid_cap(ns, kT * 4)), dim3(kT), 0, s, n, ns, src, dst, w, nb,
                               ws.keys[0], ws.vals[0], err);
        else
            hipLaunchKernelGGL(k_expand<false>, dim3(grid_cap(ns, kT * 4)), dim3(kT), 0, s, n, ns, src, dst, w, nb,
                               ws.keys[0], ws.vals[0], err);
        if ((e = hipGetLastError()) != hipSuccess) return e;

        // passes: w bits (weighted only), then the 2b key bits
        struct Pass {
            int shift;
            bool from_val;
        };
        Pass passes[16];
        int np = 0;
        if (HV)
            for (int sh = 0; sh < 32; sh += 8) passes[np++] = {sh, true};
        for (int sh = 0; sh < 2 * nb; sh += 8) passes[np++] = {sh, false};
        const int64_t nt = tiles(N);
        int cur = 0;
        for (int p = 0; p < np; ++p) {
            const uint64_t *kin = ws.keys[cur];
            uint64_t *kout = ws.keys[cur ^ 1];
            const float *vin = ws.vals[cur];
            float *vout = ws.vals[cur ^ 1];
            if (HV)
                hipLaunchKernelGGL(k_radix_hist<true>, dim3((unsigned)nt), dim3(kT), 0, s, kin, vin, N,
                                   passes[p].shift, passes[p].from_val, ws.hist, nt);
            else
                hipLaunchKernelGGL(k_radix_hist<false>, dim3((unsigned)nt), dim3(kT), 0, s, kin, vin, N,
                                   passes[p].shift, passes[p].from_val, ws.hist, nt);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = scan(ws.hist, 256 * nt, ws.offs, ws.scan_part, SumOp{}, false, s)) != hipSuccess) return e;
            if (HV)
                hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nt), dim3(kT), 0, s, kin, vin, kout, vout, N,
                                   passes[p].shift, passes[p].from_val, ws.offs, nt);
            else
                hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nt), dim3(kT), 0, s, kin, vin, kout, vout,
                                   N, passes[p].shift, passes[p].from_val, ws.offs, nt);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            cur ^= 1;
        }
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_cap(n, kT * 4)), dim3(kT), 0, s, ws.rowlast, n, (int64_t)0);
        if (HV)
            hipLaunchKernelGGL(k_finalize<true>, dim3(grid_cap(N, kT * 4)), dim3(kT), 0, s, ws.keys[cur],
                               ws.vals[cur], N, n, nb, col, val, ws.rowlast);
        else
            hipLaunchKernelGGL(k_finalize<false>, dim3(grid_cap(N, kT * 4)), dim3(kT), 0, s, ws.keys[cur],
                               ws.vals[cur], N, n, nb, col, val, ws.rowlast);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_cap(n, kT * 4)), dim3(kT), 0, s, ws.rowlast, n, (int64_t)0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // row_ptr[0] = 0; row_ptr[u + 1] = max over rows r <= u of rowlast[r]
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(1), 0, s, row_ptr, (int64_t)1, (int64_t)0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan(ws.rowlast, n, row_ptr + 1, ws.scan_part, MaxOp{}, true, s)) != hipSuccess) return e;
    if (n_hot <= 0) return hipSuccess;

    // hot-vertex slots and column encoding
    const dim3 gv(grid_cap(n, kT * 4)), b(kT);
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_cap(kDegBins, kT)), b, 0, s, ws.hot_hist, (int64_t)kDegBins, (int64_t)0);
    hipLaunchKernelGGL(k_deg_hist, dim3(grid_cap(n, kT * 16)), b, 0, s, n, (const int64_t *)row_ptr, ws.hot_hist);
    hipLaunchKernelGGL(k_hot_threshold, dim3(1), dim3(64), 0, s, (const int64_t *)ws.hot_hist, n_hot, ws.hot_par);
    hipLaunchKernelGGL(k_hot_eq, gv, b, 0, s, n, (const int64_t *)row_ptr, (const int64_t *)ws.hot_par, ws.vtmp[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan(ws.vtmp[0], n, ws.vtmp[1], ws.scan_part, SumOp{}, false, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_hot_flag, gv, b, 0, s, n, (const int64_t *)row_ptr, (const int64_t *)ws.hot_par,
                       (const int64_t *)ws.vtmp[1], ws.vtmp[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan(ws.vtmp[0], n, ws.vtmp[1], ws.scan_part, SumOp{}, false, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_hot_compact, gv, b, 0, s, n, (const int64_t *)row_ptr, ws.vtmp[0],
                       (const int64_t *)ws.vtmp[1], n_hot, ws.hkeys[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // stable sort of the hot keys on the 12 bucket bits above bit 32
    const int64_t ntk = tiles(n_hot);
    int hc = 0;
    for (int sh = 32; sh < 32 + 12; sh += 8) {
        hipLaunchKernelGGL(k_radix_hist<false>, dim3((unsigned)ntk), b, 0, s, ws.hkeys[hc], (const float *)nullptr,
                           n_hot, sh, false, ws.hist, ntk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan(ws.hist, 256 * ntk, ws.offs, ws.scan_part, SumOp{}, false, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)ntk), b, 0, s, ws.hkeys[hc], (const float *)nullptr,
                           ws.hkeys[hc ^ 1], (float *)nullptr, n_hot, sh, false, ws.offs, ntk);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hc ^= 1;
    }
    hipLaunchKernelGGL(k_hot_ids, dim3(grid_cap(n_hot, kT * 4)), b, 0, s, n, n_hot, (const uint64_t *)ws.hkeys[hc],
                       ws.vtmp[0], hot_ids);
    hipLaunchKernelGGL(k_col_encode, dim3(grid_cap(N, kT * 4)), b, 0, s, N, n, col, (const int64_t *)ws.vtmp[0]);
    return hipGetLastError();
}

} // namespace gee
