// Labels from an embedding, gfx950: the step after the edge pass when an embedding is
// used to classify vertices, or to refine a labelling that came from a clustering
// (Section II: the labels may be a few known ground truths or the output of a
// community detection), by giving each vertex the class of its largest entry of Z.
//
// A workgroup takes a tile of rows of Z: the tile is read into LDS with coalesced
// loads (a row of Z is K consecutive floats, so a tile of rows is one contiguous run
// when ldz = K), then each thread scans one row in LDS.

#include "common.h"
#include "launch.h"

namespace gee {

namespace {

constexpr int kArgT = 128;          // rows per tile, one thread each
constexpr int kArgTileFloats = 16384; // 64 KB of LDS: tiles for K <= 128

__global__ void k_zero_u64(uint64_t *p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// out[u] = 1 + the first k with Z[u][k] equal to the row's maximum when that maximum is
// above zero, else 0 (no labelled neighbour). changed (if given) += the number of rows
// with out[u] != prev[u].
template <bool TILE>
__global__ void __launch_bounds__(kArgT)
k_argmax(int64_t n, int32_t K, int64_t ldz, const float *__restrict__ Z, const int32_t *__restrict__ prev,
         int32_t *__restrict__ out, uint64_t *changed)
{
    __shared__ float tile[TILE ? kArgTileFloats : 1];
    __shared__ uint32_t s_changed;
    const int t = threadIdx.x;
    if (t == 0) s_changed = 0;
    const int64_t r0 = (int64_t)blockIdx.x * kArgT;
    const int rows = (int)((n - r0) < kArgT ? (n - r0) : kArgT);
    if (TILE) {
        const int total = rows * K;
        const float *src = Z + r0 * K; // ldz == K here
        for (int i = t; i < total; i += kArgT) tile[i] = src[i];
    }
    __syncthreads();
    uint32_t diff = 0;
    if (t < rows) {
        const int64_t u = r0 + t;
        const float *row = TILE ? tile + (int64_t)t * K : Z + u * ldz;
        float best = 0.0f;
        int32_t lab = 0;
        for (int k = 0; k < K; ++k) {
            const float x = row[k];
            if (x > best) {
                best = x;
                lab = k + 1;
            }
        }
        out[u] = lab;
        diff = prev && prev[u] != lab ? 1u : 0u;
    }
    if (changed) {
        if (diff) atomicAdd(&s_changed, 1u);
        __syncthreads();
        if (t == 0 && s_changed) atomicAdd(reinterpret_cast<unsigned long long *>(changed), (unsigned long long)s_changed);
    }
}

} // namespace

hipError_t launch_argmax(int64_t n, int32_t K, int64_t ldz, const float *Z, const int32_t *prev, int32_t *out,
                         uint64_t *changed, hipStream_t s)
{
    if (changed) {
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, changed);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)((n + kArgT - 1) / kArgT));
    if (ldz == K && (int64_t)K * kArgT <= kArgTileFloats)
        hipLaunchKernelGGL(k_argmax<true>, grid, dim3(kArgT), 0, s, n, K, ldz, Z, prev, out, changed);
    else
        hipLaunchKernelGGL(k_argmax<false>, grid, dim3(kArgT), 0, s, n, K, ldz, Z, prev, out, changed);
    return hipGetLastError();
}

} // namespace gee
