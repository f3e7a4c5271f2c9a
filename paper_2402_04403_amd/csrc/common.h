// Device-side helpers shared by the GEE kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gee.h"

namespace gee {

constexpr int kWave = 64;

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Store the lowest (most negative) status code seen into the caller's word.
__device__ inline void flag_error(int32_t *err, int code)
{
    if (err) atomicMin(err, code);
}

// Order LDS traffic between the lanes of one wavefront: every LDS access issued
// before this point is complete and visible to every lane after it.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes whose 8-bit value equals this lane's, within `active`.
__device__ inline uint64_t match8(uint32_t d, uint64_t active)
{
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

__device__ inline uint64_t lanemask_lt(int lane) { return lane == 0 ? 0ull : (~0ull >> (64 - lane)); }

// Per-vertex label record read by the edge-pass kernels.
//  - adjacency: the class alone, packed to 8 or 16 bits;
//  - Laplacian: 64 bits, class in the low word, d^-1/2 (FP32 bits) in the high word,
//    so one gather brings both.
template <typename P> struct LabelRec;
template <> struct LabelRec<uint8_t> {
    __device__ static int cls(uint8_t p) { return p; }
    __device__ static float rsd(uint8_t) { return 1.0f; }
};
template <> struct LabelRec<uint16_t> {
    __device__ static int cls(uint16_t p) { return p; }
    __device__ static float rsd(uint16_t) { return 1.0f; }
};
template <> struct LabelRec<uint64_t> {
    __device__ static int cls(uint64_t p) { return (int)(uint32_t)p; }
    __device__ static float rsd(uint64_t p) { return __uint_as_float((uint32_t)(p >> 32)); }
};

// floor(x / K) as a multiply-high by m = ceil(2^32 / K); exact whenever x * K < 2^32.
__device__ inline uint32_t div_small(uint32_t x, uint64_t m) { return (uint32_t)(((uint64_t)x * m) >> 32); }

// floor(x / K) as a multiply-high by m = ceil(2^64 / K) (K >= 2); exact whenever x * K < 2^64.
__device__ inline uint64_t div_big(uint64_t x, uint64_t m) { return __umul64hi(x, m); }

} // namespace gee
