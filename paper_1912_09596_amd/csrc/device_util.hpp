// device_util.hpp -- small device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace esk {

// Exclusive scan of one value per thread over a THREADS-thread block (wave64
// shuffles, then one LDS slot per wave).  The block total goes to *total.
// `scratch` needs THREADS/64 + 1 slots.  Every thread of the block must call.
template <int THREADS>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *scratch, uint32_t *total)
{
    constexpr int WAVES = THREADS / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) scratch[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < WAVES; ++w) {
            uint32_t t = scratch[w];
            scratch[w] = run;
            run += t;
        }
        scratch[WAVES] = run;
    }
    __syncthreads();
    uint32_t r = scratch[wave] + x - v;
    *total = scratch[WAVES];
    __syncthreads();
    return r;
}

// LDS visibility between the lanes of one wave
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// box [lo, hi) in voxels (each < 65536) as three words of two uint16
__device__ inline void pack_box(const int lo[3], const int hi[3], uint32_t w[3])
{
    w[0] = (uint32_t)lo[0] | ((uint32_t)lo[1] << 16);
    w[1] = (uint32_t)lo[2] | ((uint32_t)hi[0] << 16);
    w[2] = (uint32_t)hi[1] | ((uint32_t)hi[2] << 16);
}

__device__ inline void unpack_box_u(uint32_t w0, uint32_t w1, uint32_t w2, int lo[3], int hi[3])
{
    lo[0] = (int)(w0 & 0xffffu);
    lo[1] = (int)(w0 >> 16);
    lo[2] = (int)(w1 & 0xffffu);
    hi[0] = (int)(w1 >> 16);
    hi[1] = (int)(w2 & 0xffffu);
    hi[2] = (int)(w2 >> 16);
}

}  // namespace esk
