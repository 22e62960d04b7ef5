// Small device helpers: wave matching, block scans, fills.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace alto {

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

__device__ inline uint64_t lanemask_lt() { return (uint64_t(1) << lane_id()) - 1; }

// Lanes of `active` whose 8-bit value equals this lane's (this lane must be
// in `active` for the result to be meaningful).  Every lane of the wave that
// is executing must call it.
__device__ inline uint64_t match_byte(uint32_t d, uint64_t active) {
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return peers;
}

// Exclusive scan over the block (blockDim.x <= 1024, multiple of 64).
// `scratch` holds at least blockDim.x/64 elements.  Returns the exclusive
// prefix; *total receives the block sum.  Contains __syncthreads.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *scratch, T *total) {
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) scratch[w] = x;
    __syncthreads();
    T wbase = 0, tot = 0;
    for (int k = 0; k < nw; k++) {
        const T s = scratch[k];
        if (k < w) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

template <typename T>
__global__ void k_fill(T *p, uint64_t n, T v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

inline unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 65536) {
    uint64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace alto
