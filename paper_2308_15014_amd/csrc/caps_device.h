// Device-side helpers shared by the libcaps kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace caps {

constexpr int kWave = 64;

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

// Inclusive scan of v over the 64 lanes of a wave.
__device__ inline int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan over a block of NT threads (NT a multiple of 64, <= 1024).
// `scratch` holds NT/64 + 1 ints of LDS.  Returns the thread's exclusive
// prefix; *total receives the block sum.  Contains __syncthreads().
template <int NT>
__device__ inline int block_excl_scan(int v, int *scratch, int *total) {
    constexpr int NW = NT / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) scratch[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < NW; i++) {
            int t = scratch[i];
            scratch[i] = s;
            s += t;
        }
        scratch[NW] = s;
    }
    __syncthreads();
    int r = scratch[w] + inc - v;
    *total = scratch[NW];
    __syncthreads();
    return r;
}

__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint64_t u = __shfl_xor(v, o, kWave);
        v = u < v ? u : v;
    }
    return v;
}

__device__ inline uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint64_t u = __shfl_xor(v, o, kWave);
        v = u > v ? u : v;
    }
    return v;
}

// Lanes of the wave whose `key` equals this lane's key (key < 2^nbits).
__device__ inline uint64_t wave_match(uint32_t key, int nbits) {
    uint64_t peers = __ballot(1);
    for (int b = 0; b < nbits; b++) {
        uint64_t bal = __ballot((key >> b) & 1u);
        peers &= ((key >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

}  // namespace caps
