// rj_wave.h -- wavefront (64-lane) and block reductions used by the
// statistics and score kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace rj {

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide min / max (every thread of the block must call; s holds one int
// per wave and is not reused by the caller before the next barrier).
__device__ __forceinline__ int block_min_i32(int v, int* s) {
    v = wave_min_i32(v);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = s[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = min(r, s[i]);
    return r;
}

__device__ __forceinline__ int block_max_i32(int v, int* s) {
    v = wave_max_i32(v);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = s[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = max(r, s[i]);
    return r;
}

} // namespace rj
