// Device helpers: 64-lane wavefront reductions and broadcasts.
#pragma once

#include <hip/hip_runtime.h>

namespace tmlib {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Uniform (scalar) copy of a wave-uniform value.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// Orders a wave's LDS accesses across its lanes: what a lane wrote before
// is seen by the wave's reads after (the compiler may not move memory
// operations across it; the hardware keeps a wave's LDS operations in order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace tmlib
