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

}  // namespace tmlib
