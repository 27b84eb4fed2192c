// tm_prefilter: the library pre-filter of Section 2.2 (Fig. 3). Patterns and
// templates are integrated over the azimuth; one matrix product correlates
// every pattern profile with every template profile, and only the best
// correlating templates go on to the full in-plane search.
//
//   score[b, t] = sum_j prof_T[t, j] prof_P[j, b]
//
// with prof_T the template profiles normalised to unit length (so ranking a
// pattern's row equals ranking the cosine). The product runs on the matrix
// cores in float32, bf16, fp16 or fp8 (e4m3, each template profile scaled to
// maximum 1 and each pattern profile to maximum 1, the template scale put
// back after accumulation), always with float32 accumulation:
//   * v_mfma_f32_32x32x2_f32 / 32x32x16_bf16 / 32x32x16_f16 / 32x32x16_fp8_fp8;
//   * one wave computes a 32 (templates) x 32 (patterns) tile, a workgroup of
//     four waves 128 x 32, over K = R radii.
// Per pattern a radix select then keeps the n_keep largest scores (ties to
// the lower template index) and writes their indices in ascending order.
#include <algorithm>
#include <cmath>

#include "tm_device.h"
#include "tm_internal.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

__device__ __forceinline__ short to_bf16(float x) {
    // round to nearest even (inputs are finite)
    const uint32_t u = __float_as_uint(x);
    return static_cast<short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Per pattern b: scale = 1 / max_j |prof_P[j, b]| (1 if the profile is zero).
__device__ __forceinline__ float pattern_scale(const float* __restrict__ prof_p, int R, int B,
                                               int b, int lane) {
    float m = 0.0f;
    if (b < B)
        for (int k = (lane >> 5); k < R; k += 2) m = fmaxf(m, fabsf(prof_p[static_cast<size_t>(k) * B + b]));
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    return m > 0.0f ? 1.0f / m : 1.0f;
}

template <int PREC>
__global__ void __launch_bounds__(256)
prefilter_scores(const float* __restrict__ prof_t, const float* __restrict__ tmax,
                 const float* __restrict__ prof_p, int T, int R, int B, float* __restrict__ S) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = lane & 31, h = lane >> 5;
    const int t0 = blockIdx.x * 128 + wave * 32;
    const int b0 = blockIdx.y * 32;
    const int t = t0 + m, b = b0 + m;
    const float* trow = prof_t + static_cast<size_t>(t < T ? t : 0) * R;
    f32x16_t acc = {};
    if constexpr (PREC == TM_PREC_FP32) {
        for (int k0 = 0; k0 < R; k0 += 2) {
            const int k = k0 + h;
            const float a = (t < T && k < R) ? trow[k] : 0.0f;
            const float x = (b < B && k < R) ? prof_p[static_cast<size_t>(k) * B + b] : 0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, x, acc, 0, 0, 0);
        }
    } else {
        const float ps = pattern_scale(prof_p, R, B, b, lane);
        const float ts = (PREC == TM_PREC_FP8 && t < T && tmax[t] > 0.0f) ? 1.0f / tmax[t] : 1.0f;
        for (int k0 = 0; k0 < R; k0 += 16) {
            float a[8], x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + 8 * h + e;
                a[e] = (t < T && k < R) ? trow[k] * ts : 0.0f;
                x[e] = (b < B && k < R) ? prof_p[static_cast<size_t>(k) * B + b] * ps : 0.0f;
            }
            if constexpr (PREC == TM_PREC_BF16) {
                bf16x8_t A, X;
#pragma unroll
                for (int e = 0; e < 8; ++e) { A[e] = to_bf16(a[e]); X[e] = to_bf16(x[e]); }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, X, acc, 0, 0, 0);
            } else if constexpr (PREC == TM_PREC_FP16) {
                f16x8_t A, X;
#pragma unroll
                for (int e = 0; e < 8; ++e) { A[e] = static_cast<_Float16>(a[e]); X[e] = static_cast<_Float16>(x[e]); }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, X, acc, 0, 0, 0);
            } else {
                int alo = 0, ahi = 0, xlo = 0, xhi = 0;
                alo = __builtin_amdgcn_cvt_pk_fp8_f32(a[0], a[1], alo, false);
                alo = __builtin_amdgcn_cvt_pk_fp8_f32(a[2], a[3], alo, true);
                ahi = __builtin_amdgcn_cvt_pk_fp8_f32(a[4], a[5], ahi, false);
                ahi = __builtin_amdgcn_cvt_pk_fp8_f32(a[6], a[7], ahi, true);
                xlo = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], xlo, false);
                xlo = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], xlo, true);
                xhi = __builtin_amdgcn_cvt_pk_fp8_f32(x[4], x[5], xhi, false);
                xhi = __builtin_amdgcn_cvt_pk_fp8_f32(x[6], x[7], xhi, true);
                const long A = static_cast<long>(static_cast<uint32_t>(alo)) | (static_cast<long>(ahi) << 32);
                const long X = static_cast<long>(static_cast<uint32_t>(xlo)) | (static_cast<long>(xhi) << 32);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(A, X, acc, 0, 0, 0);
            }
        }
    }
    // D[i][j]: j = lane % 32 (pattern), i = 8 (v / 4) + 4 (lane / 32) + v % 4 (template)
    if (b < B) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int tt = t0 + 8 * (v >> 2) + 4 * h + (v & 3);
            if (tt < T) {
                const float sc = (PREC == TM_PREC_FP8 && tmax[tt] > 0.0f) ? tmax[tt] : 1.0f;
                S[static_cast<size_t>(b) * T + tt] = acc[v] * sc;
            }
        }
    }
}

// Order-preserving unsigned key of a finite float (larger float, larger key).
__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int kSelThreads = 256;

// One workgroup per pattern: the n_keep largest keys of S[b, :] (ties to the
// lower index) by a four-pass 8-bit radix select, then an ordered compaction.
__global__ void __launch_bounds__(kSelThreads)
select_kept(const float* __restrict__ S, int T, int n_keep, int32_t* __restrict__ items,
            int n_items, int mirror_T) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sh_prefix, sh_need;
    __shared__ int scan[kSelThreads];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const float* row = S + static_cast<size_t>(b) * T;
    uint32_t prefix = 0, mask = 0, need = static_cast<uint32_t>(n_keep);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0;
        __syncthreads();
        for (int t = tid; t < T; t += kSelThreads) {
            const uint32_t k = fkey(row[t]);
            if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 0xffu], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            int d = 255;
            for (; d > 0; --d) {
                if (acc + hist[d] >= need) break;
                acc += hist[d];
            }
            sh_prefix = prefix | (static_cast<uint32_t>(d) << shift);
            sh_need = need - acc;   // keys equal to the final threshold still needed
        }
        __syncthreads();
        prefix = sh_prefix;
        need = sh_need;
        mask |= 0xffu << shift;
        __syncthreads();
    }
    // prefix is the n_keep-th largest key; take every key above it and the
    // first `need` keys equal to it in index order. Waves own contiguous
    // quarters of the row and compact 64 entries at a time with ballots, so
    // the output stays in ascending order and every pass reads coalesced.
    constexpr int W = kSelThreads / 64;
    const int wave = tid >> 6, lane = tid & 63;
    const unsigned long long lt = (1ull << lane) - 1;
    const int lo = static_cast<int>((static_cast<long long>(T) * wave) / W);
    const int hi = static_cast<int>((static_cast<long long>(T) * (wave + 1)) / W);
    int gt = 0, eq = 0;
    for (int base = lo; base < hi; base += 64) {
        const int t = base + lane;
        const uint32_t k = t < hi ? fkey(row[t]) : 0u;
        gt += __popcll(__ballot(t < hi && k > prefix));
        eq += __popcll(__ballot(t < hi && k == prefix));
    }
    if (lane == 0) { scan[2 * wave] = gt; scan[2 * wave + 1] = eq; }
    __syncthreads();
    int eq_before = 0, taken_before = 0;
    for (int w = 0; w < wave; ++w) {
        const int e = scan[2 * w + 1];
        const int take_eq = max(0, min(e, static_cast<int>(need) - eq_before));
        taken_before += scan[2 * w] + take_eq;
        eq_before += e;
    }
    int32_t* out = items + static_cast<size_t>(b) * n_items;
    int pos = taken_before, eq_seen = eq_before;
    for (int base = lo; base < hi; base += 64) {
        const int t = base + lane;
        const uint32_t k = t < hi ? fkey(row[t]) : 0u;
        const bool is_eq = t < hi && k == prefix;
        const unsigned long long meq = __ballot(is_eq);
        const bool take = (t < hi && k > prefix) ||
                          (is_eq && eq_seen + __popcll(meq & lt) < static_cast<int>(need));
        const unsigned long long mt = __ballot(take);
        if (take) {
            const int at = pos + __popcll(mt & lt);
            out[at] = t;
            if (mirror_T) out[n_keep + at] = t + mirror_T;
        }
        pos += __popcll(mt);
        eq_seen += __popcll(meq);
    }
}

int launch_scores(const tm_library* lib, const float* profiles, int32_t B, int32_t prec,
                  float* S, hipStream_t s) {
    const dim3 grid((lib->T + 127) / 128, (B + 31) / 32);
    switch (prec) {
        case TM_PREC_FP32:
            hipLaunchKernelGGL(prefilter_scores<TM_PREC_FP32>, grid, dim3(256), 0, s, lib->d_prof,
                               lib->d_prof_max, profiles, lib->T, lib->R, B, S);
            break;
        case TM_PREC_BF16:
            hipLaunchKernelGGL(prefilter_scores<TM_PREC_BF16>, grid, dim3(256), 0, s, lib->d_prof,
                               lib->d_prof_max, profiles, lib->T, lib->R, B, S);
            break;
        case TM_PREC_FP16:
            hipLaunchKernelGGL(prefilter_scores<TM_PREC_FP16>, grid, dim3(256), 0, s, lib->d_prof,
                               lib->d_prof_max, profiles, lib->T, lib->R, B, S);
            break;
        case TM_PREC_FP8:
            hipLaunchKernelGGL(prefilter_scores<TM_PREC_FP8>, grid, dim3(256), 0, s, lib->d_prof,
                               lib->d_prof_max, profiles, lib->T, lib->R, B, S);
            break;
        default:
            tmlib::set_error("unknown precision %d", prec);
            return TM_EINVAL;
    }
    TM_HIP(hipGetLastError());
    return TM_OK;
}

}  // namespace

int tmlib::prefilter_kept(const tm_library* lib, const float* profiles, int32_t B, int32_t n_keep,
                          int32_t precision, int32_t* items, int32_t n_items, bool mirror,
                          hipStream_t s, float* S_given) {
    float* S = S_given;
    if (!S)
        TM_HIP(hipMallocAsync(reinterpret_cast<void**>(&S),
                              static_cast<size_t>(B) * lib->T * sizeof(float), s));
    int r = launch_scores(lib, profiles, B, precision, S, s);
    if (!r) {
        hipLaunchKernelGGL(select_kept, dim3(B), dim3(kSelThreads), 0, s, S, lib->T, n_keep,
                           items, n_items, mirror ? lib->T : 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "select_kept launch");
    }
    if (!S_given) {
        hipError_t e = hipFreeAsync(S, s);
        if (!r && e != hipSuccess) r = tmlib::hip_fail(e, "hipFreeAsync");
    }
    return r;
}

int tmlib::select_top(const float* S, int32_t B, int32_t n, int32_t n_keep, int32_t* items,
                      hipStream_t s) {
    hipLaunchKernelGGL(select_kept, dim3(B), dim3(kSelThreads), 0, s, S, n, n_keep, items, n_keep, 0);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

extern "C" int tm_prefilter(const tm_library* lib, const float* profiles, int32_t B,
                            int32_t n_keep, int32_t precision, int32_t* kept, void* hip_stream) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (n_keep < 1 || n_keep > lib->T) { tmlib::set_error("n_keep=%d outside [1, T=%d]", n_keep, lib->T); return TM_EINVAL; }
    if (precision < TM_PREC_FP32 || precision > TM_PREC_FP8) { tmlib::set_error("unknown precision %d", precision); return TM_EINVAL; }
    if (B == 0) return TM_OK;
    if (!profiles || !kept) { tmlib::set_error("profiles and kept must be non-NULL"); return TM_EINVAL; }
    if (int r = tmlib::require_device()) return r;
    return tmlib::prefilter_kept(lib, profiles, B, n_keep, precision, kept, n_keep, false,
                                 static_cast<hipStream_t>(hip_stream));
}
