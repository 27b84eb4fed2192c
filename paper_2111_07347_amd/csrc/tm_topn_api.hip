// tm_topn: sort per-template best scores and keep the N best templates per
// pattern (Section 2.2, end: sorting the per-template correlations gives the N
// best templates rather than only the best one).
//
// One workgroup per pattern, 4 waves; each wave streams a contiguous quarter
// of the templates, 4 blocks of 64 per step (coalesced loads, all four in
// flight together), tests each block against its running N-th best with one
// ballot, and inserts only the candidates that beat it, in increasing
// template order. The waves' lists are merged in LDS.
#include <algorithm>

#include "tm_device.h"
#include "tm_internal.h"
#include "tm_topn.h"

namespace {

constexpr int kTopnThreads = 256;
constexpr int kTopnWaves = kTopnThreads / 64;

__global__ void __launch_bounds__(kTopnThreads)
topn_kernel(const float* __restrict__ best_q, const short* __restrict__ best_s, int T, int N,
            int* __restrict__ top_t, int* __restrict__ top_s, float* __restrict__ top_q) {
    extern __shared__ float lds[];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = tmlib::uniform(threadIdx.x >> 6);
    const int lo = static_cast<int>((static_cast<long long>(T) * wave) / kTopnWaves);
    const int hi = static_cast<int>((static_cast<long long>(T) * (wave + 1)) / kTopnWaves);
    const float* q_row = best_q + static_cast<size_t>(b) * T;
    const short* s_row = best_s ? best_s + static_cast<size_t>(b) * T : nullptr;
    tmlib::TopState st = tmlib::topn_init();
    // 4 blocks of 64 templates per step: their loads are issued together
    constexpr int kBlocks = 4;
    for (int base0 = lo; base0 < hi; base0 += 64 * kBlocks) {
        float qv[kBlocks];
        int sv[kBlocks];
#pragma unroll
        for (int k = 0; k < kBlocks; ++k) {
            const int t = base0 + 64 * k + lane;
            const bool ok = t < hi;
            qv[k] = ok ? q_row[t] : -INFINITY;
            sv[k] = (ok && best_s) ? s_row[t] : 0;
        }
#pragma unroll
        for (int k = 0; k < kBlocks; ++k) {
            const int base = base0 + 64 * k;
            const int t = base + lane;
            const float q = qv[k];
            unsigned long long msk =
                tmlib::ballot(t < hi && (st.cnt < N || tmlib::topn_beats(st, q, t)));
            while (msk) {
                const int l = __ffsll(static_cast<long long>(msk)) - 1;
                msk &= msk - 1;
                const float Q = __shfl(q, l, 64);
                const int S = __shfl(sv[k], l, 64);
                if (st.cnt < N || tmlib::topn_beats(st, Q, base + l)) tmlib::topn_insert(st, Q, base + l, S, lane, N);
            }
        }
    }
    tmlib::topn_merge_write<kTopnWaves>(st, lds, wave, lane, N, top_t + static_cast<size_t>(b) * N,
                                     top_s + static_cast<size_t>(b) * N,
                                     top_q + static_cast<size_t>(b) * N);
}

}  // namespace

int tmlib::launch_topn(const float* best_score, const int16_t* best_angle, int32_t B, int32_t T,
                       int32_t N, int32_t* top_template, int32_t* top_angle, float* top_score,
                       hipStream_t s) {
    const size_t lds = tmlib::topn_merge_bytes(kTopnWaves, N);
    hipLaunchKernelGGL(topn_kernel, dim3(B), dim3(kTopnThreads), lds, s, best_score,
                       reinterpret_cast<const short*>(best_angle), T, N, top_template, top_angle,
                       top_score);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

extern "C" int tm_topn(const float* best_score, const int16_t* best_angle, int32_t B, int32_t T,
                       int32_t N, int32_t* top_template, int32_t* top_angle, float* top_score,
                       void* hip_stream) {
    tmlib::clear_error();
    if (B < 0 || T < 1) { tmlib::set_error("B=%d, T=%d: need B >= 0, T >= 1", B, T); return TM_EINVAL; }
    if (N < 1 || N > tmlib::kMaxN || N > T) {
        tmlib::set_error("N=%d outside [1, min(%d, T=%d)]", N, tmlib::kMaxN, T);
        return TM_EINVAL;
    }
    if (B == 0) return TM_OK;
    if (!best_score || !best_angle || !top_template || !top_angle || !top_score) {
        tmlib::set_error("all pointers must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    return tmlib::launch_topn(best_score, best_angle, B, T, N, top_template, top_angle, top_score,
                              static_cast<hipStream_t>(hip_stream));
}
