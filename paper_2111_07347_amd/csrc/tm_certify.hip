// Certified rescoring: the exact float32 top-N from per-template estimates of
// the best score that are either within a known margin of the exact score
// (the Fourier route's coarse scores) or upper bounds of it (the window
// bounds of tm_bound.hip, margin 0). The N templates with the best estimates
// (or more: n_first) are scored exactly; the N-th best of their exact scores,
// q_N, is a lower bound of the final N-th best, so every template of the
// final top-N has an estimate of at least q_N - margin. Those templates are then scored exactly and ranked
// again; a pattern with more candidates than a cap is scored in full.
#include <algorithm>
#include <cmath>

#include "tm_device.h"
#include "tm_internal.h"

namespace {

constexpr int kSelThreads = 256;

// Candidates of the certified rescoring, one workgroup per pattern: every
// t' with Qt[b, t'] >= (N-th best exact score of the rescored approximate
// top-N) - margin, in ascending order. More than cap: the pattern is marked
// for a full exact scan instead. Waves own contiguous quarters of the row and
// compact with ballots (two passes: count, then write).
__global__ void __launch_bounds__(kSelThreads)
certify_select(const float* __restrict__ Qt, int Tp, const float* __restrict__ q_exact, int N,
               double margin, int cap, int32_t* __restrict__ cand, int32_t* __restrict__ cnt,
               int32_t* __restrict__ full, int32_t* __restrict__ n_rescored) {
    constexpr int W = kSelThreads / 64;
    __shared__ int wcount[W];
    const int b = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // threshold rounded toward -inf: a template whose approximate score could
    // reach the N-th best exact score within the bound is never dropped by
    // the rounding of the subtraction
    const double thr_d = static_cast<double>(q_exact[static_cast<size_t>(b) * N + N - 1]) - margin;
    float thr = static_cast<float>(thr_d);
    if (static_cast<double>(thr) > thr_d) thr = nextafterf(thr, -INFINITY);
    const float* row = Qt + static_cast<size_t>(b) * Tp;
    const int lo = static_cast<int>((static_cast<long long>(Tp) * wave) / W);
    const int hi = static_cast<int>((static_cast<long long>(Tp) * (wave + 1)) / W);
    int c = 0;
    for (int base = lo; base < hi; base += 64) {
        const int t = base + lane;
        c += __popcll(tmlib::ballot(t < hi && row[t] >= thr));
    }
    if (lane == 0) wcount[wave] = c;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < W; ++w) {
        before += (w < wave) ? wcount[w] : 0;
        total += wcount[w];
    }
    const bool over = total > cap;
    if (!over) {
        int32_t* out = cand + static_cast<size_t>(b) * cap;
        int pos = before;
        for (int base = lo; base < hi; base += 64) {
            const int t = base + lane;
            const bool take = t < hi && row[t] >= thr;
            const unsigned long long m = tmlib::ballot(take);
            if (take) out[pos + __popcll(m & ((1ull << lane) - 1))] = t;
            pos += __popcll(m);
        }
    }
    if (threadIdx.x == 0) {
        cnt[b] = over ? 0 : total;
        full[b] = over ? 1 : 0;
        if (n_rescored) n_rescored[b] = over ? Tp : total;
    }
}

template <typename T>
int alloc_async(T** p, size_t count, hipStream_t s) {
    *p = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T), s);
    if (e != hipSuccess) {
        *p = nullptr;
        tmlib::set_error("hipMallocAsync(%zu bytes) failed: %s", count * sizeof(T), hipGetErrorString(e));
        return TM_ENOMEM;
    }
    return TM_OK;
}

}  // namespace

int tmlib::certified_rescore(const tm_library* lib, const float* polar, const double* norms,
                             int32_t B, int32_t N, int32_t n_first, const float* Qt, double margin,
                             int32_t cap, int32_t* n_rescored, int32_t* top_template,
                             int32_t* top_angle, float* top_score, bool compact, hipStream_t s) {
    const int Tp = lib->Tp;
    n_first = std::max(N, std::min(n_first, std::min(tmlib::kMaxN, Tp)));
    int r = TM_OK;
    int32_t *t0 = nullptr, *s0 = nullptr, *t1 = nullptr, *s1 = nullptr;
    float *q0 = nullptr, *q1 = nullptr;
    int32_t *cand = nullptr, *cnt = nullptr, *full = nullptr;
    const size_t bn = static_cast<size_t>(B) * N;
    const size_t bf = static_cast<size_t>(B) * n_first;
    if (!r) r = alloc_async(&t0, bf, s);
    if (!r) r = alloc_async(&s0, bf, s);
    if (!r) r = alloc_async(&q0, bf, s);
    if (!r) r = alloc_async(&t1, bn, s);
    if (!r) r = alloc_async(&s1, bn, s);
    if (!r) r = alloc_async(&q1, bn, s);
    if (!r) r = alloc_async(&cand, static_cast<size_t>(B) * cap, s);
    if (!r) r = alloc_async(&cnt, B, s);
    if (!r) r = alloc_async(&full, B, s);
    // 1. the n_first best estimates, scored exactly: their N-th best, q_N
    if (!r) r = tmlib::launch_topn(Qt, nullptr, B, Tp, n_first, t0, s0, q0, s);
    if (!r) r = tmlib::launch_match(lib, polar, norms, B, N, t1, s1, q1, nullptr, nullptr, t0,
                                    n_first, nullptr, nullptr, compact, s);
    // 2. every template whose estimate reaches q_N - margin
    if (!r) {
        hipLaunchKernelGGL(certify_select, dim3(B), dim3(kSelThreads), 0, s, Qt, Tp, q1, N, margin,
                           cap, cand, cnt, full, n_rescored);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "certify_select launch");
    }
    // 3. exact scores of the candidates; full scans where the set was too large
    if (!r) r = tmlib::launch_match(lib, polar, norms, B, N, top_template, top_angle, top_score,
                                    nullptr, nullptr, cand, cap, cnt, nullptr, compact, s);
    if (!r) r = tmlib::launch_match(lib, polar, norms, B, N, top_template, top_angle, top_score,
                                    nullptr, nullptr, nullptr, 0, nullptr, full, compact, s);
    for (void* p : {static_cast<void*>(t0), static_cast<void*>(s0), static_cast<void*>(q0),
                    static_cast<void*>(t1), static_cast<void*>(s1), static_cast<void*>(q1),
                    static_cast<void*>(cand), static_cast<void*>(cnt), static_cast<void*>(full)})
        if (p) (void)hipFreeAsync(p, s);
    return r;
}
