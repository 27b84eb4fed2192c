// tm_match_batch: the correlation index Q of Eq. (1) for every template at
// every in-plane shift (Section 2.2, Fig. 2 e: the template is slid along the
// azimuthal axis with wraparound, with spot coordinates rounded to integer
// polar pixels), its maximum and angle per template, and the N best
// templates per pattern (Section 2.2, end).
//
// Work per (pattern, template) is a sparse gather: C(s) = sum_i w_i P[j_i,
// (k_i + s) mod n_theta] for all s. The kernel is bound by LDS reads and
// VALU FMAs, not by HBM: each pattern is read once.
//
//   * One workgroup per pattern, 8 waves. The polar rows that the library
//     touches are staged into LDS, each row followed by a wraparound halo, so
//     column k_i + s needs no modulo.
//   * Lanes are shifts: lane l, slot k holds C(l + 64 k); a spot costs one
//     address add, K = ceil(n_theta / 64) conflict-free ds_read_b32 (64
//     consecutive floats each) and K FMAs with the spot weight from SGPRs.
//   * Template spots (offset, weight) are streamed with scalar loads.
//   * Per template the wave takes the lane-wise maximum and skips the rest
//     unless some lane beats the wave's current N-th best score (the
//     common case once the running list fills). Only then does it do the
//     cross-lane reduction and the first-maximum search, and insert into a
//     per-wave top-N held in lanes 0..N-1.
//   * When the touched rows exceed the LDS budget, they are processed in
//     bands: each wave keeps G templates' accumulators in registers while
//     the workgroup streams the bands through LDS.
//   * At the end the waves' lists are merged by wave 0 in LDS.
//
// Ranking order is Q descending, ties to the lower template index; within a
// template the smallest maximising shift. Summation order per (pattern,
// template) is the library's spot order, so results do not depend on the
// batch.
#include <climits>
#include <cmath>

#include "tm_device.h"
#include "tm_topn.h"
#include "tm_internal.h"

namespace {

constexpr int kMatchThreads = 512;
constexpr int kWaves = kMatchThreads / 64;

template <int K>
__device__ __forceinline__ void finalize(const float (&acc)[K], float lastpen, int t, int lane,
                                         float invP, int N, tmlib::TopState& st, bool write_all,
                                         float* __restrict__ best_q, short* __restrict__ best_s,
                                         size_t best_off) {
    // lane-wise maximum over valid slots (only the last slot can be partial)
    float m = (K == 1) ? acc[0] + lastpen : acc[0];
#pragma unroll
    for (int k = 1; k < K; ++k) m = fmaxf(m, (k == K - 1) ? acc[k] + lastpen : acc[k]);
    const float q = m * invP;
    if (!write_all && !tmlib::ballot(q > st.thr)) return;
    const float wm = tmlib::wave_max(m);
    int s = 0;
    bool found = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float v = (k == K - 1) ? acc[k] + lastpen : acc[k];
        const unsigned long long msk = tmlib::ballot(v == wm);
        if (!found && msk) {
            s = 64 * k + __ffsll(static_cast<long long>(msk)) - 1;
            found = true;
        }
    }
    const float Q = wm * invP;
    if (write_all && lane == 0) {
        best_q[best_off + t] = Q;
        best_s[best_off + t] = static_cast<short>(s);
    }
    if (!(Q > st.thr)) return;
    tmlib::topn_insert(st, Q, t, s, lane, N);
}

template <int K, int G>
__global__ void __launch_bounds__(kMatchThreads)
match_kernel(const float* __restrict__ polar, const double* __restrict__ norms, int R,
             int n_theta, const int* __restrict__ rows, const int* __restrict__ band_off,
             int n_bands, int row_width, const uint2* __restrict__ spots,
             const int* __restrict__ seg, int Tp, int N, int* __restrict__ top_t,
             int* __restrict__ top_s, float* __restrict__ top_q, float* __restrict__ best_q,
             short* __restrict__ best_s) {
    extern __shared__ float lds[];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = tmlib::uniform(threadIdx.x >> 6);
    const float* src = polar + static_cast<size_t>(b) * R * n_theta;

    auto stage = [&](int band) {
        const int r0 = band_off[band], r1 = band_off[band + 1];
        for (int r = r0 + wave; r < r1; r += kWaves) {
            const float* row = src + static_cast<size_t>(rows[r]) * n_theta;
            float* dst = lds + (r - r0) * row_width;
            for (int c = lane; c < row_width; c += 64) {
                int cc = c;
                while (cc >= n_theta) cc -= n_theta;
                dst[c] = row[cc];
            }
        }
    };

    const double pn = norms[b];
    const float invP = pn > 0.0 ? static_cast<float>(1.0 / pn) : 0.0f;
    const float lastpen = (64 * (K - 1) + lane < n_theta) ? 0.0f : -INFINITY;
    const bool write_all = best_q != nullptr;
    const size_t best_off = static_cast<size_t>(b) * Tp;
    tmlib::TopState st{-INFINITY, INT_MAX, 0, 0, -INFINITY};

    if (n_bands == 1) {
        stage(0);
        __syncthreads();
    }
    for (int c0 = 0; c0 < Tp; c0 += kWaves * G) {
        const int tb = c0 + wave * G;
        float acc[G][K];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[g][k] = 0.0f;
        for (int band = 0; band < n_bands; ++band) {
            if (n_bands > 1) {
                __syncthreads();
                stage(band);
                __syncthreads();
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int t = tb + g;
                if (t < Tp) {
                    const int* sg = seg + static_cast<size_t>(t) * (n_bands + 1) + band;
                    const int i0 = sg[0], i1 = sg[1];
                    for (int i = i0; i < i1; ++i) {
                        const uint2 sp = spots[i];
                        const float w = __uint_as_float(sp.y);
                        const float* p = lds + sp.x + lane;
#pragma unroll
                        for (int k = 0; k < K; ++k) acc[g][k] = fmaf(w, p[64 * k], acc[g][k]);
                    }
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int t = tb + g;
            if (t < Tp)
                finalize<K>(acc[g], lastpen, t, lane, invP, N, st, write_all, best_q, best_s,
                            best_off);
        }
    }

    __syncthreads();
    tmlib::topn_merge_write<kWaves>(st, lds, wave, lane, N, top_t + static_cast<size_t>(b) * N,
                                 top_s + static_cast<size_t>(b) * N,
                                 top_q + static_cast<size_t>(b) * N);
}

using MatchFn = void (*)(const float*, const double*, int, int, const int*, const int*, int, int,
                         const uint2*, const int*, int, int, int*, int*, float*, float*, short*);

template <int K>
MatchFn pick(bool multi) {
    if (!multi) return match_kernel<K, 1>;
    return K <= 6 ? match_kernel<K, 8> : match_kernel<K, 4>;
}

MatchFn select_kernel(int K, bool multi) {
    switch (K) {
        case 1: return pick<1>(multi);
        case 2: return pick<2>(multi);
        case 3: return pick<3>(multi);
        case 4: return pick<4>(multi);
        case 5: return pick<5>(multi);
        case 6: return pick<6>(multi);
        case 7: return pick<7>(multi);
        case 8: return pick<8>(multi);
        case 9: return pick<9>(multi);
        case 10: return pick<10>(multi);
        case 11: return pick<11>(multi);
        case 12: return pick<12>(multi);
        default: return nullptr;
    }
}

}  // namespace

extern "C" int tm_match_batch(const tm_library* lib, const float* polar, const double* norms,
                              const float* profiles, int32_t B, const tm_match_opts* opts,
                              int32_t N, int32_t* top_template, int32_t* top_angle,
                              float* top_score, float* best_score, int16_t* best_angle,
                              void* hip_stream) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (N < 1 || N > tmlib::kMaxN || N > lib->Tp) {
        tmlib::set_error("N=%d outside [1, min(%d, T'=%d)]", N, tmlib::kMaxN, lib->Tp);
        return TM_EINVAL;
    }
    if ((best_score == nullptr) != (best_angle == nullptr)) {
        tmlib::set_error("best_score and best_angle must be both NULL or both set");
        return TM_EINVAL;
    }
    if (opts) {
        for (int i = 0; i < 7; ++i)
            if (opts->reserved[i]) { tmlib::set_error("tm_match_opts.reserved must be zero"); return TM_EINVAL; }
        if (!(opts->prefilter_keep >= 0.0 && opts->prefilter_keep <= 1.0)) {
            tmlib::set_error("prefilter_keep=%g outside [0, 1]", opts->prefilter_keep);
            return TM_EINVAL;
        }
        if (opts->prefilter_keep > 0.0) {
            tmlib::set_error("pre-filtered matching is not available in this build");
            return TM_EUNSUPPORTED;
        }
    }
    (void)profiles;
    if (B == 0) return TM_OK;
    if (!polar || !norms || !top_template || !top_angle || !top_score) {
        tmlib::set_error("polar, norms and top_* outputs must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;

    const int K = tmlib::slots_for(lib->n_theta);
    const bool multi = lib->n_bands > 1;
    MatchFn fn = select_kernel(K, multi);
    if (!fn) { tmlib::set_error("n_theta=%d not supported", lib->n_theta); return TM_EUNSUPPORTED; }
    const size_t pattern_bytes = static_cast<size_t>(std::max(lib->band_rows, 1)) * lib->row_width * sizeof(float);
    const size_t merge_bytes = tmlib::topn_merge_bytes(kWaves, N);
    const size_t lds_bytes = std::max(pattern_bytes, merge_bytes);
    TM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(lds_bytes)));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(fn, dim3(B), dim3(kMatchThreads), lds_bytes, s, polar, norms, lib->R,
                       lib->n_theta, lib->d_rows, lib->d_band_off, lib->n_bands, lib->row_width,
                       lib->d_spots, lib->d_seg, lib->Tp, N, top_template, top_angle, top_score,
                       best_score, reinterpret_cast<short*>(best_angle));
    TM_HIP(hipGetLastError());
    return TM_OK;
}
