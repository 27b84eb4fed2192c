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
//   * Templates that share polar pixels are scored together in groups of G:
//     the library stores per group one record per union pixel (LDS offset
//     and one weight per member, zero if the member lacks the pixel), so a
//     pixel shared by several members is read from LDS once and feeds G*K
//     FMAs. Records are streamed with scalar loads.
//   * Per template the wave takes the lane-wise maximum and skips the rest
//     unless some lane beats the wave's current N-th best score (the
//     common case once the running list fills). Only then does it do the
//     cross-lane reduction and the first-maximum search, and insert into a
//     per-wave top-N held in lanes 0..N-1.
//   * When the touched rows exceed the LDS budget, they are processed in
//     bands: each wave keeps M groups' accumulators in registers while the
//     workgroup streams the bands through LDS.
//   * At the end the waves' lists are merged by wave 0 in LDS.
//
// Ranking order is Q descending, ties to the lower template index; within a
// template the smallest maximising shift. Summation order per (pattern,
// template) is the library's spot order, so results do not depend on the
// batch.
#include <algorithm>
#include <climits>
#include <cmath>

#include "tm_device.h"
#include "tm_topn.h"
#include "tm_internal.h"

namespace {

// Waves per workgroup: 8 when several workgroups share a CU, 16 when one
// workgroup holds (nearly) all of a CU's LDS.
constexpr int kWavesShared = 8;
constexpr int kWavesWhole = 16;
constexpr size_t kWholeCuLds = 80 * 1024;

// One union pixel of a group: LDS float offset within the band, then one
// weight per group member.
template <int G>
struct Rec {
    uint32_t off;
    float w[G];
};

// NB records [i, i + NB): every lane adds w * P[col + lane + 64 k] for its
// K shift slots. Slots k < CLS read from the pixel's column, the others
// (narrow rows only) one period back, where the row's wraparound continues.
// The records' scalar loads and all their LDS reads are in flight before
// the first FMA.
template <int K, int G, int CLS, int NB>
__device__ __forceinline__ void accumulate_recs(const Rec<G> (&r)[NB], const float* lds, int lane,
                                                int n_theta, float (&acc)[G][K]) {
    float v[NB][K];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const float* pa = lds + r[u].off + lane;
        const float* pb = pa - n_theta;
#pragma unroll
        for (int k = 0; k < K; ++k) v[u][k] = (k < CLS) ? pa[64 * k] : pb[64 * k];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[g][k] = fmaf(r[u].w[g], v[u][k], acc[g][k]);
}

template <int K, int G, int CLS, int NB>
__device__ __forceinline__ void accumulate_batch(const Rec<G>* __restrict__ rec, int i,
                                                 const float* lds, int lane, int n_theta,
                                                 float (&acc)[G][K]) {
    Rec<G> r[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) r[u] = rec[i + u];
    accumulate_recs<K, G, CLS, NB>(r, lds, lane, n_theta, acc);
}

// Accumulate records [i0, i1) in batches of NB (8 when a wave may hold the
// registers, i.e. when a workgroup fills the CU), then 4, then singly. The
// summation order per accumulator is the record order in every case. With
// one template per group (candidate lists: few templates per pattern, so
// the record loads' latency is not hidden by other work) the next batch's
// records are loaded while the current one is summed.
template <int K, int G, int CLS, int NB>
__device__ __forceinline__ void accumulate(const Rec<G>* __restrict__ rec, int i0, int i1,
                                           const float* lds, int lane, int n_theta,
                                           float (&acc)[G][K]) {
    int i = i0;
    if constexpr (G == 1 && NB == 8) {
        if (i + NB <= i1) {
            // Vector loads (every lane the same address; an opaque zero
            // index keeps the compiler from turning them into scalar loads,
            // whose results cannot be waited for apart from the LDS reads'):
            // the loads of the next batch stay in flight while this one is
            // summed.
            int z;
            asm volatile("v_mov_b32 %0, 0" : "=v"(z));
            const Rec<G>* vrec = rec + z;
            Rec<G> ra[NB], rb[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) ra[u] = vrec[i + u];
            for (; i + 3 * NB <= i1; i += 2 * NB) {
#pragma unroll
                for (int u = 0; u < NB; ++u) rb[u] = vrec[i + NB + u];
                accumulate_recs<K, G, CLS, NB>(ra, lds, lane, n_theta, acc);
#pragma unroll
                for (int u = 0; u < NB; ++u) ra[u] = vrec[i + 2 * NB + u];
                accumulate_recs<K, G, CLS, NB>(rb, lds, lane, n_theta, acc);
            }
            // ra holds the batch at i; one or two whole batches remain
            if (i + 2 * NB <= i1) {
#pragma unroll
                for (int u = 0; u < NB; ++u) rb[u] = vrec[i + NB + u];
                accumulate_recs<K, G, CLS, NB>(ra, lds, lane, n_theta, acc);
                accumulate_recs<K, G, CLS, NB>(rb, lds, lane, n_theta, acc);
                i += 2 * NB;
            } else {
                accumulate_recs<K, G, CLS, NB>(ra, lds, lane, n_theta, acc);
                i += NB;
            }
        }
    } else {
        for (; i + NB <= i1; i += NB) accumulate_batch<K, G, CLS, NB>(rec, i, lds, lane, n_theta, acc);
    }
    if constexpr (NB > 4) {
        if (i + 4 <= i1) {
            accumulate_batch<K, G, CLS, 4>(rec, i, lds, lane, n_theta, acc);
            i += 4;
        }
    }
    for (; i < i1; ++i) accumulate_batch<K, G, CLS, 1>(rec, i, lds, lane, n_theta, acc);
}

// Records per batch: 8 when a workgroup fills the CU (at most 4 waves per
// SIMD, so up to 128 VGPRs cost no occupancy) and the accumulators and
// values fit, else 4.
template <int K, int G, int M, int NW>
constexpr int batch_size() { return (NW >= 16 && M * G * K + 8 * K <= 96) ? 8 : 4; }

// Records of one (group, band): one segment on wide rows, K class segments
// (CLS = 1..K) on narrow rows.
template <int K, int G, bool NARROW, int NB, int CLS = 1>
__device__ __forceinline__ void accumulate_segments(const Rec<G>* __restrict__ rec,
                                                    const int* __restrict__ sg, const float* lds,
                                                    int lane, int n_theta, float (&acc)[G][K]) {
    if constexpr (!NARROW) {
        accumulate<K, G, K, NB>(rec, sg[0], sg[1], lds, lane, n_theta, acc);
    } else {
        accumulate<K, G, CLS, NB>(rec, sg[CLS - 1], sg[CLS], lds, lane, n_theta, acc);
        if constexpr (CLS < K)
            accumulate_segments<K, G, true, NB, CLS + 1>(rec, sg, lds, lane, n_theta, acc);
    }
}

// Full reduction of one template whose lane maximum may enter the list: the
// wave maximum, its first (smallest) shift, and the insertion.
template <int K>
__device__ __forceinline__ void finalize_slow(const float (&acc)[K], float mx, int t, int lane,
                                              float invP, int N, tmlib::TopState& st,
                                              bool write_all, float* __restrict__ best_q,
                                              short* __restrict__ best_s, size_t best_off) {
    const float wm = tmlib::wave_max(mx);
    int s = 0;
    bool found = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const unsigned long long msk = tmlib::ballot(acc[k] == wm);
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
    if (tmlib::topn_beats(st, Q, t)) tmlib::topn_insert(st, Q, t, s, lane, N);
}

template <int K>
__device__ __forceinline__ float lane_max(const float (&acc)[K]) {
    float m = acc[0];
#pragma unroll
    for (int k = 1; k < K; ++k) m = fmaxf(m, acc[k]);
    return m;
}

template <int K, int G, int M, bool NARROW, int NW>
__global__ void __launch_bounds__(NW * 64)
match_kernel(const float* __restrict__ polar, const double* __restrict__ norms, int R,
             int n_theta, const int* __restrict__ rows, const int* __restrict__ band_off,
             int n_bands, int row_width, const uint32_t* __restrict__ recs,
             const int* __restrict__ seg, const int* __restrict__ members, int n_groups, int Tp,
             int N, int* __restrict__ top_t, int* __restrict__ top_s, float* __restrict__ top_q,
             float* __restrict__ best_q, short* __restrict__ best_s,
             const int* __restrict__ cand, const int* __restrict__ cand_cnt,
             const int* __restrict__ pat_mask, tmlib::SplitWork split) {
    extern __shared__ float lds[];
    __shared__ int claimed;
    constexpr int NCLS = NARROW ? K : 1;
    const int lane = threadIdx.x & 63;
    const int wave = tmlib::uniform(threadIdx.x >> 6);
    const Rec<G>* rec = reinterpret_cast<const Rec<G>*>(recs);
    const bool write_all = best_q != nullptr;
    // the last slot of lanes past n_theta holds no shift: start it at -inf
    const float lastinit = (64 * (K - 1) + lane < n_theta) ? 0.0f : -INFINITY;

    // Items [lo, hi) of pattern b (groups, or in candidate mode (G = 1 only)
    // entries of the pattern's candidate row: item i is template cand[b, i],
    // whose records are the per-template segments; ids outside [0, Tp) are
    // skipped), their top-N written to out_*[0, N).
    auto run = [&](int b, int lo, int hi, int* __restrict__ out_t, int* __restrict__ out_s,
                   float* __restrict__ out_q) {
        const int* items = cand ? cand + static_cast<size_t>(b) * n_groups : nullptr;
        const float* src = polar + static_cast<size_t>(b) * R * n_theta;
        // rows of the band into LDS, each followed by its wraparound; loads
        // are issued 16 at a time per lane (two rows x 8 columns) before
        // their stores, so their latencies overlap
        auto stage = [&](int band) {
            const int r0 = band_off[band], r1 = band_off[band + 1];
            for (int ra = r0 + wave; ra < r1; ra += 2 * NW) {
                const int rb = ra + NW;
                const float* rowa = src + static_cast<size_t>(rows ? rows[ra] : ra) * n_theta;
                const float* rowb =
                    rb < r1 ? src + static_cast<size_t>(rows ? rows[rb] : rb) * n_theta : rowa;
                for (int c0 = 0; c0 < row_width; c0 += 8 * 64) {
                    float va[8], vb[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int c = c0 + lane + 64 * u;
                        const int cc = (c < row_width ? c : 0) % n_theta;
                        va[u] = rowa[cc];
                        vb[u] = rowb[cc];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int c = c0 + lane + 64 * u;
                        if (c < row_width) {
                            lds[(ra - r0) * row_width + c] = va[u];
                            if (rb < r1) lds[(rb - r0) * row_width + c] = vb[u];
                        }
                    }
                }
            }
        };

        const double pn = norms[b];
        // a polar image holding a non-finite value has a non-finite norm: its
        // rows are reported as template -1, angle -1, score NaN (and NaN / -1
        // per template). Tested on the bits, which the device build's
        // no-NaN assumption cannot fold away.
        if ((__double_as_longlong(pn) & 0x7ff0000000000000LL) == 0x7ff0000000000000LL) {
            if (best_q)
                for (int t = threadIdx.x; t < Tp; t += NW * 64) {
                    best_q[static_cast<size_t>(b) * Tp + t] = __int_as_float(0x7fc00000);
                    best_s[static_cast<size_t>(b) * Tp + t] = -1;
                }
            for (int i = threadIdx.x; i < N; i += NW * 64) {
                out_t[i] = -1;
                out_s[i] = -1;
                out_q[i] = __int_as_float(0x7fc00000);
            }
            return;
        }
        const float invP = pn > 0.0 ? static_cast<float>(1.0 / pn) : 0.0f;
        const size_t best_off = static_cast<size_t>(b) * Tp;
        tmlib::TopState st = tmlib::topn_init();

        if (n_bands == 1) {
            stage(0);
            __syncthreads();
        }
        for (int c0 = lo; c0 < hi; c0 += NW * M) {
            const int gb = c0 + wave * M;
            int mem[M][G];
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    int t = -1;
                    if (gb + m < hi) {
                        if (G == 1 && items) {
                            t = items[gb + m];
                            t = (t >= 0 && t < Tp) ? t : -1;
                        } else {
                            t = members[static_cast<size_t>(gb + m) * G + g];
                        }
                    }
                    mem[m][g] = t;
                }
            float acc[M][G][K];
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int g = 0; g < G; ++g) {
#pragma unroll
                    for (int k = 0; k < K - 1; ++k) acc[m][g][k] = 0.0f;
                    acc[m][g][K - 1] = lastinit;
                }
            for (int band = 0; band < n_bands; ++band) {
                if (n_bands > 1) {
                    __syncthreads();
                    stage(band);
                    __syncthreads();
                }
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int grp = (G == 1 && items) ? mem[m][0] : (gb + m < hi ? gb + m : -1);
                    if (grp >= 0) {
                        const int* sg = seg + (static_cast<size_t>(grp) * n_bands + band) * NCLS;
                        accumulate_segments<K, G, NARROW, batch_size<K, G, M, NW>()>(
                            rec, sg, lds, lane, n_theta, acc[m]);
                    }
                }
            }
            // a template needs the full reduction only if some lane's maximum
            // can enter the wave's list. One test per group against the
            // largest lane maximum of its members (absent members hold zeros,
            // which cannot exceed a real member's maximum unless every score
            // is <= 0) is a superset of the exact test; ties and members that
            // fail are sorted out below.
            float mx[M][G];
            float gmx = -INFINITY;
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    mx[m][g] = lane_max<K>(acc[m][g]);
                    gmx = fmaxf(gmx, mx[m][g]);
                }
            if (!tmlib::ballot(gmx * invP >= st.thr) && !write_all) continue;
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int t = mem[m][g];
                    if (t < 0) continue;
                    const float q = mx[m][g] * invP;
                    if (!write_all && !tmlib::ballot(tmlib::topn_beats(st, q, t))) continue;
                    finalize_slow<K>(acc[m][g], mx[m][g], t, lane, invP, N, st, write_all,
                                     best_q, best_s, best_off);
                }
        }

        __syncthreads();
        tmlib::topn_merge_write<NW>(st, lds, wave, lane, N, out_t, out_s, out_q);
    };

    if (!split.tasks) {
        const int b = blockIdx.x;
        // patterns masked out are left untouched (the whole workgroup returns);
        // cand_cnt[b] (optional) limits a candidate row to its first entries
        if (pat_mask && pat_mask[b] == 0) return;
        const int hi = (cand && cand_cnt) ? min(n_groups, max(0, cand_cnt[b])) : n_groups;
        run(b, 0, hi, top_t + static_cast<size_t>(b) * N, top_s + static_cast<size_t>(b) * N,
            top_q + static_cast<size_t>(b) * N);
        return;
    }
    // split launch: claim tasks in order until none is left (every workgroup
    // ends once the counter passes the task count)
    const int n_tasks = split.meta[0];
    for (;;) {
        __syncthreads();                       // the previous task's LDS use is over
        if (threadIdx.x == 0) claimed = atomicAdd(&split.meta[2], 1);
        __syncthreads();
        const int task = claimed;
        if (task >= n_tasks) return;
        const int4 w = split.tasks[task];
        const size_t o = static_cast<size_t>(w.w >= 0 ? w.w : w.x) * N;
        int* ot = (w.w >= 0 ? split.part_t : top_t) + o;
        int* os = (w.w >= 0 ? split.part_s : top_s) + o;
        float* oq = (w.w >= 0 ? split.part_q : top_q) + o;
        run(w.x, w.y, w.z, ot, os, oq);
    }
}

using MatchFn = void (*)(const float*, const double*, int, int, const int*, const int*, int, int,
                         const uint32_t*, const int*, const int*, int, int, int, int*, int*,
                         float*, float*, short*, const int*, const int*, const int*,
                         tmlib::SplitWork);

// Groups held per wave while rows stream through LDS in bands.
template <int K, int G>
constexpr int multi_groups() { return G == 3 ? (K <= 6 ? 2 : 1) : (K <= 6 ? 8 : 4); }

template <int K, int NW>
MatchFn pick(int G, bool multi, bool narrow) {
    if constexpr (K <= tmlib::kMaxNarrowSlots) {
        if (narrow) {
            if (G == 3) return multi ? match_kernel<K, 3, multi_groups<K, 3>(), true, NW>
                                     : match_kernel<K, 3, 1, true, NW>;
            return multi ? match_kernel<K, 1, multi_groups<K, 1>(), true, NW>
                         : match_kernel<K, 1, 1, true, NW>;
        }
        if (multi) return nullptr;   // multi-band libraries with K <= 6 use narrow rows
    } else {
        if (narrow) return nullptr;
        if (multi) return G == 3 ? match_kernel<K, 3, multi_groups<K, 3>(), false, NW>
                                 : match_kernel<K, 1, multi_groups<K, 1>(), false, NW>;
    }
    return G == 3 ? match_kernel<K, 3, 1, false, NW> : match_kernel<K, 1, 1, false, NW>;
}

template <int K>
MatchFn pick_nw(int G, bool multi, bool narrow, int nw) {
    return nw == kWavesWhole ? pick<K, kWavesWhole>(G, multi, narrow)
                             : pick<K, kWavesShared>(G, multi, narrow);
}

MatchFn select_kernel(int K, int G, bool multi, bool narrow, int nw) {
    switch (K) {
        case 1: return pick_nw<1>(G, multi, narrow, nw);
        case 2: return pick_nw<2>(G, multi, narrow, nw);
        case 3: return pick_nw<3>(G, multi, narrow, nw);
        case 4: return pick_nw<4>(G, multi, narrow, nw);
        case 5: return pick_nw<5>(G, multi, narrow, nw);
        case 6: return pick_nw<6>(G, multi, narrow, nw);
        case 7: return pick_nw<7>(G, multi, narrow, nw);
        case 8: return pick_nw<8>(G, multi, narrow, nw);
        case 9: return pick_nw<9>(G, multi, narrow, nw);
        case 10: return pick_nw<10>(G, multi, narrow, nw);
        case 11: return pick_nw<11>(G, multi, narrow, nw);
        case 12: return pick_nw<12>(G, multi, narrow, nw);
        default: return nullptr;
    }
}

}  // namespace

// Launch the match kernel for all templates (cand == nullptr) or for
// per-pattern candidate lists of n_items template ids (per-template records).
int tmlib::launch_match(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                        int32_t N, int32_t* top_template, int32_t* top_angle, float* top_score,
                        float* best_score, int16_t* best_angle, const int32_t* cand,
                        int32_t n_items, const int32_t* cand_count, const int32_t* pat_mask,
                        bool compact, hipStream_t s, const tmlib::SplitWork* split) {
    const int K = tmlib::slots_for(lib->n_theta);
    const bool multi = lib->n_bands > 1;
    const int G = cand ? 1 : lib->group;
    const size_t pattern_bytes = static_cast<size_t>(std::max(lib->band_rows, 1)) * lib->row_width * sizeof(float);
    const int nw = (!multi && pattern_bytes > kWholeCuLds) ? kWavesWhole : kWavesShared;
    MatchFn fn = select_kernel(K, G, multi, lib->narrow, nw);
    if (!fn) { tmlib::set_error("n_theta=%d not supported", lib->n_theta); return TM_EUNSUPPORTED; }
    const size_t merge_bytes = tmlib::topn_merge_bytes(nw, N);
    const size_t lds_bytes = std::max(pattern_bytes, merge_bytes);
    TM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(lds_bytes)));
    const uint32_t* recs = cand ? lib->recs_single() : lib->d_recs;
    const int32_t* seg = cand ? lib->seg_single() : lib->d_seg;
    const int32_t n_groups = cand ? n_items : lib->n_groups;
    const tmlib::SplitWork work = split ? *split : tmlib::SplitWork{};
    hipLaunchKernelGGL(fn, dim3(split ? split->grid : B), dim3(nw * 64), lds_bytes, s, polar, norms,
                       compact ? lib->n_rows : lib->R, lib->n_theta,
                       compact ? nullptr : lib->d_rows, lib->d_band_off, lib->n_bands, lib->row_width,
                       recs, seg, lib->d_members, n_groups, lib->Tp, N, top_template, top_angle,
                       top_score, best_score, reinterpret_cast<short*>(best_angle), cand,
                       cand_count, pat_mask, work);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

// tm_match_batch and its variant without allocations: scratch == nullptr
// takes the pre-filter's scratch (kept lists and the score matrix) from the
// stream-ordered allocator; otherwise it comes from [scratch, scratch +
// scratch_bytes) and requests that need more, or the Fourier route, are
// rejected before anything is enqueued.
int tmlib::match_batch_impl(const tm_library* lib, const float* polar, const double* norms,
                            const float* profiles, int32_t B, const tm_match_opts* opts,
                            int32_t N, int32_t* top_template, int32_t* top_angle,
                            float* top_score, float* best_score, int16_t* best_angle,
                            void* hip_stream, void* scratch, size_t scratch_bytes) {
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
    double keep = 0.0, rescore_keep = 0.0;
    int32_t prec = TM_PREC_FP32, coarse = TM_COARSE_NONE, policy = TM_RESCORE_CERTIFIED;
    int32_t* n_rescored = nullptr;
    bool compact = false;
    if (opts) {
        if (opts->compact_rows != 0 && opts->compact_rows != 1) { tmlib::set_error("compact_rows=%d must be 0 or 1", opts->compact_rows); return TM_EINVAL; }
        compact = opts->compact_rows == 1;
        if (!(opts->prefilter_keep >= 0.0 && opts->prefilter_keep <= 1.0)) {
            tmlib::set_error("prefilter_keep=%g outside [0, 1]", opts->prefilter_keep);
            return TM_EINVAL;
        }
        keep = opts->prefilter_keep;
        prec = opts->prefilter_prec;
        if (prec < TM_PREC_FP32 || prec > TM_PREC_FP8) { tmlib::set_error("unknown precision %d", prec); return TM_EINVAL; }
        coarse = opts->coarse;
        policy = opts->rescore_policy;
        rescore_keep = opts->rescore_keep;
        n_rescored = opts->n_rescored;
        if (coarse != TM_COARSE_NONE && coarse != TM_COARSE_FFT && coarse != TM_COARSE_BOUND) { tmlib::set_error("unknown coarse scorer %d", coarse); return TM_EINVAL; }
        if (policy != TM_RESCORE_CERTIFIED && policy != TM_RESCORE_KEEP) { tmlib::set_error("unknown rescore policy %d", policy); return TM_EINVAL; }
        if (!(rescore_keep >= 0.0 && rescore_keep <= 1.0)) { tmlib::set_error("rescore_keep=%g outside [0, 1]", rescore_keep); return TM_EINVAL; }
        if (coarse == TM_COARSE_FFT) {
            if (keep > 0.0) { tmlib::set_error("the pre-filter and the coarse scorer are exclusive"); return TM_EINVAL; }
            if (!lib->fft) { tmlib::set_error("TM_COARSE_FFT needs a library loaded with TM_LIB_FFT"); return TM_EINVAL; }
            if (policy == TM_RESCORE_KEEP && !(rescore_keep > 0.0)) { tmlib::set_error("TM_RESCORE_KEEP needs rescore_keep > 0"); return TM_EINVAL; }
            if (best_score) { tmlib::set_error("per-template outputs are not available with a coarse scorer"); return TM_EINVAL; }
        }
        if (coarse == TM_COARSE_BOUND) {
            if (keep > 0.0) { tmlib::set_error("the pre-filter and the coarse scorer are exclusive"); return TM_EINVAL; }
            if (policy != TM_RESCORE_CERTIFIED) { tmlib::set_error("window bounds support the certified rescoring only"); return TM_EINVAL; }
            if (best_score) { tmlib::set_error("per-template outputs are not available with a coarse scorer"); return TM_EINVAL; }
            if (!lib->bound) { tmlib::set_error("window bounds are not available for this library (negative template weights, or a window image over 64k columns x rows)"); return TM_EUNSUPPORTED; }
        }
    }
    const bool mirror = lib->Tp == 2 * lib->T;
    int32_t n_keep = 0;
    if (keep > 0.0) {
        n_keep = static_cast<int32_t>(std::ceil(keep * lib->T - 1e-9));
        n_keep = std::max(1, std::min(n_keep, lib->T));
        const int32_t n_items = mirror ? 2 * n_keep : n_keep;
        if (N > n_items) { tmlib::set_error("N=%d exceeds the %d kept templates", N, n_items); return TM_EINVAL; }
        if (best_score) { tmlib::set_error("per-template outputs are not available with a pre-filter"); return TM_EINVAL; }
        if (!profiles && B > 0) { tmlib::set_error("profiles are required with a pre-filter"); return TM_EINVAL; }
    }
    if (scratch && coarse == TM_COARSE_FFT) {
        tmlib::set_error("the Fourier route needs the spectra of a chunk of patterns as scratch "
                         "(about 2 GiB), more than the static buffer of %zu bytes", scratch_bytes);
        return TM_EUNSUPPORTED;
    }
    if (scratch && coarse == TM_COARSE_BOUND) {
        tmlib::set_error("the window-bound search needs per-template bounds [B, T'] and candidate "
                         "lists as stream-ordered scratch; not available with the static buffer "
                         "of %zu bytes", scratch_bytes);
        return TM_EUNSUPPORTED;
    }
    // scratch layout of the pre-filter: kept lists [B, n_items] int32, then
    // (256-byte aligned) the score matrix [B, T] float32
    const size_t items_bytes = (static_cast<size_t>(B) * (mirror ? 2 * n_keep : n_keep) *
                                sizeof(int32_t) + 255) / 256 * 256;
    const size_t scores_bytes = static_cast<size_t>(B) * lib->T * sizeof(float);
    if (scratch && n_keep > 0 && items_bytes + scores_bytes > scratch_bytes) {
        tmlib::set_error("B=%d with %d kept of T=%d templates needs %zu bytes of scratch, more "
                         "than the static buffer of %zu bytes", B, n_keep, lib->T,
                         items_bytes + scores_bytes, scratch_bytes);
        return TM_EINVAL;
    }
    if (B == 0) return TM_OK;
    if (!polar || !norms || !top_template || !top_angle || !top_score) {
        tmlib::set_error("polar, norms and top_* outputs must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (coarse == TM_COARSE_FFT)
        return tmlib::fft_match(lib, polar, norms, B, N, policy, rescore_keep, n_rescored,
                                top_template, top_angle, top_score, compact, s);
    if (coarse == TM_COARSE_BOUND)
        return tmlib::bound_match(lib, polar, norms, B, N, rescore_keep, n_rescored, top_template,
                                  top_angle, top_score, compact, s);
    if (n_keep == 0) {
        int r = tmlib::launch_match(lib, polar, norms, B, N, top_template, top_angle, top_score,
                                    best_score, best_angle, nullptr, 0, nullptr, nullptr, compact,
                                    s);
        if (!r && n_rescored) r = tmlib::fill_i32(n_rescored, B, lib->Tp, s);
        return r;
    }
    // pre-filter, then rescore the kept templates (and their mirrors) exactly
    const int32_t n_items = mirror ? 2 * n_keep : n_keep;
    int32_t* items = nullptr;
    float* S = nullptr;
    if (scratch) {
        items = static_cast<int32_t*>(scratch);
        S = reinterpret_cast<float*>(static_cast<char*>(scratch) + items_bytes);
    } else {
        TM_HIP(hipMallocAsync(reinterpret_cast<void**>(&items),
                              static_cast<size_t>(B) * n_items * sizeof(int32_t), s));
    }
    int r = tmlib::prefilter_kept(lib, profiles, B, n_keep, prec, items, n_items, mirror, s, S);
    if (!r) r = tmlib::launch_match(lib, polar, norms, B, N, top_template, top_angle, top_score,
                                    nullptr, nullptr, items, n_items, nullptr, nullptr, compact,
                                    s);
    if (!r && n_rescored) r = tmlib::fill_i32(n_rescored, B, n_items, s);
    if (!scratch) {
        hipError_t e = hipFreeAsync(items, s);
        if (!r && e != hipSuccess) r = tmlib::hip_fail(e, "hipFreeAsync");
    }
    return r;
}

extern "C" int tm_match_batch(const tm_library* lib, const float* polar, const double* norms,
                              const float* profiles, int32_t B, const tm_match_opts* opts,
                              int32_t N, int32_t* top_template, int32_t* top_angle,
                              float* top_score, float* best_score, int16_t* best_angle,
                              void* hip_stream) {
    return tmlib::match_batch_impl(lib, polar, norms, profiles, B, opts, N, top_template,
                                   top_angle, top_score, best_score, best_angle, hip_stream,
                                   nullptr, 0);
}

extern "C" int tm_match_candidates(const tm_library* lib, const float* polar, const double* norms,
                                   int32_t B, const int32_t* candidates, int32_t n_cand, int32_t N,
                                   int32_t* top_template, int32_t* top_angle, float* top_score,
                                   void* hip_stream) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (B < 0 || n_cand < 1) { tmlib::set_error("B=%d, n_cand=%d: need B >= 0, n_cand >= 1", B, n_cand); return TM_EINVAL; }
    if (N < 1 || N > tmlib::kMaxN || N > n_cand) {
        tmlib::set_error("N=%d outside [1, min(%d, n_cand=%d)]", N, tmlib::kMaxN, n_cand);
        return TM_EINVAL;
    }
    if (B == 0) return TM_OK;
    if (!polar || !norms || !candidates || !top_template || !top_angle || !top_score) {
        tmlib::set_error("polar, norms, candidates and top_* outputs must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    return tmlib::launch_match(lib, polar, norms, B, N, top_template, top_angle, top_score, nullptr,
                               nullptr, candidates, n_cand, nullptr, nullptr, false,
                               static_cast<hipStream_t>(hip_stream));
}

// ----------------------------------------------------- sub-bin in-plane angle

namespace {

// One wave per (pattern, rank): the exact float32 scores of the reported
// template at shifts s-1, s, s+1 (lanes stride its per-template records, a
// fixed butterfly reduces them), then the vertex of the parabola through the
// three when it is a maximum (Section 5, discussion: improving the
// optimisation of the in-plane angle).
__global__ void __launch_bounds__(256)
refine_kernel(const float* __restrict__ polar, const double* __restrict__ norms, int Rs,
              int n_theta, const int* __restrict__ rows, const int* __restrict__ band_off,
              int n_bands, int n_cls, int row_width, const uint32_t* __restrict__ recs,
              const int* __restrict__ seg, int Tp, int n_items, int N,
              const int* __restrict__ top_t, const int* __restrict__ top_s,
              float* __restrict__ out_deg) {
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (item >= n_items) return;                      // uniform per wave
    const int b = item / N;
    const int t = top_t[item];
    int s = top_s[item] % n_theta;
    if (s < 0) s += n_theta;
    const float step = 360.0f / static_cast<float>(n_theta);
    if (t < 0 || t >= Tp) {
        if (lane == 0) out_deg[item] = static_cast<float>(s) * step;
        return;
    }
    const float* src = polar + static_cast<size_t>(b) * Rs * n_theta;
    const double pn = norms[b];
    const float invP = pn > 0.0 ? static_cast<float>(1.0 / pn) : 0.0f;
    const int sm = s == 0 ? n_theta - 1 : s - 1;
    const int sp = s + 1 == n_theta ? 0 : s + 1;
    float am = 0.0f, a0 = 0.0f, ap = 0.0f;
    for (int band = 0; band < n_bands; ++band) {
        const int lo = seg[(static_cast<size_t>(t) * n_bands + band) * n_cls];
        const int hi = seg[(static_cast<size_t>(t) * n_bands + band + 1) * n_cls];
        for (int r = lo + lane; r < hi; r += 64) {
            const uint32_t off = recs[2 * static_cast<size_t>(r)];
            const float w = __uint_as_float(recs[2 * static_cast<size_t>(r) + 1]);
            const int lr = static_cast<int>(off / static_cast<uint32_t>(row_width));
            const int k = static_cast<int>(off) - lr * row_width;
            const int row = band_off[band] + lr;
            const float* p = src + static_cast<size_t>(rows ? rows[row] : row) * n_theta;
            int km = k + sm, k0 = k + s, kp = k + sp;
            if (km >= n_theta) km -= n_theta;
            if (k0 >= n_theta) k0 -= n_theta;
            if (kp >= n_theta) kp -= n_theta;
            am += w * p[km];
            a0 += w * p[k0];
            ap += w * p[kp];
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        am += __shfl_xor(am, m, 64);
        a0 += __shfl_xor(a0, m, 64);
        ap += __shfl_xor(ap, m, 64);
    }
    if (lane == 0) {
        const float qm = am * invP, q0 = a0 * invP, qp = ap * invP;
        const float den = qm - 2.0f * q0 + qp;
        float d = 0.0f;
        if (den < 0.0f) d = fminf(0.5f, fmaxf(-0.5f, 0.5f * (qm - qp) / den));
        float deg = (static_cast<float>(s) + d) * step;
        if (deg < 0.0f) deg += 360.0f;
        if (deg >= 360.0f) deg -= 360.0f;
        out_deg[item] = deg;
    }
}

}  // namespace

extern "C" int tm_refine_angles(const tm_library* lib, const float* polar, const double* norms,
                                int32_t B, int32_t compact_rows, int32_t N,
                                const int32_t* top_template, const int32_t* top_angle,
                                float* refined_deg, void* hip_stream) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (B < 0 || N < 1) { tmlib::set_error("B=%d, N=%d: need B >= 0, N >= 1", B, N); return TM_EINVAL; }
    if (compact_rows != 0 && compact_rows != 1) { tmlib::set_error("compact_rows=%d must be 0 or 1", compact_rows); return TM_EINVAL; }
    if (B == 0) return TM_OK;
    if (!polar || !norms || !top_template || !top_angle || !refined_deg) {
        tmlib::set_error("polar, norms, top_template, top_angle and refined_deg must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    const long long items = static_cast<long long>(B) * N;
    if (items > (1LL << 31) - 1) { tmlib::set_error("B*N too large"); return TM_EINVAL; }
    const bool compact = compact_rows == 1;
    hipLaunchKernelGGL(refine_kernel, dim3(static_cast<unsigned>((items + 3) / 4)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), polar, norms,
                       compact ? lib->n_rows : lib->R, lib->n_theta,
                       compact ? nullptr : lib->d_rows, lib->d_band_off, lib->n_bands, lib->n_cls,
                       lib->row_width, lib->recs_single(), lib->seg_single(), lib->Tp,
                       static_cast<int>(items), N, top_template, top_angle, refined_deg);
    TM_HIP(hipGetLastError());
    return TM_OK;
}
