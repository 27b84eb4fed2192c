// Device-side running top-N lists (score descending, ties to the lower
// template index) held in the lanes of a wave, and the merge of several
// waves' lists through LDS.
#pragma once

#include <climits>
#include <cmath>

#include "tm_device.h"

namespace tmlib {

struct TopState {
    float q;     // lanes < cnt: entry score
    int t, s;    // entry template and angle
    int cnt;     // entries held (uniform)
    float thr;   // N-th entry's score (uniform); -inf until the list is full
    int thr_t;   // N-th entry's template (uniform); INT_MAX until full
};

__device__ __forceinline__ TopState topn_init() {
    return TopState{-INFINITY, INT_MAX, 0, 0, -INFINITY, INT_MAX};
}

// True if (Q, t) ranks before the list's N-th entry: higher score, or equal
// score and lower template index.
__device__ __forceinline__ bool topn_beats(const TopState& st, float Q, int t) {
    return Q > st.thr || (Q == st.thr && t < st.thr_t);
}

// Insert (Q, t, s) into a wave's list; callers only insert entries that
// beat the N-th entry, in any template order.
__device__ __forceinline__ void topn_insert(TopState& st, float Q, int t, int s, int lane, int N) {
    const unsigned long long before =
        ballot(lane < st.cnt && (st.q > Q || (st.q == Q && st.t < t)));
    const int pos = __popcll(before);
    const float uq = __shfl_up(st.q, 1, 64);
    const int ut = __shfl_up(st.t, 1, 64);
    const int us = __shfl_up(st.s, 1, 64);
    if (lane > pos) { st.q = uq; st.t = ut; st.s = us; }
    if (lane == pos) { st.q = Q; st.t = t; st.s = s; }
    st.cnt = min(st.cnt + 1, N);
    st.thr = (st.cnt == N) ? __shfl(st.q, N - 1, 64) : -INFINITY;
    st.thr_t = (st.cnt == N) ? __shfl(st.t, N - 1, 64) : INT_MAX;
}

inline size_t topn_merge_bytes(int waves, int N) {
    return static_cast<size_t>(waves) * N * 12 + static_cast<size_t>(waves) * sizeof(int);
}

// Merge the lists of NW waves (all waves call; LDS scratch of
// topn_merge_bytes(NW, N) bytes, free for reuse by the caller) and write the
// N best entries. Wave 0 repeatedly takes the best entry ranked after the
// previous pick. The caller must have synchronised the workgroup before the
// scratch region is reused.
template <int NW>
__device__ __forceinline__ void topn_merge_write(const TopState& st, float* scratch, int wave,
                                                 int lane, int N, int* __restrict__ out_t,
                                                 int* __restrict__ out_s,
                                                 float* __restrict__ out_q) {
    float* mq = scratch;
    int* mt = reinterpret_cast<int*>(mq + NW * N);
    int* ms = mt + NW * N;
    int* mc = ms + NW * N;
    if (lane < N) {
        mq[wave * N + lane] = st.q;
        mt[wave * N + lane] = st.t;
        ms[wave * N + lane] = st.s;
    }
    if (lane == 0) mc[wave] = st.cnt;
    __syncthreads();
    if (wave != 0) return;
    float pq = INFINITY;
    int pt = -1;
    for (int r = 0; r < N; ++r) {
        float bq = -INFINITY;
        int bt = INT_MAX, bs = 0;
        for (int c = lane; c < NW * N; c += 64) {
            const int w = c / N, i = c - w * N;
            if (i < mc[w]) {
                const float q = mq[c];
                const int t = mt[c];
                const bool after = (q < pq) || (q == pq && t > pt);
                const bool better = (q > bq) || (q == bq && t < bt);
                if (after && better) { bq = q; bt = t; bs = ms[c]; }
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            const float oq = __shfl_xor(bq, m, 64);
            const int ot = __shfl_xor(bt, m, 64);
            const int os = __shfl_xor(bs, m, 64);
            if (oq > bq || (oq == bq && ot < bt)) { bq = oq; bt = ot; bs = os; }
        }
        if (lane == 0) {
            out_t[r] = bt;
            out_s[r] = bs;
            out_q[r] = bq;
        }
        pq = bq;
        pt = bt;
    }
}

}  // namespace tmlib
