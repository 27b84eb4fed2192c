// Certified rescoring: the exact float32 top-N from per-template estimates of
// the best score that are either within a known margin of the exact score
// (the Fourier route's coarse scores) or upper bounds of it (the window
// bounds of tm_bound.hip, margin 0). The N templates with the best estimates
// (or more: n_first) are scored exactly; the N-th best of their exact scores,
// q_N, is a lower bound of the final N-th best, so every template of the
// final top-N has an estimate of at least q_N - margin. Those templates
// (other than the ones already scored) are then scored exactly and their
// top-N merged with the first one; a pattern with more candidates than a
// cap is scored in full.
#include <algorithm>
#include <climits>
#include <cmath>

#include "tm_device.h"
#include "tm_internal.h"

namespace {

constexpr int kSelThreads = 256;

// Candidates of the certified rescoring, one workgroup per pattern: every
// column c with Qt[b, c] >= (N-th best exact score of the rescored
// approximate top-N) - margin, written as its template (map[c], or c)
// (columns without a template are skipped), except the n_first templates
// already scored exactly (first[b, :]); the order does not matter to the
// scorer (its ranking rule decides). More than cap
// such templates in all: the pattern is marked for a full exact scan
// instead. Waves own contiguous quarters of the row and compact with
// ballots: a counting pass over the row that touches no other memory (so
// the next step's loads stay in flight), then, reading again only the
// blocks of 64 loads that held a column at or above the threshold, a pass
// counting the new candidates and one writing them. With a map, columns
// from T' on are taken to hold no template (as the window bounds' slot map
// has it).
template <int V>
__global__ void __launch_bounds__(kSelThreads)
certify_select(const float* __restrict__ Qt, int Tp, int n_valid, const int32_t* __restrict__ map,
               const float* __restrict__ q_exact, int N, double margin, int cap,
               int32_t* __restrict__ cand, int32_t* __restrict__ cnt, int32_t* __restrict__ full,
               int32_t* __restrict__ n_rescored, int n_templates,
               const int32_t* __restrict__ first, int n_first) {
    constexpr int W = kSelThreads / 64;
    __shared__ int wcount[W], wnew[W];
    __shared__ int sfirst[tmlib::kMaxN];
    const int b = blockIdx.x;
    const int wave = tmlib::uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (threadIdx.x < n_first) sfirst[threadIdx.x] = first[static_cast<size_t>(b) * n_first + threadIdx.x];
    // threshold rounded toward -inf: a template whose approximate score could
    // reach the N-th best exact score within the bound is never dropped by
    // the rounding of the subtraction
    const double thr_d = static_cast<double>(q_exact[static_cast<size_t>(b) * N + N - 1]) - margin;
    float thr = static_cast<float>(thr_d);
    if (static_cast<double>(thr) > thr_d) thr = nextafterf(thr, -INFINITY);
    const float* row = Qt + static_cast<size_t>(b) * Tp;
    // waves own contiguous quarters, whole groups of V columns (V = 4: one
    // 16-byte load per lane and block; the row length is a multiple of 4)
    const int ng = Tp / V;
    const int lo = V * static_cast<int>((static_cast<long long>(ng) * wave) / W);
    const int hi = V * static_cast<int>((static_cast<long long>(ng) * (wave + 1)) / W);
    const int lim = min(hi, n_valid);           // columns past n_valid hold no template
    // 4 blocks of 64 V columns per step, their loads issued together;
    // column of (block k, component e) for this lane: base + V (64 k + lane) + e
    constexpr int kBlocks = 4;
    constexpr int kStep = V * 64 * kBlocks;
    auto is_first = [&](int t) {
        const int tt = map ? map[t] : t;
        bool f = false;
        for (int i = 0; i < n_first; ++i) f |= (sfirst[i] == tt);
        return f;
    };
    auto load_block = [&](int t, float (&v)[V]) {
        if constexpr (V == 4) {
            const float4 x = t < hi ? *reinterpret_cast<const float4*>(row + t)
                                    : make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
            v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        } else {
            v[0] = t < hi ? row[t] : -INFINITY;
        }
    };
    // 1. count the columns at or above the threshold (no memory access but
    // the row) and mark the blocks (among a wave's first 64) that hold one.
    // Two value sets alternate, so a step's loads are in flight while the
    // one before is tested; loads past the wave's columns repeat its last
    // group (the test masks them)
    int c = 0;
    unsigned long long hits = 0;
    if (hi > lo) {
        auto ld = [&](int base0, float (&v)[kBlocks][V]) {
#pragma unroll
            for (int k = 0; k < kBlocks; ++k) {
                const int t = min(base0 + V * (64 * k + lane), hi - V);
                if constexpr (V == 4) {
                    const float4 x = *reinterpret_cast<const float4*>(row + t);
                    v[k][0] = x.x; v[k][1] = x.y; v[k][2] = x.z; v[k][3] = x.w;
                } else {
                    v[k][0] = row[t];
                }
            }
        };
        auto test = [&](const float (&v)[kBlocks][V], int base0, int st) {
#pragma unroll
            for (int k = 0; k < kBlocks; ++k) {
                int cs = 0;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int t = base0 + V * (64 * k + lane) + e;
                    cs += __popcll(tmlib::ballot(t < lim && v[k][e] >= thr));
                }
                c += cs;
                const int blk = st * kBlocks + k;
                if (cs && blk < 64) hits |= 1ull << blk;
            }
        };
        float va[kBlocks][V], vb[kBlocks][V];
        ld(lo, va);
        for (int base0 = lo, st = 0; base0 < hi; base0 += 2 * kStep, st += 2) {
            ld(base0 + kStep, vb);
            test(va, base0, st);
            if (base0 + kStep >= hi) break;                  // uniform
            ld(base0 + 2 * kStep, va);
            test(vb, base0 + kStep, st + 1);
        }
    }
    // the blocks of a step to read again: those that held a column at or
    // above the threshold (all from block 64 on)
    auto step_sel = [&](int st) -> unsigned {
        return st * kBlocks + kBlocks <= 64
                   ? static_cast<unsigned>(hits >> (st * kBlocks)) & ((1u << kBlocks) - 1)
                   : (1u << kBlocks) - 1;
    };
    // 2. in those blocks: the candidates (a template, not scored first)
    auto visit = [&](auto&& fn) {
        for (int base0 = lo, st = 0; base0 < hi; base0 += kStep, ++st) {
            const unsigned sel = step_sel(st);
            if (!sel) continue;                                  // uniform
#pragma unroll
            for (int k = 0; k < kBlocks; ++k) {
                if (!((sel >> k) & 1)) continue;                 // uniform
                float v[V];
                load_block(base0 + V * (64 * k + lane), v);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int t = base0 + V * (64 * k + lane) + e;
                    const bool tk = t < lim && v[e] >= thr;
                    if (!tmlib::ballot(tk)) continue;           // uniform
                    fn(t, tk && (!map || map[t] >= 0) && !is_first(t));
                }
            }
        }
    };
    // 3. one more pass over those blocks writes the candidates (at most cap)
    // at places taken from a workgroup counter: their order is not
    // deterministic, which no result depends on (every merge ranks by the
    // scorer's rule)
    if (threadIdx.x == 0) wcount[0] = 0;
    __syncthreads();                             // sfirst and the counter are set
    int32_t* out = cand + static_cast<size_t>(b) * cap;
    visit([&](int t, bool take) {
        const unsigned long long m = tmlib::ballot(take);
        int base = 0;
        if (lane == 0) base = atomicAdd(&wcount[0], __popcll(m));
        base = __shfl(base, 0, 64);
        const int pos = base + __popcll(m & ((1ull << lane) - 1));
        if (take && pos < cap) out[pos] = map ? map[t] : t;
    });
    __syncthreads();
    const int total_new = wcount[0];
    if (lane == 0) wnew[wave] = c;
    __syncthreads();
    int total = 0;
    for (int w = 0; w < W; ++w) total += wnew[w];
    const bool over = total > cap;
    if (threadIdx.x == 0) {
        cnt[b] = over ? 0 : total_new;
        full[b] = over ? 1 : 0;
        if (n_rescored) n_rescored[b] = over ? n_templates : total;
    }
}

// The final top-N of a pattern not scanned in full: its candidates' top-N
// (in the output rows) merged with the top-N of the templates scored first
// (one wave per pattern; the scorer's ranking rule; a non-finite norm is
// flagged as the scorer flags it).
__global__ void __launch_bounds__(256)
merge_first(const int32_t* __restrict__ full, int B, const double* __restrict__ norms, int N,
            const int32_t* __restrict__ ft, const int32_t* __restrict__ fs,
            const float* __restrict__ fq, int32_t* __restrict__ top_t, int32_t* __restrict__ top_s,
            float* __restrict__ top_q) {
    const int lane = threadIdx.x & 63;
    const int b = (blockIdx.x * 256 + threadIdx.x) >> 6;
    if (b >= B || full[b]) return;
    const size_t o = static_cast<size_t>(b) * N;
    const double pn = norms[b];
    if ((__double_as_longlong(pn) & 0x7ff0000000000000LL) == 0x7ff0000000000000LL) {
        for (int i = lane; i < N; i += 64) {
            top_t[o + i] = -1;
            top_s[o + i] = -1;
            top_q[o + i] = __int_as_float(0x7fc00000);
        }
        return;
    }
    // entries: 0..N-1 the candidates' list, N..2N-1 the first list (N <= 64,
    // so at most two per lane)
    float q[2];
    int t[2], sh[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = lane + 64 * k;
        const bool c = e < N, f = e >= N && e < 2 * N;
        q[k] = c ? top_q[o + e] : (f ? fq[o + e - N] : -INFINITY);
        t[k] = c ? top_t[o + e] : (f ? ft[o + e - N] : INT_MAX);
        sh[k] = c ? top_s[o + e] : (f ? fs[o + e - N] : 0);
    }
    float prev_q = INFINITY;
    int prev_t = -1;
    int out_t = 0, out_s = 0;
    float out_q = 0.0f;
    for (int r = 0; r < N; ++r) {
        float bq = -INFINITY;
        int bt = INT_MAX, bs = 0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const bool after = (q[k] < prev_q) || (q[k] == prev_q && t[k] > prev_t);
            const bool better = (q[k] > bq) || (q[k] == bq && t[k] < bt);
            if (after && better) { bq = q[k]; bt = t[k]; bs = sh[k]; }
        }
#pragma unroll
        for (int x = 32; x >= 1; x >>= 1) {
            const float oq = __shfl_xor(bq, x, 64);
            const int ot = __shfl_xor(bt, x, 64);
            const int os = __shfl_xor(bs, x, 64);
            if (oq > bq || (oq == bq && ot < bt)) { bq = oq; bt = ot; bs = os; }
        }
        if (lane == r) { out_t = bt; out_s = bs; out_q = bq; }
        prev_q = bq;
        prev_t = bt;
    }
    if (lane < N) {
        top_t[o + lane] = out_t;
        top_s[o + lane] = out_s;
        top_q[o + lane] = out_q;
    }
}

// Split launches of the exact scorer: a pattern with many items (candidates,
// or every group in a full scan) is cut into tasks of about kChunk* items,
// each scored by its own workgroup into a partial top-N list, and the lists
// are merged; the other patterns keep one task that writes its output rows.
// Split tasks come first, so the longest work starts first.
constexpr int kPlanThreads = 1024;
constexpr int kSlotBudget = 16384;       // partial lists per launch
constexpr int kChunkCand = 512;          // candidate entries per task
constexpr int kChunkFull = 256;          // groups per task in a full scan
constexpr int kSplitGrid = 2048;         // workgroups of a split launch

// Exclusive prefix sums over the workgroup of three per-thread counts; also
// returns the totals. All threads call.
__device__ int3 block_scan3(int3 v, int3& total) {
    __shared__ int3 part[kPlanThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int3 inc = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int x = __shfl_up(inc.x, d, 64), y = __shfl_up(inc.y, d, 64),
                  z = __shfl_up(inc.z, d, 64);
        if (lane >= d) { inc.x += x; inc.y += y; inc.z += z; }
    }
    if (lane == 63) part[wave] = inc;
    __syncthreads();
    int3 before = make_int3(0, 0, 0);
    total = make_int3(0, 0, 0);
    for (int w = 0; w < kPlanThreads / 64; ++w) {
        const int3 p = part[w];
        if (w < wave) { before.x += p.x; before.y += p.y; before.z += p.z; }
        total.x += p.x; total.y += p.y; total.z += p.z;
    }
    __syncthreads();
    return make_int3(before.x + inc.x - v.x, before.y + inc.y - v.y, before.z + inc.z - v.z);
}

// Plan one split launch over the patterns with (full[b] != 0) == want_full:
// pattern b has n_b = cnt[b] items (clamped to [0, n_items]), or n_items
// when cnt is null. Patterns with more than `chunk` items are split into
// min(ceil(n_b / chunk), slots / n_split) tasks of near-equal ranges when
// that is at least 2 (n_split: the patterns over `chunk`); the others get
// one task. Writes tasks, merges (pattern, first slot, tasks) and meta
// (task count, merge count, two zeroed counters). One workgroup.
__global__ void __launch_bounds__(kPlanThreads)
plan_split(const int32_t* __restrict__ full, int want_full, const int32_t* __restrict__ cnt,
           int n_items, int B, int chunk, int slots, int4* __restrict__ tasks,
           int4* __restrict__ merges, int32_t* __restrict__ meta) {
    __shared__ int n_over;
    const int per = (B + kPlanThreads - 1) / kPlanThreads;
    const int b0 = min(B, static_cast<int>(threadIdx.x) * per), b1 = min(B, b0 + per);
    auto items = [&](int b) { return cnt ? min(max(cnt[b], 0), n_items) : n_items; };
    auto active = [&](int b) { return (full[b] != 0) == (want_full != 0); };
    if (threadIdx.x == 0) n_over = 0;
    __syncthreads();
    int over = 0;
    for (int b = b0; b < b1; ++b) over += (active(b) && items(b) > chunk) ? 1 : 0;
    if (over) atomicAdd(&n_over, over);
    __syncthreads();
    const int s_max = n_over > 0 ? slots / n_over : 0;
    auto splits = [&](int b) {
        const int n = items(b);
        return (n > chunk && s_max >= 2) ? min((n + chunk - 1) / chunk, s_max) : 1;
    };
    // per thread: split tasks, single tasks, merges
    int3 c = make_int3(0, 0, 0);
    for (int b = b0; b < b1; ++b) {
        if (!active(b)) continue;
        const int sb = splits(b);
        if (sb > 1) { c.x += sb; c.z += 1; } else { c.y += 1; }
    }
    int3 tot;
    int3 off = block_scan3(c, tot);
    for (int b = b0; b < b1; ++b) {
        if (!active(b)) continue;
        const int n = items(b), sb = splits(b);
        if (sb > 1) {
            merges[off.z++] = make_int4(b, off.x, sb, 0);
            for (int i = 0; i < sb; ++i) {
                const int lo = static_cast<int>(static_cast<long long>(n) * i / sb);
                const int hi = static_cast<int>(static_cast<long long>(n) * (i + 1) / sb);
                tasks[off.x] = make_int4(b, lo, hi, off.x);
                ++off.x;
            }
        } else {
            tasks[tot.x + off.y++] = make_int4(b, 0, n, -1);
        }
    }
    if (threadIdx.x == 0) {
        meta[0] = tot.x + tot.y;
        meta[1] = tot.z;
        meta[2] = 0;
        meta[3] = 0;
    }
}

// Merge the partial lists of each split pattern into its output rows (one
// wave per pattern; ranking as in the scorer: score descending, ties to the
// lower template index). A pattern with a non-finite norm is flagged as the
// scorer flags it.
__global__ void __launch_bounds__(256)
merge_split(const int4* __restrict__ merges, const int32_t* __restrict__ meta,
            const double* __restrict__ norms, int N, const int32_t* __restrict__ pt,
            const int32_t* __restrict__ ps, const float* __restrict__ pq,
            int32_t* __restrict__ top_t, int32_t* __restrict__ top_s, float* __restrict__ top_q) {
    const int lane = threadIdx.x & 63;
    const int n_merge = meta[1];
    for (int m = (blockIdx.x * 256 + threadIdx.x) >> 6; m < n_merge; m += gridDim.x * 4) {
        const int4 g = merges[m];
        int32_t* ot = top_t + static_cast<size_t>(g.x) * N;
        int32_t* os = top_s + static_cast<size_t>(g.x) * N;
        float* oq = top_q + static_cast<size_t>(g.x) * N;
        const double pn = norms[g.x];
        if ((__double_as_longlong(pn) & 0x7ff0000000000000LL) == 0x7ff0000000000000LL) {
            for (int i = lane; i < N; i += 64) {
                ot[i] = -1;
                os[i] = -1;
                oq[i] = __int_as_float(0x7fc00000);
            }
            continue;
        }
        const size_t e0 = static_cast<size_t>(g.y) * N;
        const int ne = g.z * N;
        float prev_q = INFINITY;
        int prev_t = -1;
        for (int r = 0; r < N; ++r) {
            float bq = -INFINITY;
            int bt = INT_MAX, bs = 0;
            for (int c = lane; c < ne; c += 64) {
                const float q = pq[e0 + c];
                const int t = pt[e0 + c];
                const bool after = (q < prev_q) || (q == prev_q && t > prev_t);
                const bool better = (q > bq) || (q == bq && t < bt);
                if (after && better) { bq = q; bt = t; bs = ps[e0 + c]; }
            }
#pragma unroll
            for (int x = 32; x >= 1; x >>= 1) {
                const float oq2 = __shfl_xor(bq, x, 64);
                const int ot2 = __shfl_xor(bt, x, 64);
                const int os2 = __shfl_xor(bs, x, 64);
                if (oq2 > bq || (oq2 == bq && ot2 < bt)) { bq = oq2; bt = ot2; bs = os2; }
            }
            if (lane == 0) {
                ot[r] = bt;
                os[r] = bs;
                oq[r] = bq;
            }
            prev_q = bq;
            prev_t = bt;
        }
    }
}

// First-pass picks from a short list: the n_first best entries of row b of
// first_q (n_list <= 1024 entries; value descending, list index ascending
// among equal values; NaN ranks last), each written as the template of its
// column first_col[b, i] (-1 for none), in list order. One workgroup per
// pattern: a radix select over order-preserving 32-bit keys finds the
// n_first-th largest key T in four 8-bit passes (LDS histograms), then the
// entries above T and the first entries equal to T are compacted with
// ballots.
constexpr int kPickN = 1024;
__device__ __forceinline__ uint32_t order_key(float v) {
    const uint32_t u = __float_as_uint(v);
    if (v != v) return 0u;
    return (u >> 31) ? ~u : (u | 0x80000000u);
}

__global__ void __launch_bounds__(256)
pick_listed(const float* __restrict__ first_q, const int32_t* __restrict__ first_col, int n_list,
            int n_first, int n_cols, const int32_t* __restrict__ map, int32_t* __restrict__ out) {
    constexpr int KP = kPickN / 256;             // entries per thread: i = 256 k + thread
    __shared__ uint32_t hist[256];
    __shared__ uint32_t sel[2];                  // digit, entries above it in the bucket
    __shared__ int ceq[KP][4], ctk[KP][4];       // per (k, wave): equal to T, taken
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t key[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int i = 256 * k + tid;
        key[k] = i < n_list ? order_key(first_q[static_cast<size_t>(b) * n_list + i]) : 0u;
    }
    // T: the n_first-th largest key, one 8-bit digit per pass
    uint32_t prefix = 0, mask = 0;
    int need = n_first;                          // entries still to take inside the bucket
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KP; ++k)
            if ((key[k] & mask) == prefix) atomicAdd(&hist[(key[k] >> shift) & 255u], 1u);
        __syncthreads();
        if (wave == 0) {
            // lane l holds digits 4 l .. 4 l + 3; above = entries with a
            // larger digit in higher lanes
            uint32_t h[4], sum = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                h[e] = hist[4 * lane + e];
                sum += h[e];
            }
            uint32_t x = sum;                    // inclusive suffix sum over lanes
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = __shfl_down(x, d, 64);
                if (lane + d < 64) x += o;
            }
            uint32_t above = x - sum;
#pragma unroll
            for (int e = 3; e >= 0; --e) {
                if (above < static_cast<uint32_t>(need) && static_cast<uint32_t>(need) <= above + h[e]) {
                    sel[0] = 4 * lane + e;
                    sel[1] = above;
                }
                above += h[e];
            }
        }
        __syncthreads();
        need -= static_cast<int>(sel[1]);
        prefix |= sel[0] << shift;
        mask |= 255u << shift;
        __syncthreads();                         // sel and hist are rewritten next
    }
    // every key above T, and the first `need` keys equal to T in list order
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool eq[KP];
    unsigned long long meq[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        eq[k] = key[k] == prefix;
        meq[k] = tmlib::ballot(eq[k]);
        if (lane == 0) ceq[k][wave] = __popcll(meq[k]);
    }
    __syncthreads();
    bool take[KP];
    unsigned long long mtk[KP];
    int base = 0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        int before = base;
        for (int w = 0; w < wave; ++w) before += ceq[k][w];
        for (int w = 0; w < 4; ++w) base += ceq[k][w];
        before += __popcll(meq[k] & lt);
        take[k] = key[k] > prefix || (eq[k] && before < need);
        mtk[k] = tmlib::ballot(take[k]);
        if (lane == 0) ctk[k][wave] = __popcll(mtk[k]);
    }
    __syncthreads();
    int tb = 0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        int pos = tb;
        for (int w = 0; w < wave; ++w) pos += ctk[k][w];
        for (int w = 0; w < 4; ++w) tb += ctk[k][w];
        pos += __popcll(mtk[k] & lt);
        if (take[k] && pos < n_first) {
            const int i = 256 * k + tid;
            const int c = i < n_list ? first_col[static_cast<size_t>(b) * n_list + i] : -1;
            out[static_cast<size_t>(b) * n_first + pos] = (c >= 0 && c < n_cols) ? (map ? map[c] : c) : -1;
        }
    }
}

// Column indices to templates, in place (-1 stays -1).
__global__ void __launch_bounds__(256)
map_columns(int32_t* __restrict__ idx, size_t n, const int32_t* __restrict__ map) {
    const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n && idx[i] >= 0) idx[i] = map[idx[i]];
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
                             int32_t B, int32_t N, int32_t n_first, const float* Qt,
                             int32_t n_cols, const int32_t* map, double margin, int32_t cap,
                             int32_t* n_rescored, int32_t* top_template, int32_t* top_angle,
                             float* top_score, bool compact, hipStream_t s, const float* first_q,
                             const int32_t* first_col, int32_t n_list) {
    const int Tp = lib->Tp;
    n_first = std::max(N, std::min(n_first, std::min(tmlib::kMaxN, Tp)));
    int r = TM_OK;
    int32_t *t0 = nullptr, *s0 = nullptr, *t1 = nullptr, *s1 = nullptr;
    float *q0 = nullptr, *q1 = nullptr;
    int32_t *cand = nullptr, *cnt = nullptr, *full = nullptr;
    const size_t bn = static_cast<size_t>(B) * N;
    const size_t bf = static_cast<size_t>(B) * n_first;
    if (!r) r = alloc_async(&t0, bf, s);
    if (!r && !first_q) r = alloc_async(&s0, bf, s);   // the top-n's angles and scores
    if (!r && !first_q) r = alloc_async(&q0, bf, s);
    if (!r) r = alloc_async(&t1, bn, s);
    if (!r) r = alloc_async(&s1, bn, s);
    if (!r) r = alloc_async(&q1, bn, s);
    if (!r) r = alloc_async(&cand, static_cast<size_t>(B) * cap, s);
    if (!r) r = alloc_async(&cnt, B, s);
    if (!r) r = alloc_async(&full, B, s);
    // 1. the n_first best estimates (or of the caller's short list), scored
    // exactly: their N-th best, q_N
    if (first_q) {
        if (n_list < n_first) {
            tmlib::set_error("first-pass list of %d entries for %d picks", n_list, n_first);
            r = TM_EINVAL;
        }
        if (!r && n_list > kPickN) {
            tmlib::set_error("first-pass list of %d entries (at most %d)", n_list, kPickN);
            r = TM_EINVAL;
        }
        if (!r) {
            hipLaunchKernelGGL(pick_listed, dim3(B), dim3(256), 0, s, first_q, first_col, n_list,
                               n_first, n_cols, map, t0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) r = tmlib::hip_fail(e, "pick_listed launch");
        }
    } else if (!r) {
        r = tmlib::launch_topn(Qt, nullptr, B, n_cols, n_first, t0, s0, q0, s);
    }
    if (!r && map && !first_q) {
        const size_t n = bf;
        hipLaunchKernelGGL(map_columns, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s,
                           t0, n, map);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "map_columns launch");
    }
    if (!r) r = tmlib::launch_match(lib, polar, norms, B, N, t1, s1, q1, nullptr, nullptr, t0,
                                    n_first, nullptr, nullptr, compact, s);
    // 2. every template whose estimate reaches q_N - margin
    if (!r) {
        // 16-byte loads when every row starts 16-byte aligned
        // with a map, the columns past T' hold no template (map -1)
        const int n_valid = map ? std::min(n_cols, Tp) : n_cols;
        if (n_cols % 4 == 0 && reinterpret_cast<uintptr_t>(Qt) % 16 == 0)
            hipLaunchKernelGGL(certify_select<4>, dim3(B), dim3(kSelThreads), 0, s, Qt, n_cols,
                               n_valid, map, q1, N, margin, cap, cand, cnt, full, n_rescored, Tp,
                               t0, n_first);
        else
            hipLaunchKernelGGL(certify_select<1>, dim3(B), dim3(kSelThreads), 0, s, Qt, n_cols,
                               n_valid, map, q1, N, margin, cap, cand, cnt, full, n_rescored, Tp,
                               t0, n_first);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "certify_select launch");
    }
    // 3. exact scores of the candidates; full scans where the set was too
    // large. Both passes are split launches: long candidate lists and full
    // scans are spread over many workgroups.
    int4 *tasks = nullptr, *merges = nullptr;
    int32_t *meta = nullptr, *pt = nullptr, *ps = nullptr;
    float* pq = nullptr;
    const int slots = kSlotBudget;
    if (!r) r = alloc_async(&tasks, static_cast<size_t>(B) + slots, s);
    if (!r) r = alloc_async(&merges, B, s);
    if (!r) r = alloc_async(&meta, 4, s);
    if (!r) r = alloc_async(&pt, static_cast<size_t>(slots) * N, s);
    if (!r) r = alloc_async(&ps, static_cast<size_t>(slots) * N, s);
    if (!r) r = alloc_async(&pq, static_cast<size_t>(slots) * N, s);
    const int grid = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(B) + slots, kSplitGrid));
    const tmlib::SplitWork work{tasks, meta, pt, ps, pq, grid};
    auto pass = [&](bool want_full) -> int {
        hipLaunchKernelGGL(plan_split, dim3(1), dim3(kPlanThreads), 0, s, full, want_full ? 1 : 0,
                           want_full ? nullptr : cnt, want_full ? lib->n_groups : cap, B,
                           want_full ? kChunkFull : kChunkCand, slots, tasks, merges, meta);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return tmlib::hip_fail(e, "plan_split launch");
        if (int rr = tmlib::launch_match(lib, polar, norms, B, N, top_template, top_angle, top_score,
                                         nullptr, nullptr, want_full ? nullptr : cand,
                                         want_full ? 0 : cap, nullptr, nullptr, compact, s, &work))
            return rr;
        const int mgrid = std::max(1, std::min((B + 3) / 4, 256));
        hipLaunchKernelGGL(merge_split, dim3(mgrid), dim3(256), 0, s, merges, meta, norms, N, pt, ps,
                           pq, top_template, top_angle, top_score);
        e = hipGetLastError();
        if (e != hipSuccess) return tmlib::hip_fail(e, "merge_split launch");
        return TM_OK;
    };
    if (!r) r = pass(false);
    if (!r) {
        hipLaunchKernelGGL(merge_first, dim3(static_cast<unsigned>((B + 3) / 4)), dim3(256), 0, s, full,
                           B, norms, N, t1, s1, q1, top_template, top_angle, top_score);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "merge_first launch");
    }
    if (!r) r = pass(true);
    for (void* p : {static_cast<void*>(t0), static_cast<void*>(s0), static_cast<void*>(q0),
                    static_cast<void*>(t1), static_cast<void*>(s1), static_cast<void*>(q1),
                    static_cast<void*>(cand), static_cast<void*>(cnt), static_cast<void*>(full),
                    static_cast<void*>(tasks), static_cast<void*>(merges), static_cast<void*>(meta),
                    static_cast<void*>(pt), static_cast<void*>(ps), static_cast<void*>(pq)})
        if (p) (void)hipFreeAsync(p, s);
    return r;
}
