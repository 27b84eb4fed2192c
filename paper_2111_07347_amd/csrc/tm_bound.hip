// Window upper bounds of the in-plane search and the exact search built on
// them.
//
// The plain path (Section 2.2, Fig. 2 e) slides every template over all
// n_theta columns of the polar image and keeps its best Q of Eq. (1). Most
// templates are far from the best ones, and for them a cheap bound settles
// the matter. With non-negative template weights w_i, for any window of
// `win` consecutive shifts starting at coarse shift S (s = S win + d,
// 0 <= d < win):
//
//   C(s) = sum_i w_i P[j_i, k_i + s] <= sum_i w_i M[j_i, k_i + S win],
//   M[j, x] = max(0, max_{0 <= d < win} P[j, (x + d) mod n_theta]),
//
// so one product per spot and coarse shift bounds a whole window of shifts,
// and the maximum over the coarse shifts bounds the template's best score.
// The bounds feed the certified rescoring (tm_certify.hip) with margin 0:
// the N templates with the largest bounds are scored exactly, every
// template whose bound reaches their N-th best exact score is scored
// exactly, and the result is the plain path's top-N (same float32 sums in
// the same order, so the same bits).
//
// Rigour in finite precision. The bound is evaluated with M scaled by a
// power of two and rounded up to float16, the weights (times 2^10) rounded
// up to float16, float32 products (exact) and float32 sums of non-negative
// terms (relative error at most gamma_n); the plain path's own float32 sum
// may exceed the exact C(s) by gamma_n sum_i w_i |P_i| <= gamma_n (sum_i
// w_i) A, A = max |P| over the library's rows. The stored bound is
//
//   Q^_t = ((UB_t / scale) / (1 - gamma_nmax) + gamma_{n_t} (sum w) A)
//          * (1 / ||P||) * (1 + 2^-20),   rounded up,
//
// which is at least the plain path's float32 Q_t of every template.
//
// Kernel layout (one workgroup per pattern):
//   * the window image M of the library's touched rows is built in LDS in
//     float16. When n_theta = 4 win, each row holds per phase p < win the 7
//     values M[p + win W] (W = 0..6, columns mod n_theta), so the 4 coarse
//     shifts of a pixel at column q win + p are the 4 consecutive values
//     from slot q (8 bytes: few bank conflicts); otherwise rows of
//     n_theta + 3 win columns are read at k + win S (the halo avoids any
//     modulo);
//   * a wave scores 16 templates at a time, lane = 4 slot + coarse shift S
//     (4 coarse shifts of win = ceil(n_theta / 4) columns); templates are
//     sorted by pixel count and their records interleaved per chunk of 16 in
//     blocks of 4 steps (whole units of 8 steps, zero-weight padding), all
//     slots of a chunk running the same number of steps;
//   * records reach the wave through LDS: each 512-byte unit is loaded with
//     distinct addresses by the whole wave (no broadcast loads), written to
//     one of two LDS buffers a unit ahead of its use and read back by the
//     slots;
//   * per record: one LDS read of a float16 window maximum and one mixed
//     float16 x float16 + float32 multiply-add.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "tm_device.h"
#include "tm_internal.h"

namespace {

constexpr int kShifts = 4;                 // coarse shifts per template
constexpr int kSlots = 64 / kShifts;       // templates per wave step
constexpr int kBlk = 4;                    // steps per block of records (one 16-byte read)
constexpr int kUnitSteps = 8;              // steps per unit (the stream's granularity)
constexpr int kUnitBlocks = kUnitSteps / kBlk;
constexpr int kWslots = 2 * kShifts - 1;   // window values per phase (blocked layout)
constexpr int kRing = 8;                   // chunks per result flush
constexpr int kWeightExp = 10;             // float16 weights carry w * 2^10
constexpr int kImageExp = 14;              // window maxima scaled below 2^14
constexpr size_t kLdsBudget = 128 * 1024;  // window image (16-bit offsets)
constexpr int kFirst = 32;                 // best bounds scored exactly first
constexpr int kMaxCols = 12;               // window columns per lane (n_theta <= 768)

// ---------------------------------------------------------------- host side

double gamma32(double n) {
    const double u = std::ldexp(1.0, -24);
    return n * u / (1.0 - n * u);
}

// float16 bits of the smallest float16 >= x (0 <= x < 65504).
uint16_t half_up(float x) {
    const _Float16 h = static_cast<_Float16>(x);
    uint16_t b;
    std::memcpy(&b, &h, 2);
    if (static_cast<float>(h) < x) ++b;
    return b;
}

// ---------------------------------------------------------------- device side

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float h2f(uint32_t bits16) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(bits16)));
}

// float16 bits of the smallest float16 >= x (0 <= x <= 2^14).
__device__ __forceinline__ uint16_t f16_up(float x) {
    const _Float16 h = static_cast<_Float16>(x);
    uint16_t b = __builtin_bit_cast(uint16_t, h);
    if (static_cast<float>(h) < x) ++b;
    return b;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// One unit of records (8 steps x 16 slots, 512 bytes) loaded with distinct addresses:
// lane l holds bytes 8 l .. 8 l + 7.
__device__ __forceinline__ u32x2 load_unit(const u32x2* units, int uu, int lane) {
    return units[static_cast<size_t>(uu) * 64 + lane];
}

typedef __attribute__((address_space(3))) const uint16_t lds_u16;

// LDS byte address of a record's window value for this lane: the record's
// 16-bit half offset times 2 plus the lane's base, in one multiply-add of
// the low 16 bits (v_mad_u32_u16).
__device__ __forceinline__ uint32_t rec_addr(uint32_t rec, uint32_t lane_base) {
    uint32_t a;
    asm("v_mad_u32_u16 %0, %1, 2, %2" : "=v"(a) : "v"(rec), "v"(lane_base));
    return a;
}

// Sum of weight x window maximum over one unit's records, read from the
// wave's LDS copy of the unit (block k of this slot: 16 bytes at
// (kSlots k + slot) 16; the lanes of a slot read the same bytes), all window
// reads in flight before the multiply-adds.
__device__ __forceinline__ float score_unit(const u32x4* buf, int slot, uint32_t lane_base,
                                            float acc, uint32_t& chunk_done) {
    u32x4 R[kUnitBlocks];
#pragma unroll
    for (int k = 0; k < kUnitBlocks; ++k) R[k] = buf[k * kSlots + slot];
    // the last record's weight sign bit marks a chunk's last unit
    chunk_done = R[kUnitBlocks - 1][kBlk - 1] >> 31;
    R[kUnitBlocks - 1][kBlk - 1] &= 0x7fffffffu;
    float v[kUnitSteps];
#pragma unroll
    for (int k = 0; k < kUnitBlocks; ++k)
#pragma unroll
        for (int u = 0; u < kBlk; ++u)
            v[kBlk * k + u] = h2f(*reinterpret_cast<lds_u16*>(
                static_cast<uintptr_t>(rec_addr(R[k][u], lane_base))));
#pragma unroll
    for (int k = 0; k < kUnitBlocks; ++k)
#pragma unroll
        for (int u = 0; u < kBlk; ++u) acc = fmaf(h2f(R[k][u] >> 16), v[kBlk * k + u], acc);
    return acc;
}

template <int NW>
__global__ void __launch_bounds__(NW * 64)
bound_kernel(const float* __restrict__ polar, const double* __restrict__ norms, int Rs, int n,
             const int* __restrict__ rows, int n_rows, int Lrow, int win, int blocked,
             const uint32_t* __restrict__ recs, const int* __restrict__ chunk_end,
             const int* __restrict__ part, int n_chunks, float* __restrict__ raw,
             float4* __restrict__ pat) {
    extern __shared__ uint16_t m16[];        // window image
    __shared__ float red[NW];
    __shared__ u32x4 rbuf[NW][2][kUnitBlocks * kSlots];   // per wave: two units of records
    __shared__ float res[NW][kRing][kSlots];  // per wave: window maxima of kRing chunks
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = tmlib::uniform(threadIdx.x >> 6);
    const float* src = polar + static_cast<size_t>(b) * Rs * n;
    float* rrow = raw + static_cast<size_t>(b) * n_chunks * kSlots;
    const double pn = norms[b];
    // a non-finite norm: the exact scorer flags the pattern; bounds are moot
    if ((__double_as_longlong(pn) & 0x7ff0000000000000LL) == 0x7ff0000000000000LL) {
        if (threadIdx.x == 0) pat[b] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    // 1. A = max |P| over the touched rows, and the image scale
    float a = 0.0f;
    for (int r = wave; r < n_rows; r += NW) {
        const float* row = src + static_cast<size_t>(rows ? rows[r] : r) * n;
        for (int c = lane; c < n; c += 64) a = fmaxf(a, fabsf(row[c]));
    }
    a = tmlib::wave_max(a);
    if (lane == 0) red[wave] = a;
    __syncthreads();
    float A = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) A = fmaxf(A, red[w]);
    int e = 0;
    (void)frexpf(A, &e);                        // A = m 2^e, m in [0.5, 1)
    const float scale = A > 0.0f ? ldexpf(1.0f, kImageExp - e) : 1.0f;
    // 2. window maxima (clamped at 0), scaled, rounded up to float16. The
    // image is periodic (M[x + n] = M[x]): lane l computes the o consecutive
    // columns x0 = o l .. x0 + o - 1 of [0, n) from the o + win - 1 values
    // they span: the maximum of the part every window shares, then the
    // head's suffix maxima and the tail's prefix maxima; each column is
    // stored at x and, inside the halo, at x + n.
    const int o = (n + 63) / 64;                 // columns per lane (<= kMaxCols)
    for (int r = wave; r < n_rows; r += NW) {
        const float* row = src + static_cast<size_t>(rows ? rows[r] : r) * n;
        uint16_t* dst = m16 + static_cast<size_t>(r) * Lrow;
        const int x0 = o * lane;
        if (x0 < n) {
            auto at = [&](int j) {
                const int c = x0 + j;
                return row[c < n ? c : c - n];
            };
            // loads are issued in independent batches (indices clamped, not
            // branched on), so they are in flight together
            float common = 0.0f;                 // columns o - 1 .. win - 1 of the span
            for (int j = o - 1; j < win; j += 8) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = at(min(j + u, win - 1));
#pragma unroll
                for (int u = 0; u < 8; ++u) common = fmaxf(common, v[u]);
            }
            float hv[kMaxCols], tv[kMaxCols];
#pragma unroll
            for (int d = 0; d < kMaxCols; ++d) {
                hv[d] = at(min(d, max(o - 2, 0)));          // head: columns 0 .. o - 2
                tv[d] = at(win - 1 + min(max(d, 1), o - 1));  // tail: columns win .. win + o - 2
            }
            float out[kMaxCols];
            float hmax = common, tmax = common;
#pragma unroll
            for (int d = kMaxCols - 1; d >= 0; --d) {
                if (d < o - 1) hmax = fmaxf(hmax, hv[d]);
                out[d] = hmax;
            }
#pragma unroll
            for (int d = 1; d < kMaxCols; ++d) {
                if (d < o) tmax = fmaxf(tmax, tv[d]);
                out[d] = fmaxf(out[d], tmax);
            }
#pragma unroll
            for (int d = 0; d < kMaxCols; ++d) {
                const int x = x0 + d;
                if (d < o && x < n) {
                    const uint16_t h = f16_up(out[d] * scale);
                    if (blocked) {
                        // phase p = x mod win, window W0 = x div win, at W0
                        // and (for W0 < 3) W0 + 4 of the phase's 7 slots
                        const int W0 = x / win, p = x - W0 * win;
                        dst[p * kWslots + W0] = h;
                        if (W0 < kShifts - 1) dst[p * kWslots + W0 + kShifts] = h;
                    } else {
                        dst[x] = h;
                        if (x + n < Lrow) dst[x + n] = h;
                    }
                }
            }
        }
    }
    __syncthreads();
    // 3. bounds, kSlots templates per wave step
    const int slot = lane / kShifts;
    const int S = lane % kShifts;
    const uint32_t soff = static_cast<uint32_t>(blocked ? S : S * win);
    // per-pattern factors of the stored bound (bound_finalize): the largest
    // |P|, the image and weight scale, 1 / ||P|| rounded up
    float invP = 0.0f;
    if (pn > 0.0) {
        const double ip = 1.0 / pn;
        invP = static_cast<float>(ip);
        if (static_cast<double>(invP) < ip) invP = nextafterf(invP, INFINITY);
    }
    const float out_scale = 1.0f / (scale * static_cast<float>(1 << kWeightExp));   // power of 2
    if (threadIdx.x == 0) pat[b] = make_float4(A, out_scale, invP, 1.0f);
    const uint32_t lane_base =
        static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_u16*)m16)) + 2u * soff;
    // the wave's chunks [c_begin, c_end) hold about 1/NW of the records; the
    // wave streams their units in order, one accumulator per template
    const int c_begin = part[wave], c_end = part[wave + 1];
    if (c_begin >= c_end) return;
    const u32x2* units = reinterpret_cast<const u32x2*>(recs);
    u32x2* wb0 = reinterpret_cast<u32x2*>(&rbuf[wave][0][0]);
    u32x2* wb1 = reinterpret_cast<u32x2*>(&rbuf[wave][1][0]);
    const int u_begin = (c_begin == 0) ? 0 : chunk_end[c_begin - 1];
    const int u_end = chunk_end[c_end - 1];
    int c = c_begin;
    float acc = 0.0f;
    // A chunk's last unit carries a flag (bit 31 of every slot's last record,
    // a weight's sign bit, always 0 otherwise): no memory access in the
    // stream besides the records. Each chunk's window maxima go to the
    // wave's LDS ring and leave for memory kRing chunks at a time.
    int ring0 = c_begin;                        // first chunk held by the ring
    auto flush = [&]() {
        for (int i = lane; i < (c - ring0) * kSlots; i += 64)
            rrow[static_cast<size_t>(ring0) * kSlots + i] = res[wave][i / kSlots][i % kSlots];
        ring0 = c;
    };
    auto finish = [&]() {
        float m = acc;
#pragma unroll
        for (int x = 1; x < kShifts; x <<= 1) m = fmaxf(m, __shfl_xor(m, x, 64));
        if (S == 0) res[wave][c - ring0][slot] = m;
        acc = 0.0f;
        ++c;
        if (c - ring0 == kRing) flush();
    };
    // Records stream through the wave's two LDS unit buffers: each unit is
    // loaded with distinct addresses two units ahead, written to LDS one unit
    // ahead, and read back by each slot's lanes (the wave's own LDS
    // accesses complete in order, so no barrier is needed).
    const int last = u_end - 1;
    u32x2 ga = load_unit(units, u_begin, lane);
    u32x2 gb = load_unit(units, min(u_begin + 1, last), lane);
    __builtin_amdgcn_sched_barrier(0);
    wb0[lane] = ga;
    int u = u_begin;
    for (; u + 1 < u_end; u += 2) {
        // buffer 0 holds unit u; gb (in flight) unit u + 1
        ga = load_unit(units, min(u + 2, last), lane);
        __builtin_amdgcn_sched_barrier(0);
        wb1[lane] = gb;
        uint32_t end0;
        acc = score_unit(&rbuf[wave][0][0], slot, lane_base, acc, end0);
        if (__builtin_amdgcn_readfirstlane(end0)) finish();
        // buffer 1 holds unit u + 1; ga (in flight) unit u + 2
        gb = load_unit(units, min(u + 3, last), lane);
        __builtin_amdgcn_sched_barrier(0);
        wb0[lane] = ga;
        uint32_t end1;
        acc = score_unit(&rbuf[wave][1][0], slot, lane_base, acc, end1);
        if (__builtin_amdgcn_readfirstlane(end1)) finish();
    }
    if (u < u_end) {                           // an odd last unit, in buffer 0
        uint32_t end0;
        acc = score_unit(&rbuf[wave][0][0], slot, lane_base, acc, end0);
        if (__builtin_amdgcn_readfirstlane(end0)) finish();
    }
    if (c > ring0) flush();
}

// Bounds in template order: Q^_t = ((m_t out_scale) dfac + c_t A) invP
// (1 + 2^-19), from each chunk slot's window maximum m_t and the pattern's
// factors (every operand non-negative; five float roundings of at most
// 2^-24 each are more than restored by the last factor). A pattern with a
// non-finite norm gets 0.
__global__ void __launch_bounds__(256)
bound_finalize(const float* __restrict__ raw, const float4* __restrict__ pat,
               const int2* __restrict__ tc, int n_cs, int Tp, float dfac, float* __restrict__ Qt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= n_cs) return;
    const int2 e = tc[i];
    if (e.x < 0) return;
    const float4 p = pat[b];
    const float m = raw[static_cast<size_t>(b) * n_cs + i];
    Qt[static_cast<size_t>(b) * Tp + e.x] =
        p.w != 0.0f ? ((m * p.y) * dfac + __int_as_float(e.y) * p.x) * p.z * (1.0f + 0x1p-19f) : 0.0f;
}

}  // namespace

// ------------------------------------------------------------ library data

int tmlib::bound_prepare(tm_library* L, const std::vector<std::vector<HostPixel>>& pix,
                         const std::vector<int32_t>& row_index, hipStream_t s, size_t& bytes) {
    L->bound = false;
    const int n = L->n_theta;
    const int T = L->T, Tp = L->Tp;
    for (const auto& v : pix)
        for (const HostPixel& p : v)
            if (!(p.w >= 0.0)) return TM_OK;           // bounds need non-negative weights
    const int win = (n + kShifts - 1) / kShifts;
    // Window image layout. Blocked (n_theta = 4 win): per row and phase
    // p < win, 7 slots W holding M[p + win W mod n]; a pixel at column
    // k = q win + p reads slots q + S for the 4 coarse shifts S: 8
    // consecutive bytes per template and step, few LDS bank conflicts.
    // Otherwise rows of n + 3 win columns (a halo past n) read at k + win S.
    const bool blocked = (n % kShifts) == 0;
    int Lrow = blocked ? win * kWslots : n + (kShifts - 1) * win;
    Lrow += Lrow & 1;
    const size_t halves = static_cast<size_t>(std::max(L->n_rows, 1)) * Lrow;
    if (halves * 2 > kLdsBudget || halves > 65536) return TM_OK;   // window image too large

    // per template: records (offset, float16 weight), pixel count, margin factor
    std::vector<std::vector<uint32_t>> tr(Tp);
    std::vector<int32_t> cnt(Tp, 0);
    std::vector<float> cfac(Tp, 0.0f);
    int nmax = 0;
    for (int32_t tt = 0; tt < Tp; ++tt) {
        const int32_t t = tt < T ? tt : tt - T;
        const bool is_mirror = tt >= T;
        const double nrm = L->tnorm[t];
        double wsum = 0.0;
        for (const HostPixel& p : pix[t]) {
            const int k = is_mirror ? (n - p.k) % n : p.k;
            const float w32 = nrm > 0.0 ? static_cast<float>(p.w / nrm) : 0.0f;
            wsum += w32;
            const uint32_t off = static_cast<uint32_t>(row_index[p.j]) * Lrow +
                                 (blocked ? (k % win) * kWslots + k / win : k);
            const uint32_t w16 = half_up(std::ldexp(w32, kWeightExp));
            tr[tt].push_back(off | (w16 << 16));
        }
        cnt[tt] = static_cast<int32_t>(pix[t].size());
        nmax = std::max(nmax, cnt[tt]);
        cfac[tt] = static_cast<float>(gamma32(cnt[tt]) * wsum * (1.0 + 0x1p-20));
    }
    // chunks of kSlots templates of similar size, records interleaved per step
    std::vector<int32_t> order(Tp);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cnt[a] > cnt[b]; });
    const int32_t n_chunks = (Tp + kSlots - 1) / kSlots;
    // per (chunk, slot): template (-1 none) and margin factor bits; per
    // chunk: its first unit after it
    std::vector<int32_t> tc(static_cast<size_t>(n_chunks) * kSlots * 2, 0);
    std::vector<int32_t> cend(n_chunks, 0);
    std::vector<uint32_t> recs;
    std::vector<int64_t> chunk_end(n_chunks);
    for (int32_t c = 0; c < n_chunks; ++c) {
        int m = 0;
        int32_t tid[kSlots];
        for (int sl = 0; sl < kSlots; ++sl) {
            const int32_t idx = c * kSlots + sl;
            tid[sl] = idx < Tp ? order[idx] : -1;
            if (tid[sl] >= 0) m = std::max(m, cnt[tid[sl]]);
        }
        m = std::max(kUnitSteps, (m + kUnitSteps - 1) / kUnitSteps * kUnitSteps);   // whole units
        // per step, one record per slot; in the blocked layout the records of
        // a step are chosen so that the slots' 16-byte reads fall on distinct
        // LDS banks where possible (a template's records may come in any
        // order: the bound's sum and its margin do not depend on it)
        std::vector<std::vector<uint32_t>> step(m, std::vector<uint32_t>(kSlots, 0u));
        if (blocked) {
            std::vector<std::vector<uint32_t>> left(kSlots);
            for (int sl = 0; sl < kSlots; ++sl)
                if (tid[sl] >= 0) left[sl] = tr[tid[sl]];
            auto banks = [](uint32_t rec) {          // 32 banks of 4 bytes
                const uint32_t h0 = rec & 0xffffu;
                uint32_t mask = 0;
                for (uint32_t d = h0 / 2; d <= (h0 + kShifts - 1) / 2; ++d) mask |= 1u << (d % 32);
                return mask;
            };
            for (int i = 0; i < m; ++i) {
                uint32_t used = 0;
                for (int sl = 0; sl < kSlots; ++sl) {
                    auto& L_ = left[sl];
                    if (L_.empty()) {
                        // padding (weight 0): a read on free banks
                        uint32_t pad = 0;
                        for (uint32_t h = 0; h < 64 && h + kShifts <= halves; h += 8)
                            if (!(banks(h) & used)) { pad = h; break; }
                        step[i][sl] = pad;
                        used |= banks(pad);
                        continue;
                    }
                    size_t best = 0;
                    int best_c = 99;
                    const size_t lim = std::min<size_t>(L_.size(), 24);
                    for (size_t e = 0; e < lim && best_c > 0; ++e) {
                        const int c_ = __builtin_popcount(banks(L_[e]) & used);
                        if (c_ < best_c) { best_c = c_; best = e; }
                    }
                    step[i][sl] = L_[best];
                    used |= banks(L_[best]);
                    L_.erase(L_.begin() + static_cast<long>(best));
                }
            }
        } else {
            for (int i = 0; i < m; ++i)
                for (int sl = 0; sl < kSlots; ++sl)
                    step[i][sl] = tid[sl] >= 0 && i < cnt[tid[sl]] ? tr[tid[sl]][i] : 0u;
        }
        // the last step's records carry the chunk-end flag (a weight's sign
        // bit; weights are non-negative)
        for (int sl = 0; sl < kSlots; ++sl) step[m - 1][sl] |= 0x80000000u;
        for (int q = 0; q < m; q += kBlk)
            for (int sl = 0; sl < kSlots; ++sl)
                for (int i = q; i < q + kBlk; ++i) recs.push_back(step[i][sl]);
        chunk_end[c] = static_cast<int64_t>(recs.size() / (kUnitSteps * kSlots));
        if (chunk_end[c] > INT32_MAX / 8) return TM_OK;
        cend[c] = static_cast<int32_t>(chunk_end[c]);
        for (int sl = 0; sl < kSlots; ++sl) {
            int32_t* hp = &tc[(static_cast<size_t>(c) * kSlots + sl) * 2];
            hp[0] = tid[sl];
            const float cf = tid[sl] >= 0 ? cfac[tid[sl]] : 0.0f;
            std::memcpy(&hp[1], &cf, 4);
        }
    }
    // chunk ranges of the waves of an 8-wave and a 16-wave workgroup, each
    // about 1/NW of the units (chunks are contiguous per wave)
    std::vector<int32_t> part;
    const int64_t units = n_chunks ? chunk_end[n_chunks - 1] : 0;
    for (int nw : {8, 16}) {
        for (int w = 0; w <= nw; ++w) {
            const int64_t target = units * w / nw;
            int32_t c = 0;
            while (c < n_chunks && (c == 0 ? 0 : chunk_end[c - 1]) < target) ++c;
            part.push_back(w == nw ? n_chunks : c);
        }
    }

    auto up = [&](auto** dst, const auto& v) -> int {
        using T = std::remove_reference_t<decltype(v[0])>;
        const size_t nb = std::max<size_t>(v.size(), 1) * sizeof(T);
        hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), nb);
        if (e != hipSuccess) {
            *dst = nullptr;
            tmlib::set_error("hipMalloc(%zu) failed: %s", nb, hipGetErrorString(e));
            return TM_ENOMEM;
        }
        bytes += nb;
        if (!v.empty()) TM_HIP(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
        return TM_OK;
    };
    if (int r = up(&L->d_bnd_recs, recs)) return r;
    if (int r = up(&L->d_bnd_end, cend)) return r;
    if (int r = up(&L->d_bnd_tc, tc)) return r;
    if (int r = up(&L->d_bnd_part, part)) return r;
    L->bnd_win = win;
    L->bnd_shifts = kShifts;
    L->bnd_L = Lrow;
    L->bnd_blocked = blocked;
    L->bnd_chunks = n_chunks;
    L->bnd_dfac = static_cast<float>(1.0 / (1.0 - gamma32(nmax)) * (1.0 + 0x1p-22));
    L->bound = true;
    return TM_OK;
}

void tmlib::bound_release(tm_library* L) {
    (void)hipFree(L->d_bnd_recs);
    (void)hipFree(L->d_bnd_end);
    (void)hipFree(L->d_bnd_tc);
    (void)hipFree(L->d_bnd_part);
    L->d_bnd_recs = nullptr;
    L->d_bnd_end = nullptr;
    L->d_bnd_tc = nullptr;
    L->d_bnd_part = nullptr;
    L->bound = false;
}

// ------------------------------------------------------------ launches

int tmlib::bound_scores_impl(const tm_library* L, const float* polar, const double* norms,
                             int32_t B, float* Qt, bool compact, hipStream_t s) {
    const size_t lds = static_cast<size_t>(std::max(L->n_rows, 1)) * L->bnd_L * sizeof(uint16_t);
    const int Rs = compact ? L->n_rows : L->R;
    const int* rows = compact ? nullptr : L->d_rows;
    const int n_cs = L->bnd_chunks * kSlots;
    // scratch: per pattern the chunk slots' window maxima and four factors
    float* raw = nullptr;
    TM_HIP(hipMallocAsync(reinterpret_cast<void**>(&raw),
                          static_cast<size_t>(B) * n_cs * sizeof(float) + static_cast<size_t>(B) * 16 + 16,
                          s));
    // the factors start at the next 16-byte boundary after the maxima
    const size_t nraw = (static_cast<size_t>(B) * n_cs + 3) / 4 * 4;
    float4* pat = reinterpret_cast<float4*>(raw + nraw);
    auto launch = [&](auto kern, int nw) -> int {
        TM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
        hipLaunchKernelGGL(kern, dim3(B), dim3(nw * 64), lds, s, polar, norms, Rs, L->n_theta, rows,
                           L->n_rows, L->bnd_L, L->bnd_win, L->bnd_blocked ? 1 : 0, L->d_bnd_recs,
                           L->d_bnd_end, L->d_bnd_part + (nw == 8 ? 0 : 9), L->bnd_chunks, raw, pat);
        TM_HIP(hipGetLastError());
        return TM_OK;
    };
    // one workgroup per CU when the image fills the LDS: use every wave slot
    int r = lds > 64 * 1024 ? launch(bound_kernel<16>, 16) : launch(bound_kernel<8>, 8);
    if (!r) {
        hipLaunchKernelGGL(bound_finalize, dim3((n_cs + 255) / 256, B), dim3(256), 0, s, raw, pat,
                           reinterpret_cast<const int2*>(L->d_bnd_tc), n_cs, L->Tp, L->bnd_dfac, Qt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "bound_finalize launch");
    }
    hipError_t e = hipFreeAsync(raw, s);
    if (!r && e != hipSuccess) r = tmlib::hip_fail(e, "hipFreeAsync");
    return r;
}

int tmlib::bound_match(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                       int32_t N, double cap_frac, int32_t* n_rescored, int32_t* top_template,
                       int32_t* top_angle, float* top_score, bool compact, hipStream_t s) {
    const int Tp = lib->Tp;
    float* Qt = nullptr;
    TM_HIP(hipMallocAsync(reinterpret_cast<void**>(&Qt), static_cast<size_t>(B) * Tp * sizeof(float), s));
    int r = bound_scores_impl(lib, polar, norms, B, Qt, compact, s);
    const double frac = cap_frac > 0.0 ? cap_frac : 0.1;
    int32_t cap = static_cast<int32_t>(std::ceil(frac * Tp - 1e-9));
    cap = std::max(N, std::min(cap, Tp));
    // the bound ranks templates less sharply than the exact score: score the
    // 32 best bounds exactly first, so that the threshold starts high
    if (!r) r = tmlib::certified_rescore(lib, polar, norms, B, N, std::max(N, kFirst), Qt, 0.0,
                                         cap, n_rescored, top_template, top_angle, top_score,
                                         compact, s);
    hipError_t e = hipFreeAsync(Qt, s);
    if (!r && e != hipSuccess) r = tmlib::hip_fail(e, "hipFreeAsync");
    return r;
}

// --------------------------------------------------------------- C ABI

extern "C" int tm_bound_scores(const tm_library* lib, const float* polar, const double* norms,
                               int32_t B, int32_t compact_rows, float* bound_out,
                               void* hip_stream) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (compact_rows != 0 && compact_rows != 1) { tmlib::set_error("compact_rows=%d must be 0 or 1", compact_rows); return TM_EINVAL; }
    if (!lib->bound) {
        tmlib::set_error("window bounds need non-negative template weights and a window image "
                         "of at most 64k columns x rows");
        return TM_EUNSUPPORTED;
    }
    if (B == 0) return TM_OK;
    if (!polar || !norms || !bound_out) {
        tmlib::set_error("polar, norms and bound_out must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    return tmlib::bound_scores_impl(lib, polar, norms, B, bound_out, compact_rows == 1,
                                    static_cast<hipStream_t>(hip_stream));
}
