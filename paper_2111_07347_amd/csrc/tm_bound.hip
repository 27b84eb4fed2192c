// Window upper bounds of the in-plane search and the exact search built on
// them.
//
// The plain path (Section 2.2, Fig. 2 e) slides every template over all
// n_theta columns of the polar image and keeps its best Q of Eq. (1). Most
// templates are far from the best ones, and for them a cheap bound settles
// the matter. With non-negative template weights w_i, for any window of
// `win` = ceil(n_theta / 4) consecutive shifts starting at coarse shift S
// (s = S win + d, 0 <= d < win; S = 0 .. 3 covers every shift):
//
//   C(s) = sum_i w_i P[j_i, k_i + s] <= sum_i w_i M[j_i, k_i + S win],
//   M[j, x] = max(0, max_{0 <= d < wlen} P[j, (x + d) mod n_theta]),
//
// (columns mod n_theta; wlen = min(win + 4 win - n_theta, n_theta), i.e.
// win when 4 divides n_theta, see below), so one product per spot and coarse shift
// bounds a whole window of shifts, and the maximum over the coarse shifts
// bounds the template's best score.
// The bounds feed the certified rescoring (tm_certify.hip) with margin 0:
// a few templates with large bounds (the 48 best of the kernel's per-lane
// largest bounds) are scored exactly, every template whose bound reaches
// the N-th best of those exact scores is scored exactly, and the result is
// the plain path's top-N (same float32 sums in the same order, so the same
// bits); which templates come first only changes how many pass.
//
// Rigour in finite precision. The plain path's own float32 sum may exceed
// the exact C(s) by gamma_n sum_i w_i |P_i| <= gamma_n (sum_i w_i) A, A =
// max |P| over the library's rows, so the bound adds c_t A, c_t =
// gamma_{n_t} sum_i w_i. The kernel evaluates
//
//   U_t = sum_i w^_i M^_i + c^_t A^   (float32 sums of non-negative terms)
//
// with M and A scaled by a power of two and rounded up to float16 (M^, A^)
// and the weights and c_t times 2^10 rounded up to float16 (w^, c^); the
// products are exact and the float32 sum of n_t + 1 terms is within
// gamma_{n_t + 1} of the exact one. The stored bound is
//
//   Q^_t = (U_t / (scale 2^10)) / (1 - gamma_{nmax + 1}) / ||P|| * (1 + 2^-19),
//
// rounded up, which is at least the plain path's float32 Q_t of every
// template.
//
// Quarter-turn pairing. A pixel at column k = q win + r (q = 0..3, r <
// win) needs M at r + (q + S) win for S = 0..3, the 4 maxima M[r + i win],
// i = 0..3, in some rotation. The window image stores them as two dwords,
//
//   Y[j, r] = (M[j, r], M[j, r + 2 win]),  Y[j, r + win] = (M[j, r + win],
//   M[j, r + 3 win])                         (float16 each, columns mod n),
//
// one row of 2 win dwords (plus one unused, for an odd pitch) per touched
// row, read with one 2-dword LDS read at r and r + win. acc[i] collects
// M[r + i win], which is shift S = i - q (mod 4): the pixels of one quarter
// share the rotation. A lane takes its
// template's quarters in cyclic order (its largest first); between two
// quarters every lane moves the value of shift S from acc[S + q] to
// acc[S + q + 1], the same operation in every lane. When 4 does not divide
// n, i = q + S - 4 for q + S >= 4 stands for column r + (q + S) win - n =
// r + i win + 4 win - n: read 4 win - n columns early, which the wider
// windows cover.
//
// Kernel layout (one workgroup per pattern):
//   * the window image Y of the library's touched rows is built in LDS (8
//     waves build rows); the image and those waves' row buffers fit two
//     workgroups in a CU's LDS for most libraries;
//   * a lane scores one template over the 4 coarse shifts S, a wave 64
//     templates at a time: templates are sorted by the pixel counts of
//     their quarter slots (in the lane's order; in whole units first) and
//     cut into chunks of 64; in a chunk all lanes run the same number of
//     steps in each slot (zero-weight padding to whole units of 4 steps);
//     image rows are placed so that the LDS banks the slots read are loaded
//     evenly;
//   * a lane's records come 4 at a time in one 16-byte buffer load (a wave
//     loads 1 KiB of consecutive bytes per unit, 3 units ahead of their
//     use); the units that end a chunk's quarter slots are known per chunk
//     and compared with the unit counter on the scalar unit;
//   * each template's margin term (below) is one more record: its weight
//     the margin factor, its window maxima read from an extra image row
//     that holds the largest |P| (scaled, rounded up) everywhere;
//   * per record: one address multiply-add, one 2-dword LDS read (two
//     pairs of float16 window maxima) and 4 mixed float16 x float16 +
//     float32 multiply-adds; the library orders each step's records over the
//     lanes so that the reads of a half-wave fall on distinct LDS banks (or
//     the same dword) where possible;
//   * a chunk's bounds leave as one coalesced 256-byte store, in chunk-slot
//     order (the library's slot -> template map goes with them).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "tm_device.h"
#include "tm_internal.h"

namespace {

constexpr int kShifts = 4;                 // coarse shifts per template
constexpr int kLanes = 64;                 // templates per chunk, one per lane
constexpr int kUnitSteps = 4;              // records per lane and unit (one 16-byte load)
constexpr int kBanks = 32;                 // LDS banks of 4 bytes, per half-wave
constexpr int kChoices = 64;               // records tried per lane and step
constexpr int kWeightExp = 10;             // float16 weights carry w * 2^10
constexpr int kImageExp = 14;              // window maxima scaled below 2^14
constexpr size_t kLdsBudget = 128 * 1024;  // window image (16-bit offsets)
constexpr int kFirst = 48;                 // best bounds scored exactly first
constexpr int kBuildWaves = 8;             // waves that build the window image's rows
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

// Per-wave LDS scratch of the window-image build, in halves: a row of n
// columns plus a halo of wlen + o, and its block maxima (blocks of o).
size_t scratch_halves(int n, int win) {
    const int o = (n + 63) / 64;
    const int wlen = std::min(5 * win - n, n);
    const int H = wlen + o;
    const int nb = (n + H) / o;
    return static_cast<size_t>(n + H + nb + 7) / 8 * 8;
}

// ---------------------------------------------------------------- device side

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const uint16_t lds_u16;
typedef __attribute__((address_space(3))) const uint32_t lds_u32;

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

// LDS byte address of a record's first pair: the record's 16-bit dword
// offset times 4 plus the image base, in one multiply-add of the low 16
// bits (v_mad_u32_u16).
__device__ __forceinline__ uint32_t rec_addr(uint32_t rec, uint32_t base) {
    uint32_t a;
    asm("v_mad_u32_u16 %0, %1, 4, %2" : "=v"(a) : "v"(rec), "v"(base));
    return a;
}

constexpr int kPairs = 2;                  // 32-bit LDS reads per record

// The LDS reads of one unit of a lane's records (4 steps): the two pairs of
// each record (win dwords apart), issued without waiting; the address uses
// only a record's low 16 bits.
template <int WIN>
__device__ __forceinline__ void read_unit(const u32x4 R, uint32_t base, int win,
                                          uint32_t (&v)[kUnitSteps * kPairs]) {
#pragma unroll
    for (int u = 0; u < kUnitSteps; ++u) {
        lds_u32* p = reinterpret_cast<lds_u32*>(static_cast<uintptr_t>(rec_addr(R[u], base)));
        v[u * kPairs] = p[0];
        v[u * kPairs + 1] = p[WIN ? WIN : win];
    }
}

// The multiply-adds of one unit: acc[0], acc[2] from the first pair's low
// and high halves, acc[1], acc[3] from the second's.
__device__ __forceinline__ void fma_unit(const u32x4 R, const uint32_t (&v)[kUnitSteps * kPairs],
                                         float (&acc)[kShifts]) {
#pragma unroll
    for (int u = 0; u < kUnitSteps; ++u) {
        const float w = h2f(R[u] >> 16);
        acc[0] = fmaf(w, h2f(v[u * kPairs]), acc[0]);
        acc[2] = fmaf(w, h2f(v[u * kPairs] >> 16), acc[2]);
        acc[1] = fmaf(w, h2f(v[u * kPairs + 1]), acc[1]);
        acc[3] = fmaf(w, h2f(v[u * kPairs + 1] >> 16), acc[3]);
    }
}

// WIN > 0: win as a constant (the second read's offset becomes an
// immediate of the LDS instruction); 0: taken from win. Image rows are Lrow
// (= 2 win + 1) dwords, place r holding compact row rowat[r]; wlen is the
// width of the window maxima.
template <int NW, int WIN>
__global__ void __launch_bounds__(NW * 64, (NW == 16 && WIN) ? 8 : 1)
bound_kernel(const float* __restrict__ polar, const double* __restrict__ norms, int Rs, int n,
             const int* __restrict__ rows, const int* __restrict__ rowat, int n_rows, int Lrow,
             int win, int wlen, int scr_stride,
             const u32x4* __restrict__ recs, int rec_bytes, const int* __restrict__ chunk_end,
             const int4* __restrict__ slot_end, const int* __restrict__ part, int n_cs,
             float dfac, float* __restrict__ Qc,
             float* __restrict__ lane_q, int32_t* __restrict__ lane_c) {
    extern __shared__ uint16_t m16[];        // window image: pairs of halves
    __shared__ float red[NW];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = tmlib::uniform(threadIdx.x >> 6);
    const float* src = polar + static_cast<size_t>(b) * Rs * n;
    float* qrow = Qc + static_cast<size_t>(b) * n_cs;
    const double pn = norms[b];
    // a non-finite norm: the exact scorer flags the pattern; bounds 0
    if ((__double_as_longlong(pn) & 0x7ff0000000000000LL) == 0x7ff0000000000000LL) {
        for (int i = threadIdx.x; i < n_cs; i += NW * 64) qrow[i] = 0.0f;
        if (lane_q) {
            lane_q[static_cast<size_t>(b) * NW * 64 + threadIdx.x] = -INFINITY;
            lane_c[static_cast<size_t>(b) * NW * 64 + threadIdx.x] = -1;
        }
        return;
    }
    // 1. A = max |P| over the touched rows, and the image scale; a lane
    // loads columns lane + 64 i of 4 rows at once (coalesced, in flight
    // together)
    constexpr int MC = WIN == 90 ? 6 : kMaxCols;  // bound on o = ceil(n / 64)
    float a = 0.0f;
    for (int r0 = wave; r0 < n_rows; r0 += 4 * NW) {
        float v[4][MC];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = min(r0 + k * NW, n_rows - 1);
            const float* row = src + static_cast<size_t>(rows ? rows[r] : r) * n;
#pragma unroll
            for (int i = 0; i < MC; ++i) {
                const int c = lane + 64 * i;
                v[k][i] = c < n ? row[c] : 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int i = 0; i < MC; ++i) a = fmaxf(a, fabsf(v[k][i]));
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
    // 2. window maxima. Rounding up to float16 is monotone, so the maximum
    // of the rounded values is the rounded maximum: each row goes once, as
    // clamped (at 0), scaled, rounded-up float16 bits, into the wave's row
    // buffer rb of n + H columns (the first H = wlen + o again past n), and
    // its maxima over aligned blocks of o columns into bm; non-negative
    // float16 bits order like their values. Lane l then takes the o
    // consecutive columns x0 = o l .. x0 + o - 1: the part every window
    // shares (column x0 + o - 1, q whole blocks, r more columns), then the
    // head's suffix maxima and the tail's prefix maxima. Column x is the low
    // half of Y[x] (if x < Lrow) and the high half of Y[c], c + 2 win = x
    // (mod n), if c < Lrow (Lrow = 2 win <= n: at most one of each). The
    // next row's loads are issued before the current row is processed; the
    // buffers are the wave's own (wave-level ordering only).
    const int o = (n + 63) / 64;                 // columns per lane (<= MC)
    const int H = wlen + o;
    const int nb = (n + H) / o;                  // whole blocks in rb
    const int q = (wlen - o) / o, rq = wlen - o - q * o;
    constexpr int PW = NW < kBuildWaves ? NW : kBuildWaves;   // waves that build rows
    uint16_t* rb = m16 + static_cast<size_t>(n_rows + 1) * Lrow * 2 +
                   static_cast<size_t>(wave) * scr_stride;
    uint16_t* bm = rb + n + H;
    // image row place r holds compact row rowat[r]
    auto load_row = [&](int r, float (&v)[MC]) {
        const int cr = rowat[r];
        const float* row = src + static_cast<size_t>(rows ? rows[cr] : cr) * n;
#pragma unroll
        for (int i = 0; i < MC; ++i) {
            const int c = lane + 64 * i;
            v[i] = c < n ? row[c] : 0.0f;
        }
    };
    float nv[MC];
    if (wave < PW && wave < n_rows) load_row(wave, nv);
    for (int r = wave < PW ? wave : n_rows; r < n_rows; r += PW) {
        float v[MC];
#pragma unroll
        for (int i = 0; i < MC; ++i) v[i] = nv[i];
        if (r + PW < n_rows) load_row(r + PW, nv);
#pragma unroll
        for (int i = 0; i < MC; ++i) {
            const int c = lane + 64 * i;
            if (c < n) {
                const uint16_t h = f16_up(fmaxf(v[i], 0.0f) * scale);
                rb[c] = h;
                if (c < H) rb[n + c] = h;
            }
        }
        tmlib::wave_sync();
        for (int bk = lane; bk < nb; bk += 64) {
            uint32_t m = 0;
            for (int d = 0; d < o; ++d) m = max(m, static_cast<uint32_t>(rb[bk * o + d]));
            bm[bk] = static_cast<uint16_t>(m);
        }
        tmlib::wave_sync();
        uint16_t* dst = m16 + static_cast<size_t>(r) * Lrow * 2;
        const int x0 = o * lane;
        if (x0 < n) {
            uint32_t hv[MC], tv[MC];
#pragma unroll
            for (int d = 0; d < MC; ++d) {
                hv[d] = rb[x0 + min(d, o - 1)];                      // columns x0 .. x0 + o - 1
                tv[d] = rb[x0 + wlen - 1 + min(max(d, 1), o - 1)];   // x0 + wlen .. x0 + wlen + o - 2
            }
            uint32_t common = hv[MC - 1];               // column x0 + o - 1
            for (int k = 1; k <= q; ++k) common = max(common, static_cast<uint32_t>(bm[lane + k]));
            for (int k = 0; k < rq; ++k)
                common = max(common, static_cast<uint32_t>(rb[x0 + o * (q + 1) + k]));
            uint32_t out[MC];
            uint32_t hmax = common, tmax = common;
#pragma unroll
            for (int d = MC - 1; d >= 0; --d) {
                if (d < o - 1) hmax = max(hmax, hv[d]);
                out[d] = hmax;
            }
#pragma unroll
            for (int d = 1; d < MC; ++d) {
                if (d < o) tmax = max(tmax, tv[d]);
                out[d] = max(out[d], tmax);
            }
#pragma unroll
            for (int d = 0; d < MC; ++d) {
                const int x = x0 + d;
                if (d < o && x < n) {
                    const uint16_t h = static_cast<uint16_t>(out[d]);
                    if (x < Lrow) dst[2 * x] = h;
                    const int c = x - 2 * win + (x < 2 * win ? n : 0);
                    if (c < Lrow) dst[2 * c + 1] = h;
                }
            }
        }
        tmlib::wave_sync();                     // rb and bm are rewritten next
    }
    __syncthreads();
    // the extra row n_rows: A scaled, rounded up (the margin records' value)
    {
        const uint16_t h = f16_up(A * scale);
        uint16_t* dst = m16 + static_cast<size_t>(n_rows) * Lrow * 2;
        for (int x = threadIdx.x; x < 2 * Lrow; x += NW * 64) dst[x] = h;
    }
    __syncthreads();
    // 3. bounds: per template Q^ = ((m out_scale) dfac) invP (1 + 2^-19), m
    // the largest of its 4 window sums (margin record included), out_scale
    // = 1 / (scale 2^10) a power of 2, invP = 1 / ||P|| rounded up (every
    // operand non-negative; the three roundings are more than restored by
    // the last factor)
    float invP = 0.0f;
    if (pn > 0.0) {
        const double ip = 1.0 / pn;
        invP = static_cast<float>(ip);
        if (static_cast<double>(invP) < ip) invP = nextafterf(invP, INFINITY);
    }
    const float out_scale = 1.0f / (scale * static_cast<float>(1 << kWeightExp));   // power of 2
    const uint32_t base = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_u16*)m16));
    // the wave's chunks [c_begin, c_end) hold about 1/NW of the units
    // each lane also keeps its largest bound and that bound's column (the
    // first of equal ones), optionally written out at the end
    const int c_begin = part[wave], c_end = part[wave + 1];
    float best_q = -INFINITY;
    int best_c = -1;
    if (c_begin < c_end) {
    const int u_begin = (c_begin == 0) ? 0 : chunk_end[c_begin - 1];
    const int u_end = chunk_end[c_end - 1];
    const int last = u_end - 1;
    // records through a buffer resource: lane offset in a register, unit
    // offset (1 KiB per unit) in a scalar, no per-load address arithmetic
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<u32x4*>(recs), 0, rec_bytes, 0x00020000);
    const int voff = lane * 16;
    auto ld = [&](int k) {
        return __builtin_bit_cast(
            u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, min(k, last) * 1024, 0));
    };
    int c = c_begin;
    float acc[kShifts];
#pragma unroll
    for (int S = 0; S < kShifts; ++S) acc[S] = 0.0f;
    // the last units of the current chunk's quarter slots (s0 the current
    // slot's, p its index), from lane c - cb of registers holding 64
    // chunks' entries; an empty slot ends where the one before it does
    int cb = c_begin;
    int4 vse = make_int4(0, 0, 0, 0);
    auto load_events = [&]() { vse = slot_end[min(cb + lane, c_end - 1)]; };
    int s0 = 0, s1 = 0, s2 = 0, s3 = 0, p = 0;
    auto chunk_events = [&]() {
        if (c - cb == 64) {
            cb = c;
            load_events();
        }
        const int i = c - cb;
        s0 = __builtin_amdgcn_readlane(vse.x, i) - 1;
        s1 = __builtin_amdgcn_readlane(vse.y, i) - 1;
        s2 = __builtin_amdgcn_readlane(vse.z, i) - 1;
        s3 = __builtin_amdgcn_readlane(vse.w, i) - 1;
        p = 0;
    };
    load_events();
    chunk_events();
    // consume unit uu whose reads are in v: multiply-adds; after each
    // quarter slot but the last the accumulators rotate by one (the value of
    // shift S moves from acc[S + q] to acc[S + q + 1], mod 4); at the chunk's
    // end its bounds (one coalesced store) and fresh accumulators
    auto consume = [&](const u32x4 R, const uint32_t (&v)[kUnitSteps * kPairs], int uu) {
        fma_unit(R, v, acc);
        if (uu == s0) {
            do {
                if (p == kShifts - 1) {
                    float m = acc[0];
#pragma unroll
                    for (int S = 1; S < kShifts; ++S) m = fmaxf(m, acc[S]);
                    const float qv = ((m * out_scale) * dfac) * invP * (1.0f + 0x1p-19f);
                    qrow[static_cast<size_t>(c) * kLanes + lane] = qv;
                    if (qv > best_q) {
                        best_q = qv;
                        best_c = c * kLanes + lane;
                    }
                    ++c;
#pragma unroll
                    for (int S = 0; S < kShifts; ++S) acc[S] = 0.0f;
                    if (c < c_end) chunk_events();
                    break;
                }
                const float t = acc[3];
                acc[3] = acc[2];
                acc[2] = acc[1];
                acc[1] = acc[0];
                acc[0] = t;
                ++p;
                s0 = s1;
                s1 = s2;
                s2 = s3;
            } while (uu == s0);
        }
    };
    // Units stream through four registers g0..g3, each reloaded with the
    // unit 4 places on once consumed (loads past the last unit repeat it and
    // are not used). In the main loop the LDS reads of unit u + 1 are issued
    // before unit u is consumed, into the other of two value sets; the
    // pipeline fills and drains within each 8-unit iteration, so no read is
    // in flight across the loop's back edge.
    u32x4 g0 = ld(u_begin);
    u32x4 g1 = ld(u_begin + 1);
    u32x4 g2 = ld(u_begin + 2);
    u32x4 g3 = ld(u_begin + 3);
    uint32_t va[kUnitSteps * kPairs], vb[kUnitSteps * kPairs];
#define TM_BOUND_SB __builtin_amdgcn_sched_barrier(0)
    int u = u_begin;
    for (; u + 8 <= u_end; u += 8) {
        read_unit<WIN>(g0, base, win, va); TM_BOUND_SB;
        read_unit<WIN>(g1, base, win, vb); TM_BOUND_SB;
        consume(g0, va, u); g0 = ld(u + 4); TM_BOUND_SB;
        read_unit<WIN>(g2, base, win, va); TM_BOUND_SB;
        consume(g1, vb, u + 1); g1 = ld(u + 5); TM_BOUND_SB;
        read_unit<WIN>(g3, base, win, vb); TM_BOUND_SB;
        consume(g2, va, u + 2); g2 = ld(u + 6); TM_BOUND_SB;
        read_unit<WIN>(g0, base, win, va); TM_BOUND_SB;
        consume(g3, vb, u + 3); g3 = ld(u + 7); TM_BOUND_SB;
        read_unit<WIN>(g1, base, win, vb); TM_BOUND_SB;
        consume(g0, va, u + 4); g0 = ld(u + 8); TM_BOUND_SB;
        read_unit<WIN>(g2, base, win, va); TM_BOUND_SB;
        consume(g1, vb, u + 5); g1 = ld(u + 9); TM_BOUND_SB;
        read_unit<WIN>(g3, base, win, vb); TM_BOUND_SB;
        consume(g2, va, u + 6); g2 = ld(u + 10); TM_BOUND_SB;
        consume(g3, vb, u + 7); g3 = ld(u + 11); TM_BOUND_SB;
    }
    // the last 0..7 units, one at a time
    auto process = [&](u32x4 R, int uu) {
        read_unit<WIN>(R, base, win, va);
        consume(R, va, uu);
    };
    for (; u + 4 <= u_end; u += 4) {
        process(g0, u); g0 = ld(u + 4); TM_BOUND_SB;
        process(g1, u + 1); g1 = ld(u + 5); TM_BOUND_SB;
        process(g2, u + 2); g2 = ld(u + 6); TM_BOUND_SB;
        process(g3, u + 3); g3 = ld(u + 7); TM_BOUND_SB;
    }
#undef TM_BOUND_SB
    if (u < u_end) process(g0, u);
    if (u + 1 < u_end) process(g1, u + 1);
    if (u + 2 < u_end) process(g2, u + 2);
    }
    if (lane_q) {
        lane_q[static_cast<size_t>(b) * NW * 64 + threadIdx.x] = best_q;
        lane_c[static_cast<size_t>(b) * NW * 64 + threadIdx.x] = best_c;
    }
}

// Bounds from chunk-slot order to template order.
__global__ void __launch_bounds__(256)
bound_permute(const float* __restrict__ Qc, const int* __restrict__ tid, int n_cs, int Tp,
              float* __restrict__ Qt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= n_cs) return;
    const int t = tid[i];
    if (t >= 0) Qt[static_cast<size_t>(b) * Tp + t] = Qc[static_cast<size_t>(b) * n_cs + i];
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
    // (n_theta >= 16, so that 2 win <= n_theta)
    if (n < 16) return TM_OK;
    const int win = (n + kShifts - 1) / kShifts;
    // window image rows of 2 win dwords (pairs of float16 window maxima),
    // read at r and r + win, plus one unused dword: an odd pitch, so that a
    // row's place in the image sets the LDS bank of its column 0 to any of
    // the 32 (rows are placed below to even out the banks)
    const int Lrow = 2 * win + 1;
    // rows: the touched ones, then one holding A (the margin records' value)
    const size_t dwords = static_cast<size_t>(L->n_rows + 1) * Lrow;
    if (dwords * 4 > kLdsBudget || dwords > 65536) return TM_OK;   // window image too large
    // with the row buffers of the waves that build it, the workgroup's LDS
    // must fit the device's
    {
        int dev = 0, max_lds = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return TM_OK;
        if (dwords * 4 + kBuildWaves * 2 * scratch_halves(n, win) > static_cast<size_t>(max_lds))
            return TM_OK;
    }
    const uint32_t a_row = static_cast<uint32_t>(L->n_rows) * Lrow;

    // per template and quarter-turn q = k / win: records (dword offset of
    // column k - q win, float16 weight); the margin record joins the
    // smallest quarter; the lane's order of quarters is the rotation
    // (starting quarter o, then o + 1, ... mod 4) that puts the most
    // records first (ties: the largest count vector)
    std::vector<std::array<std::vector<uint32_t>, kShifts>> tr(Tp);
    std::vector<std::array<int32_t, kShifts>> qc(Tp);
    int nmax = 0;
    for (int32_t tt = 0; tt < Tp; ++tt) {
        const int32_t t = tt < T ? tt : tt - T;
        const bool is_mirror = tt >= T;
        const double nrm = L->tnorm[t];
        double wsum = 0.0;
        std::array<std::vector<uint32_t>, kShifts> qv;
        for (const HostPixel& p : pix[t]) {
            const int k = is_mirror ? (n - p.k) % n : p.k;
            const int q = k / win;
            const float w32 = nrm > 0.0 ? static_cast<float>(p.w / nrm) : 0.0f;
            wsum += w32;
            // (compact row) * Lrow + column for now; rows move to their
            // places in the image below
            const uint32_t off = static_cast<uint32_t>(row_index[p.j]) * Lrow +
                                 static_cast<uint32_t>(k - q * win);
            const uint32_t w16 = half_up(std::ldexp(w32, kWeightExp));
            qv[q].push_back(off | (w16 << 16));
        }
        const int cnt = static_cast<int>(pix[t].size());
        nmax = std::max(nmax, cnt);
        // the margin record: weight c_t 2^10 (rounded up), value A (one
        // place for all: a broadcast read)
        const double cf = gamma32(cnt) * wsum * (1.0 + 0x1p-20);
        const uint32_t c16 = half_up(static_cast<float>(std::ldexp(cf, kWeightExp) * (1.0 + 0x1p-20)));
        int qs = 0;
        for (int q = 1; q < kShifts; ++q)
            if (qv[q].size() < qv[qs].size()) qs = q;
        qv[qs].push_back(a_row | (c16 << 16));
        std::array<int32_t, kShifts> best{};
        int bo = 0;
        for (int o = 0; o < kShifts; ++o) {
            std::array<int32_t, kShifts> v;
            for (int p = 0; p < kShifts; ++p) v[p] = static_cast<int32_t>(qv[(o + p) % kShifts].size());
            if (o == 0 || v > best) { best = v; bo = o; }
        }
        for (int p = 0; p < kShifts; ++p) tr[tt][p] = std::move(qv[(bo + p) % kShifts]);
        qc[tt] = best;
    }
    // chunks of 64 templates of similar slot sizes: ordered by the slot
    // sizes in whole units first (a chunk pays each slot's largest, rounded
    // up to whole units), then by the sizes themselves
    std::vector<int32_t> order(Tp);
    std::iota(order.begin(), order.end(), 0);
    auto units_of = [](const std::array<int32_t, kShifts>& v) {
        std::array<int32_t, kShifts> u;
        for (int p = 0; p < kShifts; ++p) u[p] = (v[p] + kUnitSteps - 1) / kUnitSteps;
        return u;
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const auto ua = units_of(qc[a]), ub = units_of(qc[b]);
        return ua != ub ? ua > ub : qc[a] > qc[b];
    });
    const int32_t n_chunks = (Tp + kLanes - 1) / kLanes;
    std::vector<int32_t> tid(static_cast<size_t>(n_chunks) * kLanes, -1);
    for (int32_t i = 0; i < n_chunks * kLanes; ++i) tid[i] = i < Tp ? order[i] : -1;
    // Row places. The pixels of one (chunk, slot, half-wave) are read in
    // its steps, one per lane and step; their columns' banks, (place * Lrow
    // + r) mod 32, should be spread evenly. Rows are placed in decreasing
    // order of pixel count, each at the free place whose bank shift meets
    // the least load already placed in the groups where the row has pixels
    // (sum of products of the two bank histograms).
    const int n_rows = L->n_rows;
    std::vector<int32_t> rowat(n_rows), place(n_rows, -1);
    {
        const int n_groups = n_chunks * kShifts * 2;
        std::vector<std::vector<std::pair<int, std::array<uint16_t, kBanks>>>> hist(n_rows);
        std::vector<int64_t> rowcnt(n_rows, 0);
        std::vector<std::array<uint16_t, kBanks>> acc(n_rows);
        std::vector<int> touched;
        for (int32_t c = 0; c < n_chunks; ++c)
            for (int p = 0; p < kShifts; ++p)
                for (int h = 0; h < 2; ++h) {
                    const int g = (c * kShifts + p) * 2 + h;
                    touched.clear();
                    for (int l = h * 32; l < h * 32 + 32; ++l) {
                        const int32_t t = tid[c * kLanes + l];
                        if (t < 0) continue;
                        for (uint32_t rec : tr[t][p]) {
                            const uint32_t off = rec & 0xffffu;
                            if (off == a_row) continue;
                            const int row = static_cast<int>(off / Lrow);
                            bool seen = false;
                            for (int x : touched) seen |= (x == row);
                            if (!seen) { touched.push_back(row); acc[row].fill(0); }
                            ++acc[row][(off % Lrow) % kBanks];
                            ++rowcnt[row];
                        }
                    }
                    for (int row : touched) hist[row].push_back({g, acc[row]});
                }
        std::vector<int32_t> byc(n_rows);
        std::iota(byc.begin(), byc.end(), 0);
        std::stable_sort(byc.begin(), byc.end(), [&](int a, int b) { return rowcnt[a] > rowcnt[b]; });
        std::vector<std::array<int32_t, kBanks>> load(n_groups);
        for (auto& a : load) a.fill(0);
        std::vector<char> used(n_rows, 0);
        for (int row : byc) {
            // one free place per bank shift
            int cand[kBanks];
            std::fill(cand, cand + kBanks, -1);
            for (int pl = 0; pl < n_rows; ++pl)
                if (!used[pl]) {
                    const int s = static_cast<int>((static_cast<int64_t>(pl) * Lrow) % kBanks);
                    if (cand[s] < 0) cand[s] = pl;
                }
            int64_t best = -1;
            int bs = 0;
            for (int s = 0; s < kBanks; ++s) {
                if (cand[s] < 0) continue;
                int64_t cost = 0;
                for (const auto& [g, hb] : hist[row])
                    for (int b = 0; b < kBanks; ++b)
                        if (hb[b]) cost += static_cast<int64_t>(hb[b]) * load[g][(b + s) % kBanks];
                if (best < 0 || cost < best) { best = cost; bs = s; }
            }
            place[row] = cand[bs];
            used[cand[bs]] = 1;
            rowat[cand[bs]] = row;
            for (const auto& [g, hb] : hist[row])
                for (int b = 0; b < kBanks; ++b) load[g][(b + bs) % kBanks] += hb[b];
        }
        // records to image offsets
        for (int32_t tt = 0; tt < Tp; ++tt)
            for (int p = 0; p < kShifts; ++p)
                for (uint32_t& rec : tr[tt][p]) {
                    const uint32_t off = rec & 0xffffu;
                    if (off == a_row) continue;
                    const uint32_t row = off / Lrow, col = off % Lrow;
                    rec = (rec & 0xffff0000u) | (static_cast<uint32_t>(place[row]) * Lrow + col);
                }
    }
    std::vector<int32_t> cend(n_chunks, 0), send(static_cast<size_t>(n_chunks) * 4, 0);
    std::vector<uint32_t> recs;
    // LDS bank model of the pair reads: kBanks banks of 4 bytes, lanes
    // grouped in half-waves; the dword of a record's read r
    const int nbanks = kBanks, group = kLanes / 2;
    auto dword = [&](uint32_t rec, int r) { return (rec & 0xffffu) + r * static_cast<uint32_t>(win); };
    auto whole = [](int m) { return (m + kUnitSteps - 1) / kUnitSteps * kUnitSteps; };
    for (int32_t c = 0; c < n_chunks; ++c) {
        int mh[kShifts] = {0, 0, 0, 0};
        for (int l = 0; l < kLanes; ++l) {
            const int32_t idx = c * kLanes + l;
            if (tid[idx] >= 0)
                for (int p = 0; p < kShifts; ++p) mh[p] = std::max(mh[p], qc[tid[idx]][p]);
        }
        // whole units per slot; the first slot holds every template's
        // largest quarter (at least the margin record); later ones may be
        // empty
        int sb[kShifts + 1] = {0};
        for (int p = 0; p < kShifts; ++p)
            sb[p + 1] = sb[p] + (p == 0 ? std::max(kUnitSteps, whole(mh[0])) : whole(mh[p]));
        const int m = sb[kShifts];
        std::vector<uint32_t> step(static_cast<size_t>(m) * kLanes, 0u);
        for (int p = 0; p < kShifts; ++p) {
            // per step one record per lane, chosen so that the lanes of each
            // half-wave read distinct banks where possible (a template's
            // records may come in any order within a slot: the bound's sum
            // and its margin do not depend on it); padding (weight 0) reads
            // a free bank of row 0
            std::vector<std::vector<uint32_t>> left(kLanes);
            for (int l = 0; l < kLanes; ++l)
                if (tid[c * kLanes + l] >= 0) left[l] = tr[tid[c * kLanes + l]][p];
            for (int i = sb[p]; i < sb[p + 1]; ++i) {
                // per read and bank: the first dword read there and the
                // number of distinct dwords (a second lane on the same dword
                // is free)
                std::vector<uint32_t> first(static_cast<size_t>(kPairs) * nbanks);
                std::vector<uint8_t> ndist(static_cast<size_t>(kPairs) * nbanks);
                for (int l = 0; l < kLanes; ++l) {
                    if (l % group == 0) std::fill(ndist.begin(), ndist.end(), 0);
                    auto cost = [&](uint32_t rec) {
                        int k = 0;
                        for (int r = 0; r < kPairs; ++r) {
                            const uint32_t d = dword(rec, r);
                            const size_t ix = static_cast<size_t>(r) * nbanks + d % nbanks;
                            if (ndist[ix] && first[ix] != d) k += ndist[ix];
                        }
                        return k;
                    };
                    auto take = [&](uint32_t rec) {
                        for (int r = 0; r < kPairs; ++r) {
                            const uint32_t d = dword(rec, r);
                            const size_t ix = static_cast<size_t>(r) * nbanks + d % nbanks;
                            if (!ndist[ix]) { first[ix] = d; ndist[ix] = 1; }
                            else if (first[ix] != d && ndist[ix] < 255) ++ndist[ix];
                        }
                        step[static_cast<size_t>(i) * kLanes + l] = rec;
                    };
                    auto& L_ = left[l];
                    if (L_.empty()) {
                        uint32_t pad = 0;
                        int best_c = 99;
                        for (uint32_t x = 0; x < 64 && x < static_cast<uint32_t>(win); ++x) {
                            const int k = cost(x);
                            if (k < best_c) { best_c = k; pad = x; }
                            if (k == 0) break;
                        }
                        take(pad);
                        continue;
                    }
                    size_t best = 0;
                    int best_c = 99;
                    const size_t lim = std::min<size_t>(L_.size(), kChoices);
                    for (size_t e = 0; e < lim && best_c > 0; ++e) {
                        const int k = cost(L_[e]);
                        if (k < best_c) { best_c = k; best = e; }
                    }
                    take(L_[best]);
                    L_.erase(L_.begin() + static_cast<long>(best));
                }
            }
        }
        // the first unit after each slot (the last one: after the chunk)
        const int32_t u0 = static_cast<int32_t>(recs.size() / (kUnitSteps * kLanes));
        for (int p = 0; p < kShifts; ++p) send[static_cast<size_t>(c) * 4 + p] = u0 + sb[p + 1] / kUnitSteps;
        for (int q = 0; q < m; q += kUnitSteps)
            for (int l = 0; l < kLanes; ++l)
                for (int i = q; i < q + kUnitSteps; ++i)
                    recs.push_back(step[static_cast<size_t>(i) * kLanes + l]);
        // (1 KiB per unit, addressed with 32-bit offsets)
        const int64_t units = static_cast<int64_t>(recs.size() / (kUnitSteps * kLanes));
        if (units >= INT32_MAX / 1024) return TM_OK;
        cend[c] = static_cast<int32_t>(units);
    }
    // chunk ranges of the waves of an 8-wave and a 16-wave workgroup, each
    // about 1/NW of the units (chunks are contiguous per wave)
    std::vector<int32_t> part;
    const int64_t units = n_chunks ? cend[n_chunks - 1] : 0;
    for (int nw : {8, 16}) {
        for (int w = 0; w <= nw; ++w) {
            const int64_t target = units * w / nw;
            int32_t c = 0;
            while (c < n_chunks && (c == 0 ? 0 : cend[c - 1]) < target) ++c;
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
    if (int r = up(&L->d_bnd_slots, send)) return r;
    if (int r = up(&L->d_bnd_rowat, rowat)) return r;
    if (int r = up(&L->d_bnd_tid, tid)) return r;
    L->bnd_tid = tid;
    if (int r = up(&L->d_bnd_part, part)) return r;
    L->bnd_win = win;
    L->bnd_shifts = kShifts;
    L->bnd_L = Lrow;
    L->bnd_chunks = n_chunks;
    L->bnd_units = units;
    L->bnd_dfac = static_cast<float>(1.0 / (1.0 - gamma32(nmax + 1)) * (1.0 + 0x1p-22));
    L->bound = true;
    return TM_OK;
}

void tmlib::bound_release(tm_library* L) {
    (void)hipFree(L->d_bnd_recs);
    (void)hipFree(L->d_bnd_end);
    (void)hipFree(L->d_bnd_slots);
    (void)hipFree(L->d_bnd_rowat);
    (void)hipFree(L->d_bnd_tid);
    (void)hipFree(L->d_bnd_part);
    L->d_bnd_recs = nullptr;
    L->d_bnd_end = nullptr;
    L->d_bnd_slots = nullptr;
    L->d_bnd_rowat = nullptr;
    L->d_bnd_tid = nullptr;
    L->d_bnd_part = nullptr;
    L->bound = false;
}

// ------------------------------------------------------------ launches

int tmlib::bound_scores_impl(const tm_library* L, const float* polar, const double* norms,
                             int32_t B, float* out, bool template_order, bool compact,
                             hipStream_t s, float* lane_q, int32_t* lane_c, int* n_list) {
    const size_t image = static_cast<size_t>(L->n_rows + 1) * L->bnd_L * sizeof(uint32_t);
    // window maxima over win + 4 win - n columns (see the header), at most a row
    const int n = L->n_theta, win = L->bnd_win;
    const int wlen = std::min(5 * win - n, n);
    const size_t scr = scratch_halves(n, win);
    const int Rs = compact ? L->n_rows : L->R;
    const int* rows = compact ? nullptr : L->d_rows;
    const int n_cs = L->bnd_chunks * kLanes;
    float* Qc = out;
    if (template_order)
        TM_HIP(hipMallocAsync(reinterpret_cast<void**>(&Qc),
                              std::max<size_t>(static_cast<size_t>(B) * n_cs, 1) * sizeof(float), s));
    auto launch = [&](auto kern, int nw) -> int {
        const size_t lds = image + std::min(nw, kBuildWaves) * scr * sizeof(uint16_t);
        TM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
        hipLaunchKernelGGL(kern, dim3(B), dim3(nw * 64), lds, s, polar, norms, Rs, L->n_theta, rows,
                           L->d_bnd_rowat, L->n_rows, L->bnd_L, win, wlen, static_cast<int>(scr),
                           reinterpret_cast<const u32x4*>(L->d_bnd_recs),
                           static_cast<int>(L->bnd_units * 1024), L->d_bnd_end,
                           reinterpret_cast<const int4*>(L->d_bnd_slots),
                           L->d_bnd_part + (nw == 8 ? 0 : 9), n_cs, L->bnd_dfac, Qc, lane_q,
                           lane_c);
        if (n_list) *n_list = nw * 64;
        TM_HIP(hipGetLastError());
        return TM_OK;
    };
    // one workgroup per CU when the image fills the LDS: use every wave slot
    const bool whole = image > 64 * 1024;
    // n_theta = 360 (windows of 90 columns) has its own instance
    int r;
    if (L->bnd_win == 90)
        r = whole ? launch(bound_kernel<16, 90>, 16) : launch(bound_kernel<8, 90>, 8);
    else
        r = whole ? launch(bound_kernel<16, 0>, 16) : launch(bound_kernel<8, 0>, 8);
    if (template_order) {
        if (!r) {
            hipLaunchKernelGGL(bound_permute, dim3((n_cs + 255) / 256, B), dim3(256), 0, s, Qc,
                               L->d_bnd_tid, n_cs, L->Tp, out);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) r = tmlib::hip_fail(e, "bound_permute launch");
        }
        hipError_t e = hipFreeAsync(Qc, s);
        if (!r && e != hipSuccess) r = tmlib::hip_fail(e, "hipFreeAsync");
    }
    return r;
}

int tmlib::bound_match(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                       int32_t N, double cap_frac, int32_t* n_rescored, int32_t* top_template,
                       int32_t* top_angle, float* top_score, bool compact, hipStream_t s) {
    const int Tp = lib->Tp;
    const int n_cs = lib->bnd_chunks * kLanes;
    float* Qc = nullptr;
    float* lq = nullptr;
    int32_t* lc = nullptr;
    TM_HIP(hipMallocAsync(reinterpret_cast<void**>(&Qc), static_cast<size_t>(B) * n_cs * sizeof(float), s));
    int r = TM_OK;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&lq), static_cast<size_t>(B) * 1024 * sizeof(float), s);
    if (e == hipSuccess)
        e = hipMallocAsync(reinterpret_cast<void**>(&lc), static_cast<size_t>(B) * 1024 * sizeof(int32_t), s);
    if (e != hipSuccess) r = tmlib::hip_fail(e, "hipMallocAsync");
    int n_list = 0;
    if (!r) r = bound_scores_impl(lib, polar, norms, B, Qc, false, compact, s, lq, lc, &n_list);
    const double frac = cap_frac > 0.0 ? cap_frac : 0.1;
    int32_t cap = static_cast<int32_t>(std::ceil(frac * Tp - 1e-9));
    cap = std::max(N, std::min(cap, Tp));
    // the bound ranks templates less sharply than the exact score: the 48
    // best of the lanes' largest bounds (at most one per lane) are scored
    // exactly first, so that the threshold starts high
    if (!r) r = tmlib::certified_rescore(lib, polar, norms, B, N, std::max(N, kFirst), Qc, n_cs,
                                         lib->d_bnd_tid, 0.0, cap, n_rescored, top_template,
                                         top_angle, top_score, compact, s, lq, lc, n_list);
    for (void* p : {static_cast<void*>(lq), static_cast<void*>(lc), static_cast<void*>(Qc)}) {
        if (!p) continue;
        e = hipFreeAsync(p, s);
        if (!r && e != hipSuccess) r = tmlib::hip_fail(e, "hipFreeAsync");
    }
    return r;
}

// --------------------------------------------------------------- C ABI

namespace {

int bound_scores_entry(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                       int32_t compact_rows, float* bound_out, bool template_order,
                       int32_t* slot_template, void* hip_stream) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (compact_rows != 0 && compact_rows != 1) { tmlib::set_error("compact_rows=%d must be 0 or 1", compact_rows); return TM_EINVAL; }
    if (!lib->bound) {
        tmlib::set_error("window bounds need non-negative template weights and a window image "
                         "within the LDS budget");
        return TM_EUNSUPPORTED;
    }
    if (slot_template) std::copy(lib->bnd_tid.begin(), lib->bnd_tid.end(), slot_template);
    if (B == 0) return TM_OK;
    if (!polar || !norms || !bound_out) {
        tmlib::set_error("polar, norms and bound_out must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    return tmlib::bound_scores_impl(lib, polar, norms, B, bound_out, template_order,
                                    compact_rows == 1, static_cast<hipStream_t>(hip_stream));
}

}  // namespace

extern "C" int tm_bound_scores(const tm_library* lib, const float* polar, const double* norms,
                               int32_t B, int32_t compact_rows, float* bound_out,
                               void* hip_stream) {
    return bound_scores_entry(lib, polar, norms, B, compact_rows, bound_out, true, nullptr,
                              hip_stream);
}

extern "C" int tm_bound_scores_slots(const tm_library* lib, const float* polar,
                                     const double* norms, int32_t B, int32_t compact_rows,
                                     float* bound_out, int32_t* slot_template,
                                     void* hip_stream) {
    return bound_scores_entry(lib, polar, norms, B, compact_rows, bound_out, false,
                              slot_template, hip_stream);
}

extern "C" int tm_bound_layout(const tm_library* lib, int32_t* chunks, int64_t* units,
                               int32_t* win) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (!lib->bound) {
        tmlib::set_error("this library has no window bounds");
        return TM_EUNSUPPORTED;
    }
    if (chunks) *chunks = lib->bnd_chunks;
    if (units) *units = lib->bnd_units;
    if (win) *win = lib->bnd_win;
    return TM_OK;
}
