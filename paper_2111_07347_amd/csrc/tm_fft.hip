// Fourier route of the in-plane search (Section 2.2, computational cost): the
// azimuthal sliding of a template over the polar image is a circular
// cross-correlation along theta, so per pattern and template
//
//   C(k)  = sum_j conj(T^[j, k]) P^[j, k]        (k = 0 .. n/2, n = n_theta)
//   Q(s)  = (1/n) sum_k c_k Re(C(k) e^{2 pi i k s / n}),  c_k = 1 at k = 0, n/2
//
// with T^, P^ the spectra along theta of the normalised template image and
// polar rows. The mirror of a template has spectrum conj(T^), so both come
// out of one product: with T^ = a + ib and P^ = c + id,
//   C_base   = (ac + bd) + i(ad - bc),   C_mirror = (ac - bd) + i(ad + bc).
//
// Kernels (float16 operands on the matrix cores, float32 accumulation):
//   fft_patterns  P^ of a chunk of patterns, float64 DFT, stored float16 x 2^8
//                 as [k][2 b + (re|im)][j] (rows j contiguous: matrix operand)
//   fft_forward   per frequency a [2T x R] x [R x 2B] product giving ac, bc,
//                 ad, bd; neighbouring lanes exchange halves and form C_base
//                 (even lanes) and C_mirror (odd lanes); C(k) stored float16
//                 x 2^sc, four frequencies of one parity per 16-byte record:
//                 [parity][chunk][t'][b][re, im x 4]
//   fft_inverse   the inverse transform as a product with cosine / sine tables
//                 held in LDS, split by frequency parity: with A(s) the even
//                 and B(s) the odd frequencies' sums, Q(s) = A + B and
//                 Q(s + n/2) = A - B for s < n/2, so max(Q(s), Q(s + n/2)) =
//                 A + |B|. Only the per-template maximum and its shift leave
//                 the chip.
// The certified rescoring that follows (tm_certify.hip) scores exactly every
// template whose approximate score could still reach the N-th best exact
// score within the error bound.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "tm_device.h"
#include "tm_internal.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int kScaleT = 8;     // template spectra x 2^8 before float16 rounding
constexpr int kScaleP = 8;     // pattern spectra x 2^8
constexpr int kScaleW = 12;    // inverse cosine / sine tables x 2^12
constexpr int kDftRows = 8;    // polar rows per fft_patterns workgroup (one 16-byte store)
constexpr int kFwdWaves = 8;   // fft_forward: 2 row blocks x 4 column blocks of 32
constexpr int kInvWaves = 12;  // fft_inverse: 6 pair tiles x 2 halves of the shifts
constexpr int kInvTiles = kInvWaves / 2;
constexpr int kInvMaxBlocks = 3;                // 32-shift blocks per wave per part
constexpr size_t kInvLdsBudget = 160 * 1024 - 2048;
// Bytes of stored C(k) per chunk of patterns. Larger chunks bring nothing
// (64 patterns already fill the chip) and multi-GiB stream-ordered
// allocations made on several streams stalled the host for seconds.
constexpr double kChatBudget = 2.0 * 1024 * 1024 * 1024;

// ---------------------------------------------------------------- host side

// float64 -> float16 bits, round to nearest even (finite input).
uint16_t half_bits(double x) {
    uint64_t b;
    std::memcpy(&b, &x, 8);
    const uint16_t sign = static_cast<uint16_t>((b >> 48) & 0x8000u);
    b &= 0x7fffffffffffffffull;
    const int e = static_cast<int>(b >> 52);
    if (e == 0) return sign;                                  // zero or float64 subnormal
    const uint64_t m = (b & ((1ull << 52) - 1)) | (1ull << 52);   // value m * 2^(e - 1075)
    auto rne = [](uint64_t v, int sh) -> uint64_t {
        if (sh >= 64) return 0;
        const uint64_t q = v >> sh;
        const uint64_t rem = v & ((1ull << sh) - 1);
        const uint64_t halfv = 1ull << (sh - 1);
        return (rem > halfv || (rem == halfv && (q & 1))) ? q + 1 : q;
    };
    int E = e - 1008;                                         // float16 biased exponent
    if (E >= 1) {
        uint64_t q = rne(m, 42);                              // 11 significant bits
        if (q == 2048) { q = 1024; ++E; }
        if (E >= 31) return sign | 0x7c00u;
        return static_cast<uint16_t>(sign | (E << 10) | (q - 1024));
    }
    const uint64_t q = rne(m, 1051 - e);                      // units of 2^-24
    return static_cast<uint16_t>(sign | q);                   // q = 1024 is the smallest normal
}

double gamma32(double n) {
    const double u = std::ldexp(1.0, -24);
    return n * u / (1.0 - n * u);
}

// Worst case of |Q~ - Q32| over every template and shift: float16 rounding of
// both spectra (relative 2^-11, plus 2^-14 absolute in scaled units should
// subnormals be flushed), float32 accumulation over the R rows, float16
// storage of C(k), float16 tables and float32 accumulation in the inverse,
// the final addition and scaling, and the float32 direct path's own error.
// Per-element errors become a bound on Q through Cauchy-Schwarz and
// Parseval's identity: (1/n) ||X||_c ||Y||_c <= 1 for the exact normalised
// spectra, ||X||_c^2 = sum_j sum_k c_k |X[j, k]|^2.
double error_bound(int R, int Fp, int sc, int n_max) {
    const double u16 = std::ldexp(1.0, -11), u32 = std::ldexp(1.0, -24);
    const double tiny = std::ldexp(1.0, -14), r2 = std::sqrt(2.0), rr = std::sqrt(double(R));
    const double eT = tiny * std::ldexp(1.0, -kScaleT), eP = tiny * std::ldexp(1.0, -kScaleP);
    const double eC = tiny * std::ldexp(1.0, -sc), eW = tiny * std::ldexp(1.0, -kScaleW);
    const double aT = u16 + r2 * eT * rr;
    const double aP = u16 + 2.0 * u32 + r2 * eP * rr;   // float64 -> float32 -> float16
    const double e1 = aT + aP + aT * aP;
    const double rho2 = (1.0 + aT) * (1.0 + aP);
    const double gf = gamma32(R + 2);
    const double e2 = 2.0 * gf * rho2;
    const double m0 = (1.0 + 2.0 * gf) * rho2;
    const double e3 = u16 * m0 + r2 * eC;
    const double m = (1.0 + u16) * m0 + r2 * eC;
    const double gi = gamma32(Fp + 1);
    const double e4 = (u16 + r2 * eW) * m + gi * (1.0 + u16 + r2 * eW) * m;
    const double e5 = 3.0 * u32 * (m + e4);
    const double d32 = gamma32(n_max + 3);
    return e1 + e2 + e3 + e4 + e5 + d32 + 1e-9;
}

template <typename T>
int upload_vec(T** dst, const std::vector<T>& src, hipStream_t s, size_t& bytes) {
    *dst = nullptr;
    const size_t n = std::max<size_t>(src.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), n);
    if (e != hipSuccess) {
        *dst = nullptr;
        tmlib::set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
        return TM_ENOMEM;
    }
    bytes += n;
    if (!src.empty())
        TM_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return TM_OK;
}

int device_cus() {
    static int n = 0;
    if (!n) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) v = 256;
        n = v;
    }
    return n;
}

// -------------------------------------------------------------- device side

__device__ __forceinline__ float dpp_xor1(float v) {
    // quad_perm [1, 0, 3, 2]: each lane reads its neighbour lane ^ 1
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ uint32_t pack_half2(float lo, float hi) {
    const _Float16 a = static_cast<_Float16>(lo), b = static_cast<_Float16>(hi);
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, a)) |
           (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, b)) << 16);
}

// Pattern spectra of one chunk: workgroup (pattern bl, touched rows j0..j0+7), in
// float64 by one Cooley-Tukey split n = n1 * n2 (theta = n2 a + b,
// k = k1 + n1 k2, W(m) = e^{-2 pi i m / n}):
//   Z[k1][b] = W(k1 b) * sum_a x[n2 a + b] W(n2 a k1)      (n2 DFTs of length n1)
//   X[k]     = sum_b Z[k1][b] W(n1 b k2)                    (k < F only)
// then scaled by 2^8/||P|| and rounded to float16. Thread item of the second
// stage: one frequency for all 8 rows (one 16-byte store per half).
__global__ void __launch_bounds__(256)
fft_patterns(const float* __restrict__ polar, const double* __restrict__ norms,
             const int* __restrict__ rows, int Rs, int nr, int n_theta, int n1, int F, int Fp,
             int Rp, int nb_valid, int ld_cols, const double* __restrict__ dft,
             _Float16* __restrict__ Ph) {
    extern __shared__ double smem[];
    double* cs = smem;                                   // [n_theta][2] cos, sin
    double* zr = cs + 2 * n_theta;                       // [kDftRows][n_theta] re Z
    double* zi = zr + kDftRows * n_theta;                // [kDftRows][n_theta] im Z
    float* xs = reinterpret_cast<float*>(zi + kDftRows * n_theta);   // [kDftRows][n_theta]
    const int n2 = n_theta / n1;
    const int bl = blockIdx.x;
    const int j0 = blockIdx.y * kDftRows;
    const bool valid = bl < nb_valid;
    double scale = 0.0;
    if (valid) {
        const double pn = norms[bl];
        scale = pn > 0.0 ? 256.0 / pn : 0.0;
    }
    const bool live = scale != 0.0 && j0 < nr;
    if (live) {
        // spectrum row j (a touched row) reads polar row rows[j], or row j of
        // a compact polar image
        const float* src = polar + static_cast<size_t>(bl) * Rs * n_theta;
        for (int i = threadIdx.x; i < kDftRows * n_theta; i += 256) {
            const int r = i / n_theta, c = i - r * n_theta;
            const int j = j0 + r;
            xs[i] = j < nr ? src[static_cast<size_t>(rows ? rows[j] : j) * n_theta + c] : 0.0f;
        }
        for (int i = threadIdx.x; i < 2 * n_theta; i += 256) cs[i] = dft[i];
        __syncthreads();
        // first stage: item (row r, k1, b)
        for (int it = threadIdx.x; it < kDftRows * n_theta; it += 256) {
            const int r = it / n_theta, rem = it - r * n_theta;
            const int k1 = rem / n2, b = rem - k1 * n2;
            const float* x = xs + r * n_theta + b;
            double yr = 0.0, yi = 0.0;
            const int step = n2 * k1;                    // W(n2 a k1), a = 0, 1, ...
            int m = 0;
            for (int a = 0; a < n1; ++a) {
                const double v = x[n2 * a];
                yr = fma(v, cs[2 * m], yr);
                yi = fma(-v, cs[2 * m + 1], yi);
                m += step;
                if (m >= n_theta) m -= n_theta;
            }
            const int mt = (k1 * b) % n_theta;           // twiddle W(k1 b)
            const double c = cs[2 * mt], sn = -cs[2 * mt + 1];
            zr[it] = yr * c - yi * sn;
            zi[it] = yr * sn + yi * c;
        }
        __syncthreads();
    }
    // second stage: item k, all rows
    for (int k = threadIdx.x; k < Fp; k += 256) {
        double xr[kDftRows], xi[kDftRows];
#pragma unroll
        for (int r = 0; r < kDftRows; ++r) xr[r] = xi[r] = 0.0;
        if (live && k < F) {
            const int k1 = k % n1, k2 = k / n1;
            const int step = (n1 * k2) % n_theta;        // W(n1 b k2), b = 0, 1, ...
            int m = 0;
            for (int b = 0; b < n2; ++b) {
                const double c = cs[2 * m], sn = -cs[2 * m + 1];
#pragma unroll
                for (int r = 0; r < kDftRows; ++r) {
                    const double ar = zr[r * n_theta + k1 * n2 + b];
                    const double ai = zi[r * n_theta + k1 * n2 + b];
                    xr[r] = fma(ar, c, fma(-ai, sn, xr[r]));
                    xi[r] = fma(ar, sn, fma(ai, c, xi[r]));
                }
                m += step;
                if (m >= n_theta) m -= n_theta;
            }
        }
        f16x8_t vr, vi;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            vr[r] = static_cast<_Float16>(static_cast<float>(xr[r] * scale));
            vi[r] = static_cast<_Float16>(static_cast<float>(xi[r] * scale));
        }
        _Float16* dst = Ph + (static_cast<size_t>(k) * ld_cols + 2 * bl) * Rp + j0;
        *reinterpret_cast<f16x8_t*>(dst) = vr;
        *reinterpret_cast<f16x8_t*>(dst + Rp) = vi;
    }
}

// Split n = n1 * n2 with n1 the largest divisor not above sqrt(n).
int dft_split(int n) {
    int best = 1;
    for (int d = 1; d * d <= n; ++d)
        if (n % d == 0) best = d;
    return best;
}

// Linear workgroup id remapped so that consecutive ids on one XCD (hardware
// ids l, l + 8, l + 16, ...) get consecutive work items: workgroups sharing
// a template tile then share that XCD's L2.
__device__ __forceinline__ int xcd_item(int L, int n) {
    const int q = n / 8, r = n % 8, x = L % 8, slot = L / 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + slot;
}

// C(k) for a tile of 32 base templates x 64 patterns at the four frequencies
// of one record chunk (one parity). The grid runs chunk-major: all
// workgroups in flight share one chunk's pattern spectra (L2-resident), and
// the XCD remap keeps the workgroups of one template tile on one XCD.
// Per frequency, the workgroup stages the template tile (64 rows: 32
// templates x re/im) and the pattern tile (128 columns: 64 patterns x re/im)
// in LDS, in slabs of up to 128 rows j, with rows padded by 16 bytes so that
// the 16-byte fragment reads of 16 lanes hit distinct banks.
// Wave w: rows 32 * (w & 1) .. (16 templates x re/im), columns of the
// 32-column block 32 * (w >> 1) .. (16 patterns x re/im).
// MFMA 32x32x16 output: lane l holds column l % 32, rows 8 (v / 4) +
// 4 (l / 32) + v % 4, so a lane has both halves (a, b) of its templates and
// one half (c or d) of its pattern; lane l ^ 1 has the other half.
constexpr int kFwdSlab = 128;                  // rows j per LDS slab
constexpr int kFwdPitch = kFwdSlab + 8;        // halves per LDS row
constexpr int kFwdRows = 64 + 128;             // template rows + pattern columns

__global__ void __launch_bounds__(kFwdWaves * 64, 4)
fft_forward(const _Float16* __restrict__ Th, const _Float16* __restrict__ Ph,
            _Float16* __restrict__ Ch, int T, int Tp, int Tpad, int Rp, int Fp, int nbp,
            float resc) {
    __shared__ _Float16 tile[kFwdRows * kFwdPitch];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rb = wave & 1, cb0 = wave >> 1;
    const int n_pt = nbp / 64;
    const int group = n_pt * (Tpad / 32);
    const int kc = static_cast<int>(blockIdx.x) / group;          // record chunk: parity, q
    const int item = xcd_item(static_cast<int>(blockIdx.x) - kc * group, group);
    const int t0 = (item / n_pt) * 32, b0 = (item % n_pt) * 64;
    const int col = lane & 31, hi = lane >> 5;
    const bool odd = lane & 1;
    const int Q = Fp / 8;
    const int p = kc / Q, q = kc - p * Q;
    const size_t slabA = static_cast<size_t>(2) * Tpad * Rp;
    const size_t slabB = static_cast<size_t>(2) * nbp * Rp;
    const bool mirror = Tp > T;
    const _Float16* a_frag = tile + (rb * 32 + col) * kFwdPitch + 8 * hi;
    const _Float16* b_frag = tile + (64 + cb0 * 32 + col) * kFwdPitch + 8 * hi;
    uint32_t stage[8][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int k = p + 8 * q + 2 * e;
        const _Float16* A = Th + k * slabA + static_cast<size_t>(2 * t0) * Rp;
        const _Float16* X = Ph + k * slabB + static_cast<size_t>(2 * b0) * Rp;
        f32x16_t acc = {};
        for (int j0 = 0; j0 < Rp; j0 += kFwdSlab) {
            const int w = min(kFwdSlab, Rp - j0);              // multiple of 16
            const int vpr = w / 8;                               // 16-byte vectors per row
            __syncthreads();
            for (int i = threadIdx.x; i < kFwdRows * vpr; i += kFwdWaves * 64) {
                const int r = i / vpr, c = i - r * vpr;
                const _Float16* src = r < 64 ? A + static_cast<size_t>(r) * Rp
                                             : X + static_cast<size_t>(r - 64) * Rp;
                *reinterpret_cast<uint4*>(tile + r * kFwdPitch + c * 8) =
                    *reinterpret_cast<const uint4*>(src + j0 + c * 8);
            }
            __syncthreads();
            for (int ks = 0; ks < w / 16; ++ks) {
                const f16x8_t a = *reinterpret_cast<const f16x8_t*>(a_frag + ks * 16);
                const f16x8_t x = *reinterpret_cast<const f16x8_t*>(b_frag + ks * 16);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, x, acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {       // i = 2 g + h2, rows 8 g + 4 hi + 2 h2 + {0, 1}
            const int v = 4 * (i >> 1) + 2 * (i & 1);
            const float own0 = acc[v], own1 = acc[v + 1];   // a x, b x
            const float par0 = dpp_xor1(own0), par1 = dpp_xor1(own1);
            const float s1 = own0 + par1, s2 = par0 - own1;
            const float X_ = odd ? s2 : s1, Y_ = odd ? s1 : s2;
            stage[i][e] = pack_half2(X_ * resc, Y_ * resc);
        }
    }
    const size_t cbase = static_cast<size_t>(kc) * Tp * nbp;
    const int b = b0 + cb0 * 16 + (col >> 1);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int tau = 4 * (i >> 1) + 2 * hi + (i & 1);
        const int t = t0 + rb * 16 + tau;
        if (t >= T || (odd && !mirror)) continue;
        const int tq = odd ? T + t : t;
        uint4 v;
        v.x = stage[i][0];
        v.y = stage[i][1];
        v.z = stage[i][2];
        v.w = stage[i][3];
        *reinterpret_cast<uint4*>(Ch + (cbase + static_cast<size_t>(tq) * nbp + b) * 8) = v;
    }
}

// Inverse transform and maximum over shifts. Workgroup: 8 waves, each pair
// of waves one tile of 32 pairs (one t', 32 consecutive patterns) splitting
// the 32-shift blocks of the current part. MFMA A = tables (rows = shifts,
// from LDS), B = C(k) records (columns = pairs), K = one parity's
// frequencies; a lane ends with 16 shifts of one pair per block.
template <bool ANGLE>
__global__ void __launch_bounds__(kInvWaves * 64)
fft_inverse(const _Float16* __restrict__ Ch, const _Float16* __restrict__ Wg, int Fp, int half_n,
            int Sh, int part_blocks, int n_parts, int Tp, int nbp, int nb_valid, float out_scale,
            float* __restrict__ Qt, short* __restrict__ St, int n_groups) {
    extern __shared__ _Float16 wl[];                    // [2][part_blocks * 32][Fp + 8]
    __shared__ float hv[kInvTiles][32];
    __shared__ int hs[kInvTiles][32];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int h = wave & 1, slot = wave >> 1;
    const int col = lane & 31, hi = lane >> 5;
    const int pitch = Fp + 8;
    const int nbt = nbp / 32;
    const int n_tiles = Tp * nbt;
    const int KS = Fp / 16, Q = Fp / 8, NB = Sh / 32;
    const int pbs = part_blocks * 32;
    const size_t cq = static_cast<size_t>(Tp) * nbp * 8;   // halves per chunk
    for (int g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const int tile = g * kInvTiles + slot;
        const bool tvalid = tile < n_tiles;
        const int tp = tvalid ? tile / nbt : 0;
        const int bb = tvalid ? tile - tp * nbt : 0;
        const _Float16* cb = Ch + (static_cast<size_t>(tp) * nbp + bb * 32 + col) * 8;
        float bv = -INFINITY;
        int bi = 0;
        for (int part = 0; part < n_parts; ++part) {
            const int nb0 = part * part_blocks;
            const int pb = min(part_blocks, NB - nb0);
            if (n_parts > 1 || g == static_cast<int>(blockIdx.x)) {
                __syncthreads();
                const int vpr = pitch / 8;              // 16-byte vectors per table row
                const int per_par = pb * 32 * vpr;
                for (int i = threadIdx.x; i < 2 * per_par; i += kInvWaves * 64) {
                    const int p = i / per_par, rem = i - p * per_par;
                    const int r = rem / vpr, c = rem - r * vpr;
                    const uint4 v = *reinterpret_cast<const uint4*>(
                        Wg + (static_cast<size_t>(p) * Sh + nb0 * 32 + r) * pitch + c * 8);
                    *reinterpret_cast<uint4*>(wl + (static_cast<size_t>(p) * pbs + r) * pitch + c * 8) = v;
                }
                __syncthreads();
            }
            const int lo = h ? (pb + 1) / 2 : 0;
            const int cnt = h ? pb / 2 : (pb + 1) / 2;
            if (!tvalid || cnt == 0) continue;
            f32x16_t aE[kInvMaxBlocks], aO[kInvMaxBlocks];
#pragma unroll
            for (int j = 0; j < kInvMaxBlocks; ++j) { aE[j] = {}; aO[j] = {}; }
            f16x8_t cE = *reinterpret_cast<const f16x8_t*>(cb + static_cast<size_t>(hi) * cq);
            f16x8_t cO = *reinterpret_cast<const f16x8_t*>(cb + static_cast<size_t>(Q + hi) * cq);
            for (int m = 0; m < KS; ++m) {
                f16x8_t nE = cE, nO = cO;
                if (m + 1 < KS) {
                    nE = *reinterpret_cast<const f16x8_t*>(cb + static_cast<size_t>(2 * m + 2 + hi) * cq);
                    nO = *reinterpret_cast<const f16x8_t*>(cb + static_cast<size_t>(Q + 2 * m + 2 + hi) * cq);
                }
#pragma unroll
                for (int j = 0; j < kInvMaxBlocks; ++j) {
                    if (j < cnt) {
                        const int srow = (lo + j) * 32 + col;
                        const f16x8_t wE = *reinterpret_cast<const f16x8_t*>(
                            wl + static_cast<size_t>(srow) * pitch + 16 * m + 8 * hi);
                        const f16x8_t wO = *reinterpret_cast<const f16x8_t*>(
                            wl + static_cast<size_t>(pbs + srow) * pitch + 16 * m + 8 * hi);
                        aE[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wE, cE, aE[j], 0, 0, 0);
                        aO[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wO, cO, aO[j], 0, 0, 0);
                    }
                }
                cE = nE;
                cO = nO;
            }
#pragma unroll
            for (int j = 0; j < kInvMaxBlocks; ++j) {
                if (j >= cnt) continue;
                const int sb = (nb0 + lo + j) * 32 + 4 * hi;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int s = sb + 8 * (v >> 2) + (v & 3);
                    if (s >= half_n) continue;
                    const float a = aE[j][v], o = aO[j][v];
                    const float q0 = a + o, q1 = a - o;     // shifts s and s + n/2
                    if (ANGLE) {
                        if (q0 > bv || (q0 == bv && s < bi)) { bv = q0; bi = s; }
                        if (q1 > bv || (q1 == bv && s + half_n < bi)) { bv = q1; bi = s + half_n; }
                    } else {
                        bv = fmaxf(bv, fmaxf(q0, q1));
                    }
                }
            }
        }
        // lanes l and l ^ 32 hold the same pair
        {
            const float ov = __shfl_xor(bv, 32, 64);
            const int oi = __shfl_xor(bi, 32, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (h == 1 && hi == 0) {
            hv[slot][col] = bv;
            hs[slot][col] = bi;
        }
        __syncthreads();
        if (h == 0 && hi == 0 && tvalid) {
            const float ov = hv[slot][col];
            const int oi = hs[slot][col];
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            const int b = bb * 32 + col;
            if (b < nb_valid) {
                Qt[static_cast<size_t>(b) * Tp + tp] = bv * out_scale;
                if (ANGLE) St[static_cast<size_t>(b) * Tp + tp] = static_cast<short>(bi);
            }
        }
        __syncthreads();
    }
}

__global__ void fill_kernel(int32_t* dst, int64_t n, int32_t value) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = value;
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

// Approximate per-template best scores (and angles) for B patterns, chunked
// so that the stored C(k) stays within kChatBudget.
int fft_scores_impl(const tm_library* L, const float* polar, const double* norms, int32_t B,
                    float* Qt, short* St, bool compact, hipStream_t s) {
    const int n = L->n_theta, Tp = L->Tp;
    const int Rs = compact ? L->n_rows : L->R;   // rows per pattern in the polar input
    const int F = L->fft_F, Fp = L->fft_Fp, Rp = L->fft_Rp, Tpad = L->fft_Tpad, Sh = L->fft_Sh;
    const double per_pattern = static_cast<double>(Fp) * Tp * 4.0;
    int64_t bc_max = static_cast<int64_t>(kChatBudget / per_pattern) / 64 * 64;
    bc_max = std::max<int64_t>(64, bc_max);
    const int64_t n_chunks = (B + bc_max - 1) / bc_max;
    const int64_t bc = ((B + n_chunks - 1) / n_chunks + 63) / 64 * 64;

    // inverse table parts: as many 32-shift blocks as fit the LDS budget
    const int NB = Sh / 32;
    const size_t block_bytes = static_cast<size_t>(2) * 32 * (Fp + 8) * sizeof(_Float16);
    int part_blocks = static_cast<int>(std::min<size_t>(kInvLdsBudget / block_bytes, 2 * kInvMaxBlocks));
    if (part_blocks < 1) { tmlib::set_error("n_theta=%d too wide for the inverse tables", n); return TM_EUNSUPPORTED; }
    part_blocks = std::min(part_blocks, NB);
    const int n_parts = (NB + part_blocks - 1) / part_blocks;
    const size_t inv_lds = block_bytes * part_blocks;
    const size_t dft_lds = 2 * static_cast<size_t>(n) * sizeof(double) +
                           2 * static_cast<size_t>(kDftRows) * n * sizeof(double) +
                           static_cast<size_t>(kDftRows) * n * sizeof(float);
    const int n1 = dft_split(n);
    auto inv = St ? fft_inverse<true> : fft_inverse<false>;
    TM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(inv),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(inv_lds)));
    TM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fft_patterns),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dft_lds)));

    _Float16* Ph = nullptr;
    _Float16* Ch = nullptr;
    int r = alloc_async(&Ph, static_cast<size_t>(Fp) * 2 * bc * Rp, s);
    if (!r) r = alloc_async(&Ch, static_cast<size_t>(Fp) * Tp * bc * 2, s);   // re, im per (k, pair)
    const float resc = std::ldexp(1.0f, L->fft_sc - kScaleT - kScaleP);
    const float out_scale = static_cast<float>(std::ldexp(1.0, -(kScaleW + L->fft_sc)) / n);
    for (int64_t c0 = 0; !r && c0 < B; c0 += bc) {
        const int nb = static_cast<int>(std::min<int64_t>(bc, B - c0));
        const int nbp = (nb + 63) / 64 * 64;
        hipLaunchKernelGGL(fft_patterns, dim3(nbp, Rp / kDftRows), dim3(256),
                           dft_lds, s, polar + c0 * Rs * n, norms + c0,
                           compact ? nullptr : L->d_rows, Rs, L->n_rows, n, n1, F, Fp, Rp, nb,
                           2 * nbp, L->d_fft_dft, Ph);
        hipLaunchKernelGGL(fft_forward, dim3((Fp / 4) * (nbp / 64) * (Tpad / 32)), dim3(kFwdWaves * 64), 0, s,
                           reinterpret_cast<const _Float16*>(L->d_fft_t), Ph, Ch, L->T, Tp, Tpad,
                           Rp, Fp, nbp, resc);
        const int n_tiles = Tp * (nbp / 32);
        const int n_groups = (n_tiles + kInvTiles - 1) / kInvTiles;
        const int grid = std::min(n_groups, device_cus());
        hipLaunchKernelGGL(inv, dim3(grid), dim3(kInvWaves * 64), inv_lds, s, Ch,
                           reinterpret_cast<const _Float16*>(L->d_fft_w), Fp, n / 2, Sh,
                           part_blocks, n_parts, Tp, nbp, nb, out_scale, Qt + c0 * Tp,
                           St ? St + c0 * Tp : nullptr, n_groups);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "Fourier-route kernel launch");
    }
    if (Ph) (void)hipFreeAsync(Ph, s);
    if (Ch) (void)hipFreeAsync(Ch, s);
    return r;
}

int check_fft_lib(const tm_library* lib) {
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (!lib->fft) { tmlib::set_error("library was loaded without TM_LIB_FFT"); return TM_EINVAL; }
    return TM_OK;
}

}  // namespace

// ------------------------------------------------------------ library data

int tmlib::fft_prepare(tm_library* L, const std::vector<std::vector<HostPixel>>& pix,
                       hipStream_t s, size_t& bytes) {
    const int n = L->n_theta, T = L->T;
    const int F = n / 2 + 1;
    const int Fp = (F + 15) / 16 * 16;
    const int nr = std::max(1, L->n_rows);       // spectra cover the touched rows only
    const int Rp = (nr + 15) / 16 * 16;
    const int Tpad = (T + 31) / 32 * 32;
    const int half = n / 2;
    const int Sh = (half + 31) / 32 * 32;
    int row_max = 1, n_max = 0;
    for (const auto& px : pix) {
        n_max = std::max(n_max, static_cast<int>(px.size()));
        for (size_t i = 0; i < px.size();) {   // pixels are sorted by (j, k)
            size_t e = i;
            while (e < px.size() && px[e].j == px[i].j) ++e;
            row_max = std::max(row_max, static_cast<int>(e - i));
            i = e;
        }
    }
    const int sc = static_cast<int>(std::floor(std::log2(32768.0 / std::sqrt(double(row_max) * n))));

    std::vector<double> cs(2 * static_cast<size_t>(n));
    for (int m = 0; m < n; ++m) {
        const double a = 2.0 * M_PI * m / n;
        cs[2 * m] = std::cos(a);
        cs[2 * m + 1] = std::sin(a);
    }
    // template spectra [Fp][2 Tpad][Rp]: rows 2t (re) and 2t + 1 (im)
    std::vector<uint16_t> th(static_cast<size_t>(Fp) * 2 * Tpad * Rp, 0);
    auto work = [&](int t_lo, int t_hi) {
        std::vector<double> re(F), im(F);
        for (int t = t_lo; t < t_hi; ++t) {
            const double nrm = L->tnorm[t];
            if (!(nrm > 0.0)) continue;
            const double scale = std::ldexp(1.0, kScaleT) / nrm;
            const auto& px = pix[t];
            for (size_t i = 0; i < px.size();) {
                size_t e = i;
                while (e < px.size() && px[e].j == px[i].j) ++e;
                std::fill(re.begin(), re.end(), 0.0);
                std::fill(im.begin(), im.end(), 0.0);
                for (size_t q = i; q < e; ++q) {
                    const double w = px[q].w * scale;
                    const int kp = px[q].k;
                    int m = 0;
                    for (int k = 0; k < F; ++k) {
                        re[k] += w * cs[2 * m];
                        im[k] -= w * cs[2 * m + 1];
                        m += kp;
                        if (m >= n) m -= n;
                    }
                }
                const int j = L->row_index[px[i].j];
                for (int k = 0; k < F; ++k) {
                    const size_t row = (static_cast<size_t>(k) * 2 * Tpad + 2 * t) * Rp + j;
                    th[row] = half_bits(re[k]);
                    th[row + Rp] = half_bits(im[k]);
                }
                i = e;
            }
        }
    };
    const int n_threads = std::max(1, std::min<int>(16, static_cast<int>(std::thread::hardware_concurrency())));
    {
        std::vector<std::thread> pool;
        for (int w = 0; w < n_threads; ++w)
            pool.emplace_back(work, static_cast<int>(static_cast<long long>(T) * w / n_threads),
                              static_cast<int>(static_cast<long long>(T) * (w + 1) / n_threads));
        for (auto& th_ : pool) th_.join();
    }
    // inverse tables [parity][Sh][Fp + 8]: entry kk = 8 q + 2 e + part is
    // frequency k = parity + 8 q + 2 e; part 0 = c_k cos, 1 = -c_k sin (x 2^12)
    const int pitch = Fp + 8;
    std::vector<uint16_t> tw(static_cast<size_t>(2) * Sh * pitch, 0);
    for (int p = 0; p < 2; ++p)
        for (int sft = 0; sft < half; ++sft)
            for (int kk = 0; kk < Fp; ++kk) {
                const int q = kk / 8, e = (kk % 8) / 2, part = kk % 2;
                const int k = p + 8 * q + 2 * e;
                if (k >= F) continue;
                const int m = static_cast<int>((static_cast<long long>(k) * sft) % n);
                const double ck = (k == 0 || 2 * k == n) ? 1.0 : 2.0;
                const double v = part == 0 ? ck * cs[2 * m] : -ck * cs[2 * m + 1];
                tw[(static_cast<size_t>(p) * Sh + sft) * pitch + kk] = half_bits(std::ldexp(v, kScaleW));
            }

    L->fft_F = F;
    L->fft_Fp = Fp;
    L->fft_Rp = Rp;
    L->fft_Tpad = Tpad;
    L->fft_Sh = Sh;
    L->fft_sc = sc;
    L->fft_eps = error_bound(nr, Fp, sc, n_max);
    int r = upload_vec(&L->d_fft_t, th, s, bytes);
    if (!r) r = upload_vec(&L->d_fft_w, tw, s, bytes);
    if (!r) r = upload_vec(&L->d_fft_dft, cs, s, bytes);
    if (!r) {
        // the host vectors above must outlive the copies
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) r = tmlib::hip_fail(e, "hipStreamSynchronize");
    }
    if (!r) L->fft = true;
    return r;
}

void tmlib::fft_release(tm_library* L) {
    (void)hipFree(L->d_fft_t);
    (void)hipFree(L->d_fft_w);
    (void)hipFree(L->d_fft_dft);
    L->d_fft_t = nullptr;
    L->d_fft_w = nullptr;
    L->d_fft_dft = nullptr;
}

int tmlib::fill_i32(int32_t* dst, int64_t n, int32_t value, hipStream_t s) {
    if (n <= 0) return TM_OK;
    hipLaunchKernelGGL(fill_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, dst, n, value);
    TM_HIP(hipGetLastError());
    return TM_OK;
}

// ------------------------------------------------------ coarse + rescoring

int tmlib::fft_match(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                     int32_t N, int32_t policy, double keep, int32_t* n_rescored,
                     int32_t* top_template, int32_t* top_angle, float* top_score, bool compact,
                     hipStream_t s) {
    const int Tp = lib->Tp;
    float* Qt = nullptr;
    int r = alloc_async(&Qt, static_cast<size_t>(B) * Tp, s);
    if (!r) r = fft_scores_impl(lib, polar, norms, B, Qt, nullptr, compact, s);
    if (policy == TM_RESCORE_KEEP) {
        int32_t n_keep = static_cast<int32_t>(std::ceil(keep * Tp - 1e-9));
        n_keep = std::max(N, std::min(n_keep, Tp));
        int32_t* cand = nullptr;
        if (!r) r = alloc_async(&cand, static_cast<size_t>(B) * n_keep, s);
        if (!r) r = tmlib::select_top(Qt, B, Tp, n_keep, cand, s);
        if (!r) r = tmlib::launch_match(lib, polar, norms, B, N, top_template, top_angle, top_score,
                                        nullptr, nullptr, cand, n_keep, nullptr, nullptr, compact, s);
        if (!r && n_rescored) r = tmlib::fill_i32(n_rescored, B, n_keep, s);
        if (cand) (void)hipFreeAsync(cand, s);
    } else {
        const double frac = keep > 0.0 ? keep : 0.1;
        int32_t cap = static_cast<int32_t>(std::ceil(frac * Tp - 1e-9));
        cap = std::max(N, std::min(cap, Tp));
        if (!r) r = tmlib::certified_rescore(lib, polar, norms, B, N, N, Qt, Tp, nullptr,
                                             lib->fft_eps, cap, n_rescored, top_template,
                                             top_angle, top_score, compact, s);
    }
    if (Qt) (void)hipFreeAsync(Qt, s);
    return r;
}

// --------------------------------------------------------------- C ABI

extern "C" int tm_fft_scores(const tm_library* lib, const float* polar, const double* norms,
                             int32_t B, int32_t compact_rows, float* approx_score,
                             int16_t* approx_angle, void* hip_stream) {
    tmlib::clear_error();
    if (int r = check_fft_lib(lib)) return r;
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (compact_rows != 0 && compact_rows != 1) { tmlib::set_error("compact_rows=%d must be 0 or 1", compact_rows); return TM_EINVAL; }
    if (B == 0) return TM_OK;
    if (!polar || !norms || !approx_score) {
        tmlib::set_error("polar, norms and approx_score must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    return fft_scores_impl(lib, polar, norms, B, approx_score,
                           reinterpret_cast<short*>(approx_angle), compact_rows == 1,
                           static_cast<hipStream_t>(hip_stream));
}

extern "C" int tm_fft_error_bound(const tm_library* lib, double* eps) {
    tmlib::clear_error();
    if (int r = check_fft_lib(lib)) return r;
    if (!eps) { tmlib::set_error("eps must be non-NULL"); return TM_EINVAL; }
    *eps = lib->fft_eps;
    return TM_OK;
}
