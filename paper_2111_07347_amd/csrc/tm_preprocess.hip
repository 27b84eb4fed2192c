// Pattern preprocessing before indexing (Section 4.1: the direct beam is
// centred, the diffuse background removed by a difference of Gaussians, the
// result smoothed by a Gaussian blur and low intensities set to zero; the
// discussion names parallelising these steps as an open optimisation).
//
//   centre_kernel  one workgroup per pattern: the maximum of the square box
//                  |x - W/2| <= r_box, |y - H/2| <= r_box, then the
//                  intensity-weighted centroid (float64) of the box pixels
//                  >= frac times that maximum.
//   row_kernel     one wave per image row (4 per workgroup): the row of the
//                  centred pattern, out(x, y) = in(x + cx - W/2, y + cy - H/2)
//                  (bilinear, zero outside), or of an intermediate image, is
//                  built in LDS, then correlated along x with one or two
//                  sampled Gaussians (mirror boundary).
//   col_tile_kernel  32-column strips of images up to 256 rows, staged whole
//                  in LDS: correlation along y with one or two Gaussians; two
//                  give the difference of Gaussians; an optional threshold
//                  sets values below it to 0. col_kernel does the same for
//                  taller images, one thread per column (coalesced rows).
//
// Gaussians: exp(-t^2 / (2 sigma^2)) on |t| <= floor(4 sigma + 0.5),
// normalised in float64 on the host, applied in float32; mirror boundary
// (... c b a | a b c ...) by folding indices modulo 2n. The passes run over
// chunks of patterns so that the two float32 scratch images stay within
// 1 GiB. The filters cost 2 (2 r + 1) FMAs per pixel and Gaussian, more
// than the machine balance for the default radii, but each pass also
// streams images through HBM (about ten image sizes per pattern with all
// steps on) and waits on its staging loads.
#include <algorithm>
#include <cmath>

#include "tm_internal.h"

namespace {

constexpr int kMaxRadius = 64;            // sigma <= 15.9
constexpr int kRowThreads = 256;
constexpr int kRowWaves = kRowThreads / 64;
constexpr size_t kLdsLimit = 156 * 1024;
constexpr int kTileRows = 256;            // column-strip kernel: images up to this high
constexpr int kTapBlock = 8;              // taps per weight block of the column-strip kernel
constexpr int kStageBatch = 8;            // loads in flight per thread while staging
constexpr int kRowBatch = 4;              // columns per lane in flight while staging a row

// Floats of one wave's row strip: the row rounded up to 256 columns (the
// last chunk's lanes read past W) plus the two halos of rh (a multiple of 4)
// and 16 more, which the last tap block's window may reach.
__host__ __device__ inline int row_strip(int W, int rh) { return (W + 255) / 256 * 256 + 2 * rh + 16; }

constexpr int kCentreThreads = 256;
constexpr size_t kScratchBudget = size_t(1) << 30;

// Zero-padded copy of a tap table for the row kernel: wp[t + r4] = w(t) for
// t in [-r4, r4 + 7], r4 = the radius rounded up to a multiple of 4, zero
// past the radius.
constexpr int kWLen = 2 * kMaxRadius + 16;

struct Taps {
    int r;
    float w[2 * kMaxRadius + 1];
    alignas(32) float wp[kWLen];
};


// acc[m] += sum_t w(t) * row[c + m + t], m < 4, over the padded table of
// tp, in blocks of 8 taps: per block one 32-byte scalar load of weights and
// a 12-float window (aligned 16-byte LDS reads) feed 32 FMAs. c and the
// block starts are multiples of 4.
__device__ __forceinline__ void conv4(const float* row, int c, const Taps& tp, float (&acc)[4]) {
    const int r4 = (tp.r + 3) & ~3;
    for (int t0 = -r4; t0 <= r4; t0 += 8) {
        float w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) w[j] = tp.wp[t0 + r4 + j];
        const float4* p = static_cast<const float4*>(__builtin_assume_aligned(row + c + t0, 16));
        float win[12];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float4 v = p[q];
            win[4 * q] = v.x; win[4 * q + 1] = v.y; win[4 * q + 2] = v.z; win[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int m = 0; m < 4; ++m) acc[m] += w[j] * win[m + j];
    }
}


__device__ __forceinline__ int mirror(int i, int n) {
    if (static_cast<unsigned>(i) < static_cast<unsigned>(n)) return i;
    if (i < 0 && i >= -n) return -i - 1;
    if (i >= n && i < 2 * n) return 2 * n - 1 - i;
    // images narrower than the halo: fold modulo the period 2n
    const int p = 2 * n;
    int j = i % p;
    if (j < 0) j += p;
    return j < n ? j : p - 1 - j;
}

template <typename Tin>
__device__ __forceinline__ float load_px(const Tin* img, int H, int W, int y, int x) {
    return (x >= 0 && x < W && y >= 0 && y < H) ? static_cast<float>(img[static_cast<size_t>(y) * W + x])
                                                 : 0.0f;
}

template <typename Tin>
__global__ void __launch_bounds__(kCentreThreads)
centre_kernel(const Tin* __restrict__ patterns, int H, int W, int r_box, double frac,
              double* __restrict__ centre) {
    __shared__ double red[4][kCentreThreads / 64];
    const int b = blockIdx.x;
    const Tin* img = patterns + static_cast<size_t>(b) * H * W;
    const double x0 = 0.5 * W, y0 = 0.5 * H;
    const int xl = max(0, static_cast<int>(ceil(x0 - r_box))), xh = min(W - 1, static_cast<int>(floor(x0 + r_box)));
    const int yl = max(0, static_cast<int>(ceil(y0 - r_box))), yh = min(H - 1, static_cast<int>(floor(y0 + r_box)));
    const int bw = xh - xl + 1, n = (xh >= xl && yh >= yl) ? bw * (yh - yl + 1) : 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double m = -INFINITY;
    for (int i = threadIdx.x; i < n; i += kCentreThreads) {
        const int y = yl + i / bw, x = xl + i % bw;
        m = fmax(m, static_cast<double>(img[static_cast<size_t>(y) * W + x]));
    }
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) red[0][wave] = m;
    __syncthreads();
    m = red[0][0];
    for (int w = 1; w < kCentreThreads / 64; ++w) m = fmax(m, red[0][w]);
    __syncthreads();
    double s = 0.0, sx = 0.0, sy = 0.0;
    const double thr = frac * m;
    for (int i = threadIdx.x; i < n; i += kCentreThreads) {
        const int y = yl + i / bw, x = xl + i % bw;
        const double v = static_cast<double>(img[static_cast<size_t>(y) * W + x]);
        if (v >= thr) {
            s += v;
            sx += v * x;
            sy += v * y;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
    }
    if (lane == 0) {
        red[1][wave] = s;
        red[2][wave] = sx;
        red[3][wave] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ts = 0.0, tx = 0.0, ty = 0.0;
        for (int w = 0; w < kCentreThreads / 64; ++w) {
            ts += red[1][w];
            tx += red[2][w];
            ty += red[3][w];
        }
        const bool ok = n > 0 && m > 0.0;
        centre[2 * b] = ok ? tx / ts : x0;
        centre[2 * b + 1] = ok ? ty / ts : y0;
    }
}

// One image row per wave (4 rows per workgroup): the row of the source is
// staged in the wave's LDS strip with a mirrored halo of rh columns on each
// side (rh a multiple of 4, at least the largest radius), then correlated
// along x with taps a (-> out_a) and, when out_b is given, taps b
// (-> out_b). The source is the input pattern (`in`), centred when `centre`
// is given, else the float image `src`. Lanes own 4 consecutive columns of
// each 256-column chunk and share one tap window among them (conv4).
template <typename Tin>
__global__ void __launch_bounds__(kRowThreads)
row_kernel(const Tin* __restrict__ in, const float* __restrict__ src,
           const double* __restrict__ centre, int H, int W, Taps a, Taps bt, int rh,
           float* __restrict__ out_a, float* __restrict__ out_b) {
    extern __shared__ float lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int y = blockIdx.x * kRowWaves + wave, b = blockIdx.y;
    if (y >= H) return;    // the wave leaves; no workgroup barrier follows
    const int span = W + 2 * rh;
    float* row = lds + static_cast<size_t>(wave) * row_strip(W, rh);
    const size_t base = (static_cast<size_t>(b) * H + y) * W;
    if (in && centre) {
        const Tin* img = in + static_cast<size_t>(b) * H * W;
        const double dx = centre[2 * b] - 0.5 * W, dy = centre[2 * b + 1] - 0.5 * H;
        const double ys = y + dy;
        const double yf = floor(ys);
        const float fy = static_cast<float>(ys - yf);
        const int yi = static_cast<int>(fmax(fmin(yf, 1e9), -1e9));
        // kRowBatch columns per lane in flight: all taps are loaded first
        for (int i0 = lane; i0 < span; i0 += 64 * kRowBatch) {
            float p[kRowBatch][4], fx[kRowBatch];
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) {
                const int i = min(i0 + 64 * u, span - 1);
                const double xs = mirror(i - rh, W) + dx;
                const double xf = floor(xs);
                fx[u] = static_cast<float>(xs - xf);
                const int xi = static_cast<int>(fmax(fmin(xf, 1e9), -1e9));
                p[u][0] = load_px(img, H, W, yi, xi);
                p[u][1] = load_px(img, H, W, yi, xi + 1);
                p[u][2] = load_px(img, H, W, yi + 1, xi);
                p[u][3] = load_px(img, H, W, yi + 1, xi + 1);
            }
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) {
                const int i = i0 + 64 * u;
                if (i < span)
                    row[i] = (1.0f - fx[u]) * (1.0f - fy) * p[u][0] + fx[u] * (1.0f - fy) * p[u][1] +
                             (1.0f - fx[u]) * fy * p[u][2] + fx[u] * fy * p[u][3];
            }
        }
    } else {
        for (int i0 = lane; i0 < span; i0 += 64 * kRowBatch) {
            float v[kRowBatch];
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u) {
                const size_t q = base + mirror(min(i0 + 64 * u, span - 1) - rh, W);
                v[u] = in ? static_cast<float>(in[q]) : src[q];
            }
#pragma unroll
            for (int u = 0; u < kRowBatch; ++u)
                if (i0 + 64 * u < span) row[i0 + 64 * u] = v[u];
        }
    }
    // the tail of the strip (past the right halo) holds zeros: the zero
    // weights of the last tap blocks read it
    for (int i = span + lane; i < row_strip(W, rh); i += 64) row[i] = 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // each lane owns 4 consecutive columns of every 256-column chunk
    for (int x0 = 0; x0 < W; x0 += 4 * 64) {
        const int x = x0 + 4 * lane;
        float va[4] = {0.0f, 0.0f, 0.0f, 0.0f}, vb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        conv4(row, x + rh, a, va);
        if (out_b) conv4(row, x + rh, bt, vb);
        if ((W & 3) == 0 && x + 3 < W) {
            *reinterpret_cast<float4*>(out_a + base + x) = make_float4(va[0], va[1], va[2], va[3]);
            if (out_b) *reinterpret_cast<float4*>(out_b + base + x) = make_float4(vb[0], vb[1], vb[2], vb[3]);
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (x + m < W) {
                    out_a[base + x + m] = va[m];
                    if (out_b) out_b[base + x + m] = vb[m];
                }
            }
        }
    }
}

// acc[i] += sum_t w[t] * L[(y + i + t) * 32 + c] for kTileRows / 8 rows i,
// taps in blocks of kTapBlock: per block the weights are loaded once and a
// window of rows + kTapBlock - 1 LDS values serves kTapBlock * rows FMAs
// (weights past the radius are zero; the tile carries kTapBlock spare rows).
template <int kRows>
__device__ __forceinline__ void tap_block_col(const float* L, const Taps& tp, int y, int c,
                                              float (&acc)[kRows]) {
    for (int t0 = -tp.r; t0 <= tp.r; t0 += kTapBlock) {
        float w[kTapBlock];
#pragma unroll
        for (int j = 0; j < kTapBlock; ++j) w[j] = t0 + j <= tp.r ? tp.w[t0 + j + tp.r] : 0.0f;
        const float* p = L + (y + t0) * 32 + c;
        float win[kRows + kTapBlock - 1];
#pragma unroll
        for (int i = 0; i < kRows + kTapBlock - 1; ++i) win[i] = p[i * 32];
#pragma unroll
        for (int j = 0; j < kTapBlock; ++j)
#pragma unroll
            for (int i = 0; i < kRows; ++i) acc[i] += w[j] * win[i + j];
    }
}

// Correlation along y for a strip of 32 columns of an image at most
// kTileRows high, held whole in LDS with a mirrored halo of rh rows:
// out = G_a(ia) [- G_b(ib)], then the threshold. Threads: 32 columns x 8
// row groups of kTileRows / 8 consecutive rows (rows of 128 bytes load
// coalesced); the tap loop is the outer one, so each weight is loaded once
// per thread and feeds 32 FMAs.
__global__ void __launch_bounds__(kRowThreads)
col_tile_kernel(const float* __restrict__ ia, const float* __restrict__ ib, int H, int W, Taps a,
                Taps bt, int rh, bool thresh, float threshold, float* __restrict__ out) {
    extern __shared__ float lds[];
    constexpr int kRows = kTileRows / (kRowThreads / 32);
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int x = blockIdx.x * 32 + c, b = blockIdx.y;
    const bool col_ok = x < W;
    const int hp = kTileRows + 2 * rh + kTapBlock;
    float* la = lds;
    float* lb = lds + static_cast<size_t>(hp) * 32;
    const size_t img = static_cast<size_t>(b) * H * W;
    // staging: kStageBatch rows per thread loaded before any is stored, so
    // their latencies overlap (every lane loads; columns past W read column
    // 0 and store zeros)
    constexpr int kGroups = kRowThreads / 32;
    for (int i0 = g; i0 < hp; i0 += kGroups * kStageBatch) {
        float va[kStageBatch], vb[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int i = min(i0 + kGroups * u, hp - 1);
            const size_t src = img + static_cast<size_t>(mirror(i - rh, H)) * W + (col_ok ? x : 0);
            va[u] = ia[src];
            vb[u] = ib ? ib[src] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int i = i0 + kGroups * u;
            if (i < hp) {
                la[i * 32 + c] = col_ok ? va[u] : 0.0f;
                if (ib) lb[i * 32 + c] = col_ok ? vb[u] : 0.0f;
            }
        }
    }
    __syncthreads();
    const int y0 = g * kRows;
    if (!col_ok || y0 >= H) return;
    float va[kRows], vb[kRows];
#pragma unroll
    for (int i = 0; i < kRows; ++i) va[i] = vb[i] = 0.0f;
    tap_block_col(la, a, y0 + rh, c, va);
    if (ib) tap_block_col(lb, bt, y0 + rh, c, vb);
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
        if (y0 + i >= H) break;
        float v = ib ? va[i] - vb[i] : va[i];
        if (thresh && v < threshold) v = 0.0f;
        out[img + static_cast<size_t>(y0 + i) * W + x] = v;
    }
}

// Correlation along y for any height (one thread per column, coalesced rows):
// out = G_a(ia) [- G_b(ib)], then the threshold.
__global__ void __launch_bounds__(kRowThreads)
col_kernel(const float* __restrict__ ia, const float* __restrict__ ib, int H, int W, Taps a,
           Taps bt, bool thresh, float threshold, float* __restrict__ out) {
    const int x = blockIdx.x * kRowThreads + threadIdx.x;
    const int b = blockIdx.y;
    if (x >= W) return;
    const size_t img = static_cast<size_t>(b) * H * W;
    for (int y = 0; y < H; ++y) {
        float v = 0.0f;
        for (int t = -a.r; t <= a.r; ++t) v += a.w[t + a.r] * ia[img + static_cast<size_t>(mirror(y + t, H)) * W + x];
        if (ib) {
            float u = 0.0f;
            for (int t = -bt.r; t <= bt.r; ++t) u += bt.w[t + bt.r] * ib[img + static_cast<size_t>(mirror(y + t, H)) * W + x];
            v -= u;
        }
        if (thresh && v < threshold) v = 0.0f;
        out[img + static_cast<size_t>(y) * W + x] = v;
    }
}

void pad_taps(Taps& t) {
    const int r4 = (t.r + 3) & ~3;
    for (int i = 0; i < kWLen; ++i) {
        const int k = i - r4;
        t.wp[i] = (k >= -t.r && k <= t.r) ? t.w[k + t.r] : 0.0f;
    }
}

bool make_taps(double sigma, Taps& t) {
    t = Taps{};
    if (!(sigma > 0.0)) {
        t.r = 0;
        t.w[0] = 1.0f;
        pad_taps(t);
        return true;
    }
    const int r = static_cast<int>(4.0 * sigma + 0.5);
    if (r > kMaxRadius) return false;
    double w[2 * kMaxRadius + 1], s = 0.0;
    for (int i = -r; i <= r; ++i) {
        w[i + r] = std::exp(-static_cast<double>(i) * i / (2.0 * sigma * sigma));
        s += w[i + r];
    }
    t.r = r;
    for (int i = 0; i <= 2 * r; ++i) t.w[i] = static_cast<float>(w[i] / s);
    pad_taps(t);
    return true;
}

template <typename Tin>
int run(const Tin* in, int B, int H, int W, const tm_preprocess_opts& o, float* out,
        double* centre_out, hipStream_t s) {
    Taps ta, tb, tblur, tid;
    if (!make_taps(o.sigma_min, ta) || !make_taps(o.sigma_max, tb) ||
        !make_taps(o.sigma_blur, tblur)) {
        tmlib::set_error("Gaussian sigma above %g (radius %d)", (kMaxRadius - 0.5) / 4.0, kMaxRadius);
        return TM_EINVAL;
    }
    make_taps(0.0, tid);
    const bool dog = o.sigma_max > 0.0;
    const bool thresh = std::isfinite(o.threshold);
    const size_t img = static_cast<size_t>(H) * W;
    const int chunk = static_cast<int>(std::max<size_t>(
        1, std::min<size_t>({static_cast<size_t>(B), kScratchBudget / (2 * img * 4), size_t(65535)})));
    float* s1 = nullptr;
    float* s2 = nullptr;
    double* cen = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&s1), img * 4 * chunk, s);
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&s2), img * 4 * chunk, s);
    if (e == hipSuccess && !centre_out) e = hipMallocAsync(reinterpret_cast<void**>(&cen), 16 * static_cast<size_t>(B), s);
    int r = TM_OK;
    if (e != hipSuccess) r = tmlib::hip_fail(e, "hipMallocAsync");
    double* cptr = centre_out ? centre_out : cen;
    // LDS: rows with a mirrored halo (any W up to 8192 fits), column strips
    // of the full height when they fit, else the per-column kernel
    const int rh1 = dog ? std::max(ta.r, tb.r) : 0, rhb = tblur.r;
    // row halos rounded up to multiples of 4 (aligned tap windows)
    const int rr1 = (rh1 + 3) & ~3, rrb = (rhb + 3) & ~3;
    const size_t row_lds1 = static_cast<size_t>(kRowWaves) * row_strip(W, rr1) * sizeof(float);
    const size_t row_ldsb = static_cast<size_t>(kRowWaves) * row_strip(W, rrb) * sizeof(float);
    const size_t col_lds1 =
        static_cast<size_t>(kTileRows + 2 * rh1 + kTapBlock) * 32 * sizeof(float) * (dog ? 2 : 1);
    const size_t col_ldsb = static_cast<size_t>(kTileRows + 2 * rhb + kTapBlock) * 32 * sizeof(float);
    const bool tile1 = H <= kTileRows && col_lds1 <= kLdsLimit;
    const bool tileb = H <= kTileRows && col_ldsb <= kLdsLimit;
    if (r == TM_OK) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(row_kernel<Tin>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(row_lds1));
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(row_kernel<float>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(std::max(row_ldsb, row_lds1)));
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(col_tile_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(std::min(kLdsLimit, std::max(col_lds1, col_ldsb))));
        if (e != hipSuccess) r = tmlib::hip_fail(e, "hipFuncSetAttribute");
    }
    const dim3 rgrid((H + kRowWaves - 1) / kRowWaves, 1);
    const dim3 tgrid((W + 31) / 32, 1);
    const dim3 cgrid((W + kRowThreads - 1) / kRowThreads, 1);
    const bool blur = o.sigma_blur > 0.0;
    for (int b0 = 0; r == TM_OK && b0 < B; b0 += chunk) {
        const int nb = std::min(chunk, B - b0);
        const Tin* cin = in + static_cast<size_t>(b0) * img;
        float* cout = out + static_cast<size_t>(b0) * img;
        double* cc = cptr + 2 * static_cast<size_t>(b0);
        if (o.r_box >= 0 || centre_out) {
            // with r_box < 0 the box is empty and the centre is (W/2, H/2)
            hipLaunchKernelGGL(centre_kernel<Tin>, dim3(nb), dim3(kCentreThreads), 0, s, cin, H, W,
                               o.r_box, o.frac, cc);
        }
        // centred rows, correlated along x with G(sigma_min) and G(sigma_max)
        hipLaunchKernelGGL(row_kernel<Tin>, dim3(rgrid.x, nb), dim3(kRowThreads), row_lds1, s, cin,
                           static_cast<const float*>(nullptr), o.r_box >= 0 ? cc : nullptr, H, W,
                           dog ? ta : tid, tb, rr1, s1, dog ? s2 : nullptr);
        // along y: difference of Gaussians (or the plain centred image) -> out
        if (tile1)
            hipLaunchKernelGGL(col_tile_kernel, dim3(tgrid.x, nb), dim3(kRowThreads), col_lds1, s,
                               s1, dog ? s2 : nullptr, H, W, dog ? ta : tid, tb, rh1,
                               !blur && thresh, static_cast<float>(o.threshold), cout);
        else
            hipLaunchKernelGGL(col_kernel, dim3(cgrid.x, nb), dim3(kRowThreads), 0, s, s1,
                               dog ? s2 : nullptr, H, W, dog ? ta : tid, tb, !blur && thresh,
                               static_cast<float>(o.threshold), cout);
        if (blur) {
            // rows of the difference image (now in out) -> s1, then columns -> out
            hipLaunchKernelGGL(row_kernel<float>, dim3(rgrid.x, nb), dim3(kRowThreads), row_ldsb, s,
                               static_cast<const float*>(nullptr), static_cast<const float*>(cout),
                               static_cast<const double*>(nullptr), H, W, tblur, tid, rrb, s1,
                               static_cast<float*>(nullptr));
            if (tileb)
                hipLaunchKernelGGL(col_tile_kernel, dim3(tgrid.x, nb), dim3(kRowThreads), col_ldsb,
                                   s, s1, static_cast<const float*>(nullptr), H, W, tblur, tid,
                                   rhb, thresh, static_cast<float>(o.threshold), cout);
            else
                hipLaunchKernelGGL(col_kernel, dim3(cgrid.x, nb), dim3(kRowThreads), 0, s, s1,
                                   static_cast<const float*>(nullptr), H, W, tblur, tid, thresh,
                                   static_cast<float>(o.threshold), cout);
        }
        e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "preprocess kernel launch");
    }
    if (s1) (void)hipFreeAsync(s1, s);
    if (s2) (void)hipFreeAsync(s2, s);
    if (cen) (void)hipFreeAsync(cen, s);
    return r;
}

}  // namespace

extern "C" int tm_preprocess(const void* patterns, tm_dtype dtype, int32_t B, int32_t H,
                             int32_t W, const tm_preprocess_opts* opts, float* out,
                             double* centre_out, void* hip_stream) {
    tmlib::clear_error();
    if (!opts) { tmlib::set_error("opts is NULL"); return TM_EINVAL; }
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (H < 1 || W < 1 || H > 8192 || W > 8192) { tmlib::set_error("H=%d, W=%d outside [1, 8192]", H, W); return TM_EINVAL; }
    if (dtype != TM_U16 && dtype != TM_F32) { tmlib::set_error("unknown dtype %d", static_cast<int>(dtype)); return TM_EINVAL; }
    const tm_preprocess_opts& o = *opts;
    if (o.r_box > 4096) { tmlib::set_error("r_box=%d too large", o.r_box); return TM_EINVAL; }
    if (!std::isfinite(o.frac) || !std::isfinite(o.sigma_min) || !std::isfinite(o.sigma_max) ||
        !std::isfinite(o.sigma_blur) || o.sigma_min < 0.0 || o.sigma_max < 0.0 ||
        o.sigma_blur < 0.0 || std::isnan(o.threshold)) {
        tmlib::set_error("frac and sigmas must be finite, sigmas >= 0, threshold not NaN");
        return TM_EINVAL;
    }
    if (o.sigma_max > 0.0 && !(o.sigma_min < o.sigma_max)) {
        tmlib::set_error("difference of Gaussians needs sigma_min < sigma_max");
        return TM_EINVAL;
    }
    for (double sg : {o.sigma_min, o.sigma_max, o.sigma_blur}) {
        if (static_cast<int>(4.0 * sg + 0.5) > kMaxRadius) {
            tmlib::set_error("Gaussian sigma %g above %g (radius %d)", sg, (kMaxRadius - 0.5) / 4.0,
                             kMaxRadius);
            return TM_EINVAL;
        }
    }
    if (B > 0 && (!patterns || !out)) { tmlib::set_error("patterns and out must be non-NULL"); return TM_EINVAL; }
    if (int r = tmlib::require_device()) return r;
    if (B == 0) return TM_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (dtype == TM_F32)
        return run(static_cast<const float*>(patterns), B, H, W, o, out, centre_out, s);
    return run(static_cast<const uint16_t*>(patterns), B, H, W, o, out, centre_out, s);
}
