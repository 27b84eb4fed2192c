// Pattern preprocessing before indexing (Section 4.2: the direct beam is
// centred, the diffuse background removed by a difference of Gaussians, the
// result smoothed by a Gaussian blur and low intensities set to zero; the
// discussion names parallelising these steps as an open optimisation).
//
//   centre_kernel  one workgroup per pattern: the maximum of the square box
//                  |x - W/2| <= r_box, |y - H/2| <= r_box, then the
//                  intensity-weighted centroid (float64) of the box pixels
//                  >= frac times that maximum.
//   row_kernel     one workgroup per image row: the row of the centred
//                  pattern, out(x, y) = in(x + cx - W/2, y + cy - H/2)
//                  (bilinear, zero outside), or of an intermediate image, is
//                  built in LDS, then correlated along x with one or two
//                  sampled Gaussians (mirror boundary).
//   col_kernel     one thread per column (coalesced rows): correlation along
//                  y with one or two Gaussians; two give the difference of
//                  Gaussians; an optional threshold sets values below it to 0.
//
// Gaussians: exp(-t^2 / (2 sigma^2)) on |t| <= floor(4 sigma + 0.5),
// normalised in float64 on the host, applied in float32; mirror boundary
// (... c b a | a b c ...) by folding indices modulo 2n. The passes run over
// chunks of patterns so that the two float32 scratch images stay within
// 1 GiB. Every pass streams images through HBM: the work is bound by memory
// traffic (about ten image sizes per pattern with all steps on).
#include <algorithm>
#include <cmath>

#include "tm_internal.h"

namespace {

constexpr int kMaxRadius = 64;            // sigma <= 15.9
constexpr int kRowThreads = 256;
constexpr int kCentreThreads = 256;
constexpr size_t kScratchBudget = size_t(1) << 30;

struct Taps {
    int r;
    float w[2 * kMaxRadius + 1];
};

__device__ __forceinline__ int mirror(int i, int n) {
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

// One row of the source correlated along x with taps a (-> out_a) and, when
// out_b is given, taps b (-> out_b). The source is the input pattern (`in`),
// centred when `centre` is given, else the float image `src`.
template <typename Tin>
__global__ void __launch_bounds__(kRowThreads)
row_kernel(const Tin* __restrict__ in, const float* __restrict__ src,
           const double* __restrict__ centre, int H, int W, Taps a, Taps bt,
           float* __restrict__ out_a, float* __restrict__ out_b) {
    extern __shared__ float row[];
    const int y = blockIdx.x, b = blockIdx.y;
    const size_t base = (static_cast<size_t>(b) * H + y) * W;
    if (in && !centre) {
        for (int x = threadIdx.x; x < W; x += kRowThreads) row[x] = static_cast<float>(in[base + x]);
    } else if (in) {
        const Tin* img = in + static_cast<size_t>(b) * H * W;
        const double dx = centre[2 * b] - 0.5 * W, dy = centre[2 * b + 1] - 0.5 * H;
        const double ys = y + dy;
        const double yf = floor(ys);
        const float fy = static_cast<float>(ys - yf);
        const int yi = static_cast<int>(fmax(fmin(yf, 1e9), -1e9));
        for (int x = threadIdx.x; x < W; x += kRowThreads) {
            const double xs = x + dx;
            const double xf = floor(xs);
            const float fx = static_cast<float>(xs - xf);
            const int xi = static_cast<int>(fmax(fmin(xf, 1e9), -1e9));
            const float p00 = load_px(img, H, W, yi, xi), p01 = load_px(img, H, W, yi, xi + 1);
            const float p10 = load_px(img, H, W, yi + 1, xi), p11 = load_px(img, H, W, yi + 1, xi + 1);
            row[x] = (1.0f - fx) * (1.0f - fy) * p00 + fx * (1.0f - fy) * p01 +
                     (1.0f - fx) * fy * p10 + fx * fy * p11;
        }
    } else {
        for (int x = threadIdx.x; x < W; x += kRowThreads) row[x] = src[base + x];
    }
    __syncthreads();
    for (int x = threadIdx.x; x < W; x += kRowThreads) {
        float va = 0.0f;
        for (int t = -a.r; t <= a.r; ++t) va += a.w[t + a.r] * row[mirror(x + t, W)];
        out_a[base + x] = va;
        if (out_b) {
            float vb = 0.0f;
            for (int t = -bt.r; t <= bt.r; ++t) vb += bt.w[t + bt.r] * row[mirror(x + t, W)];
            out_b[base + x] = vb;
        }
    }
}

// Correlation along y: out = G_a(ia) [- G_b(ib)], then the threshold.
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

bool make_taps(double sigma, Taps& t) {
    t = Taps{};
    if (!(sigma > 0.0)) {
        t.r = 0;
        t.w[0] = 1.0f;
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
    const size_t row_lds = static_cast<size_t>(W) * sizeof(float);
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
        hipLaunchKernelGGL(row_kernel<Tin>, dim3(H, nb), dim3(kRowThreads), row_lds, s, cin,
                           static_cast<const float*>(nullptr), o.r_box >= 0 ? cc : nullptr, H, W,
                           dog ? ta : tid, tb, s1, dog ? s2 : nullptr);
        // along y: difference of Gaussians (or the plain centred image)
        const dim3 cgrid((W + kRowThreads - 1) / kRowThreads, nb);
        const bool blur = o.sigma_blur > 0.0;
        hipLaunchKernelGGL(col_kernel, cgrid, dim3(kRowThreads), 0, s, s1, dog ? s2 : nullptr, H, W,
                           dog ? ta : tid, tb, !blur && thresh, static_cast<float>(o.threshold),
                           cout);
        if (blur) {
            // rows of the difference image (now in out) -> s1, then columns -> out
            hipLaunchKernelGGL(row_kernel<float>, dim3(H, nb), dim3(kRowThreads), row_lds, s,
                               static_cast<const float*>(nullptr), static_cast<const float*>(cout),
                               static_cast<const double*>(nullptr), H, W, tblur, tid, s1,
                               static_cast<float*>(nullptr));
            hipLaunchKernelGGL(col_kernel, cgrid, dim3(kRowThreads), 0, s, s1,
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
