// tm_polar_transform: intensity transform, polar resampling about the
// direct-beam centre, image norms and azimuthal profiles (Section 2.2 and
// Fig. 2 c for the polar image; Eq. (1) for the image norm; Fig. 3 for the
// azimuthal integral used by the pre-filter).
//
// Geometry is computed once per (H, W, grid) on the host in float64 and
// cached on the device as a look-up table: per polar sample the integer base
// pixel (x0, y0) = floor(x), floor(y) (or the nearest pixel) and the float32
// fractions (x - x0, y - y0). The kernel then only gathers and blends, so the
// float32 device path never recomputes cos/sin.
//
// Kernel layout: one workgroup per pattern, 8 waves; wave w owns polar rows
// w, w + 8, ...; lane l owns columns l, l + 64, ... of the row, so the polar
// writes are coalesced along theta. Row sums (profile) are reduced across the
// wave in float64; the float64 sum of squares is reduced wave by wave and
// then across waves in a fixed order, so norms are bit-reproducible.
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "tm_device.h"
#include "tm_internal.h"

namespace {

struct LutKey {
    int device, H, W, R, n_theta, interp;
    double r0, dr, cx, cy;
    bool operator<(const LutKey& o) const {
        return std::tie(device, H, W, R, n_theta, interp, r0, dr, cx, cy) <
               std::tie(o.device, o.H, o.W, o.R, o.n_theta, o.interp, o.r0, o.dr, o.cx, o.cy);
    }
};

struct Lut {
    short2* xy = nullptr;   // [R * n_theta] base pixel (x0, y0)
    float2* f = nullptr;    // [R * n_theta] fractions (fx, fy)
};

std::mutex g_lut_mu;
std::map<LutKey, Lut> g_luts;

int get_lut(const LutKey& key, hipStream_t s, Lut& out) {
    std::lock_guard<std::mutex> lock(g_lut_mu);
    auto it = g_luts.find(key);
    if (it != g_luts.end()) { out = it->second; return TM_OK; }
    const size_t n = static_cast<size_t>(key.R) * key.n_theta;
    std::vector<short2> xy(n);
    std::vector<float2> f(n);
    const double two_pi = 2.0 * M_PI;
    for (int j = 0; j < key.R; ++j) {
        const double r = key.r0 + key.dr * j;
        for (int k = 0; k < key.n_theta; ++k) {
            const double th = two_pi * k / key.n_theta;
            const double x = key.cx + r * std::cos(th);
            const double y = key.cy + r * std::sin(th);
            double x0, y0, fx, fy;
            if (key.interp == 1) {
                x0 = std::floor(x); y0 = std::floor(y);
                fx = x - x0; fy = y - y0;
            } else {
                x0 = std::nearbyint(x); y0 = std::nearbyint(y);
                fx = 0.0; fy = 0.0;
            }
            // samples far outside the image read nothing: clamp to a
            // position whose four taps are all out of range
            x0 = std::fmin(std::fmax(x0, -2.0), 32767.0);
            y0 = std::fmin(std::fmax(y0, -2.0), 32767.0);
            xy[static_cast<size_t>(j) * key.n_theta + k] =
                make_short2(static_cast<short>(x0), static_cast<short>(y0));
            f[static_cast<size_t>(j) * key.n_theta + k] =
                make_float2(static_cast<float>(fx), static_cast<float>(fy));
        }
    }
    Lut L;
    hipError_t e = hipMalloc(&L.xy, n * sizeof(short2));
    if (e == hipSuccess) e = hipMalloc(&L.f, n * sizeof(float2));
    if (e != hipSuccess) {
        hipFree(L.xy);
        hipFree(L.f);
        tmlib::set_error("polar LUT allocation failed: %s", hipGetErrorString(e));
        return TM_ENOMEM;
    }
    TM_HIP(hipMemcpyAsync(L.xy, xy.data(), n * sizeof(short2), hipMemcpyHostToDevice, s));
    TM_HIP(hipMemcpyAsync(L.f, f.data(), n * sizeof(float2), hipMemcpyHostToDevice, s));
    TM_HIP(hipStreamSynchronize(s));   // host staging must outlive the copies
    g_luts[key] = L;
    out = L;
    return TM_OK;
}

template <typename Tin>
__device__ __forceinline__ float tap(const Tin* __restrict__ img, int H, int W, int x, int y,
                                     bool pw, float gamma, float sub) {
    if (x < 0 || x >= W || y < 0 || y >= H) return 0.0f;   // zero padding
    float v = static_cast<float>(img[y * W + x]);
    if (pw) v = powf(fmaxf(v, 0.0f), gamma);
    return v - sub;
}

constexpr int kPolarThreads = 512;

template <typename Tin>
__global__ void __launch_bounds__(kPolarThreads)
polar_kernel(const Tin* __restrict__ patterns, int B, int H, int W,
             const short2* __restrict__ lut_xy, const float2* __restrict__ lut_f, int R,
             int n_theta, float gamma, float sub, float* __restrict__ polar,
             double* __restrict__ norm_out, float* __restrict__ prof_out) {
    __shared__ double partial[kPolarThreads / 64];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = tmlib::uniform(threadIdx.x >> 6);
    const int nw = kPolarThreads / 64;
    const bool pw = gamma != 1.0f;
    const Tin* img = patterns + static_cast<size_t>(b) * H * W;
    float* out = polar + static_cast<size_t>(b) * R * n_theta;
    double sq = 0.0;
    for (int j = wave; j < R; j += nw) {
        double rs = 0.0;
        for (int k = lane; k < n_theta; k += 64) {
            const int i = j * n_theta + k;
            const short2 p = lut_xy[i];
            const float2 fr = lut_f[i];
            const int x0 = p.x, y0 = p.y;
            const float fx = fr.x, fy = fr.y;
            const float p00 = tap(img, H, W, x0, y0, pw, gamma, sub);
            const float p01 = tap(img, H, W, x0 + 1, y0, pw, gamma, sub);
            const float p10 = tap(img, H, W, x0, y0 + 1, pw, gamma, sub);
            const float p11 = tap(img, H, W, x0 + 1, y0 + 1, pw, gamma, sub);
            const float gx = 1.0f - fx, gy = 1.0f - fy;
            const float v = gx * gy * p00 + fx * gy * p01 + gx * fy * p10 + fx * fy * p11;
            out[i] = v;
            rs += static_cast<double>(v);
            sq += static_cast<double>(v) * static_cast<double>(v);
        }
        rs = tmlib::wave_sum(rs);
        if (prof_out && lane == 0) prof_out[static_cast<size_t>(j) * B + b] = static_cast<float>(rs);
    }
    sq = tmlib::wave_sum(sq);
    if (lane == 0) partial[wave] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += partial[w];
        norm_out[b] = sqrt(s);
    }
}

}  // namespace

extern "C" int tm_polar_transform(const void* patterns, tm_dtype dtype, int32_t B, int32_t H,
                                  int32_t W, const tm_polar_grid* grid, float gamma,
                                  float subtract, float* polar_out, double* norm_out,
                                  float* profile_out, void* hip_stream) {
    tmlib::clear_error();
    if (int r = tmlib::validate_grid(grid)) return r;
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (H < 1 || W < 1 || H > 32767 || W > 32767) { tmlib::set_error("H=%d, W=%d outside [1, 32767]", H, W); return TM_EINVAL; }
    if (dtype != TM_U16 && dtype != TM_F32) { tmlib::set_error("unknown dtype %d", static_cast<int>(dtype)); return TM_EINVAL; }
    if (!(gamma > 0.0f) || !std::isfinite(gamma) || !std::isfinite(subtract)) {
        tmlib::set_error("gamma must be positive and finite, subtract finite");
        return TM_EINVAL;
    }
    if (grid->interp != 0 && grid->interp != 1) { tmlib::set_error("interp=%d must be 0 or 1", grid->interp); return TM_EINVAL; }
    if (!std::isfinite(grid->cx) || !std::isfinite(grid->cy)) { tmlib::set_error("centre must be finite"); return TM_EINVAL; }
    if (B == 0) return TM_OK;
    if (!patterns || !polar_out || !norm_out) { tmlib::set_error("patterns, polar_out and norm_out must be non-NULL"); return TM_EINVAL; }
    if (int r = tmlib::require_device()) return r;
    int dev = 0;
    TM_HIP(hipGetDevice(&dev));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    LutKey key{dev, H, W, grid->R, grid->n_theta, grid->interp, grid->r0, grid->dr, grid->cx, grid->cy};
    Lut lut;
    if (int r = get_lut(key, s, lut)) return r;
    if (dtype == TM_F32) {
        polar_kernel<float><<<B, kPolarThreads, 0, s>>>(
            static_cast<const float*>(patterns), B, H, W, lut.xy, lut.f, grid->R, grid->n_theta,
            gamma, subtract, polar_out, norm_out, profile_out);
    } else {
        polar_kernel<uint16_t><<<B, kPolarThreads, 0, s>>>(
            static_cast<const uint16_t*>(patterns), B, H, W, lut.xy, lut.f, grid->R,
            grid->n_theta, gamma, subtract, polar_out, norm_out, profile_out);
    }
    TM_HIP(hipGetLastError());
    return TM_OK;
}
