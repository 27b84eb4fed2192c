// Mask of the dominant phase's reflections for two-stage indexing (Section 4.3,
// custom indexation procedures: average all patterns, threshold the average,
// erode and dilate to drop small features and cover the peak tails; the mask
// then multiplies every pattern before the precipitate library is matched).
//
//   bright = mean_b(pattern_b) > threshold              (float64 per pixel)
//   bright = dilate^n_open(erode^n_open(bright))         (3x3 square, outside
//   bright = dilate^n_grow(bright)                        the image = not set)
//   mask   = bright ? 0 : 1                              (float32)
//
// The batch mean is a two-pass reduction in a fixed order (per-chunk sums,
// then the chunks in order), so the mask is reproducible.
#include <algorithm>
#include <cmath>

#include "tm_internal.h"

namespace {

constexpr int kMaskThreads = 256;
constexpr int kMaxChunks = 64;

template <typename Tin>
__global__ void __launch_bounds__(kMaskThreads)
chunk_sums(const Tin* __restrict__ patterns, int B, int HW, int n_chunks,
           double* __restrict__ partial) {
    const int p = blockIdx.x * kMaskThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= HW) return;
    const int b0 = static_cast<int>(static_cast<long long>(B) * c / n_chunks);
    const int b1 = static_cast<int>(static_cast<long long>(B) * (c + 1) / n_chunks);
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += static_cast<double>(patterns[static_cast<size_t>(b) * HW + p]);
    partial[static_cast<size_t>(c) * HW + p] = s;
}

__global__ void __launch_bounds__(kMaskThreads)
mean_threshold(const double* __restrict__ partial, int HW, int n_chunks, int B,
               double threshold, uint8_t* __restrict__ bright) {
    const int p = blockIdx.x * kMaskThreads + threadIdx.x;
    if (p >= HW) return;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += partial[static_cast<size_t>(c) * HW + p];
    bright[p] = (s / B > threshold) ? 1 : 0;
}

// One erosion (dilate == false) or dilation of a binary image, 3x3 square.
__global__ void __launch_bounds__(kMaskThreads)
morph(const uint8_t* __restrict__ in, int H, int W, bool dilate, uint8_t* __restrict__ out) {
    const int p = blockIdx.x * kMaskThreads + threadIdx.x;
    if (p >= H * W) return;
    const int y = p / W, x = p - y * W;
    bool any = false, all = true;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int yy = y + dy, xx = x + dx;
            const bool v = yy >= 0 && yy < H && xx >= 0 && xx < W && in[yy * W + xx];
            any |= v;
            all &= v;
        }
    out[p] = dilate ? any : all;
}

__global__ void __launch_bounds__(kMaskThreads)
to_mask(const uint8_t* __restrict__ bright, int HW, float* __restrict__ mask) {
    const int p = blockIdx.x * kMaskThreads + threadIdx.x;
    if (p < HW) mask[p] = bright[p] ? 0.0f : 1.0f;
}

}  // namespace

extern "C" int tm_mask_from_mean(const void* patterns, tm_dtype dtype, int32_t B, int32_t H,
                                 int32_t W, double threshold, int32_t n_open, int32_t n_grow,
                                 float* mask_out, void* hip_stream) {
    tmlib::clear_error();
    if (B < 1) { tmlib::set_error("B=%d < 1", B); return TM_EINVAL; }
    if (H < 1 || W < 1 || H > 32767 || W > 32767) { tmlib::set_error("H=%d, W=%d outside [1, 32767]", H, W); return TM_EINVAL; }
    if (dtype != TM_U16 && dtype != TM_F32) { tmlib::set_error("unknown dtype %d", static_cast<int>(dtype)); return TM_EINVAL; }
    if (n_open < 0 || n_grow < 0 || n_open > 64 || n_grow > 64) {
        tmlib::set_error("n_open=%d, n_grow=%d outside [0, 64]", n_open, n_grow);
        return TM_EINVAL;
    }
    if (!std::isfinite(threshold)) { tmlib::set_error("threshold must be finite"); return TM_EINVAL; }
    if (!patterns || !mask_out) { tmlib::set_error("patterns and mask_out must be non-NULL"); return TM_EINVAL; }
    if (int r = tmlib::require_device()) return r;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int HW = H * W;
    const int n_chunks = std::min(B, kMaxChunks);
    double* partial = nullptr;
    uint8_t* buf = nullptr;
    TM_HIP(hipMallocAsync(reinterpret_cast<void**>(&partial),
                          static_cast<size_t>(n_chunks) * HW * sizeof(double), s));
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&buf), 2 * static_cast<size_t>(HW), s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(partial, s);
        return tmlib::hip_fail(e, "hipMallocAsync");
    }
    const dim3 grid1((HW + kMaskThreads - 1) / kMaskThreads);
    if (dtype == TM_F32)
        hipLaunchKernelGGL(chunk_sums<float>, dim3(grid1.x, n_chunks), dim3(kMaskThreads), 0, s,
                           static_cast<const float*>(patterns), B, HW, n_chunks, partial);
    else
        hipLaunchKernelGGL(chunk_sums<uint16_t>, dim3(grid1.x, n_chunks), dim3(kMaskThreads), 0, s,
                           static_cast<const uint16_t*>(patterns), B, HW, n_chunks, partial);
    hipLaunchKernelGGL(mean_threshold, grid1, dim3(kMaskThreads), 0, s, partial, HW, n_chunks, B,
                       threshold, buf);
    uint8_t* cur = buf;
    uint8_t* nxt = buf + HW;
    auto step = [&](bool dilate) {
        hipLaunchKernelGGL(morph, grid1, dim3(kMaskThreads), 0, s, cur, H, W, dilate, nxt);
        std::swap(cur, nxt);
    };
    for (int i = 0; i < n_open; ++i) step(false);
    for (int i = 0; i < n_open; ++i) step(true);
    for (int i = 0; i < n_grow; ++i) step(true);
    hipLaunchKernelGGL(to_mask, grid1, dim3(kMaskThreads), 0, s, cur, HW, mask_out);
    int r = TM_OK;
    e = hipGetLastError();
    if (e != hipSuccess) r = tmlib::hip_fail(e, "mask kernel launch");
    (void)hipFreeAsync(partial, s);
    (void)hipFreeAsync(buf, s);
    return r;
}
