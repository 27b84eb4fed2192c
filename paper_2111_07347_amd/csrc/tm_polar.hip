// tm_polar_transform: intensity transform, polar resampling about the
// direct-beam centre, image norms and azimuthal profiles (Section 2.2 and
// Fig. 2 c for the polar image; Eq. (1) for the image norm; Fig. 3 for the
// azimuthal integral used by the pre-filter).
//
// Sample coordinates are formed in float64 on the device from per-column
// cos/sin tables built on the host (x = cx + r_j cos theta_k with separately
// rounded multiply and add, bit-identical to the host's computation), then
// split into the base pixel and float32 fractions; the float32 path never
// evaluates trigonometry.
//
// Kernel layout: one workgroup per pattern, 16 waves (two per CU: at most 64
// registers per lane). The polar grid is cut
// into blocks (angular sectors, and radial bands if needed) whose bilinear
// tap footprint, clipped to the image plus a one-pixel zero ring, fits the
// LDS budget; for a centred grid these are the four quadrants. Per block the
// footprint is staged into LDS with coalesced row loads, the intensity
// transform applied once per pixel and out-of-image pixels set to zero, so
// the tap reads need no bounds checks. Half-waves own polar rows and their
// lanes consecutive columns, so the polar writes are coalesced along theta.
// Each lane accumulates float32 partial row sums (profile; a dozen samples
// per lane and row) and float64 squares (norm) in registers across blocks;
// rows are reduced once per half-wave (in float64) and the squares per wave
// and then across waves in a fixed order, so norms and profiles are
// bit-reproducible.
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

// One block of the polar grid: rows [j0, j1) x columns [k0, k1), with the
// footprint box [x_lo, x_lo + bw) x [y_lo, y_lo + bh) staged in LDS with a
// row pitch >= bw chosen so that a wave's taps along an arc spread over the
// LDS banks.
struct PolarBlock {
    int j0, j1, k0, k1;
    int x_lo, y_lo, bw, bh, pitch;
};

struct Lut {
    PolarBlock* blocks = nullptr;   // device [n_blocks]
    double2* cs = nullptr;          // device [n_theta] (cos theta_k, sin theta_k)
    int n_blocks = 0;
    int lds_floats = 0;             // max over blocks of bw * bh + bw + 2
};

// LDS budget for one block's footprint (two workgroups per CU).
constexpr size_t kBoxBytes = 76 * 1024;

std::mutex g_lut_mu;
std::map<LutKey, Lut> g_luts;

// Base pixel of a sample, computed exactly as the kernel does.
struct Sample { int x0, y0; };

// LDS row pitch for a block: among bw .. bw + 31 (multiples of step) the one that minimises the
// mean worst-bank load of the four taps over each half-wave of consecutive
// columns (32 banks of 4 bytes; equal addresses broadcast), within the LDS
// budget.
template <typename BaseFn, typename InFn>
int choose_pitch(const PolarBlock& B, BaseFn base_pixel, InFn inside, size_t max_floats, int step) {
    int best_p = B.bw;
    double best_c = 1e30;
    std::vector<int> addr;
    for (int p = B.bw; p < B.bw + 32; p += step) {
        if (static_cast<size_t>(p) * B.bh + p + 2 > max_floats) break;
        double cost = 0.0;
        for (int j = B.j0; j < B.j1; ++j) {
            for (int k = B.k0; k < B.k1; k += 32) {
                const int k_end = std::min(B.k1, k + 32);
                for (int tap = 0; tap < 4; ++tap) {
                    addr.clear();
                    for (int kk = k; kk < k_end; ++kk) {
                        const Sample q = base_pixel(j, kk);
                        if (!inside(q)) continue;
                        addr.push_back((q.y0 - B.y_lo + (tap >> 1)) * p + (q.x0 - B.x_lo + (tap & 1)));
                    }
                    std::sort(addr.begin(), addr.end());
                    addr.erase(std::unique(addr.begin(), addr.end()), addr.end());
                    int bank[32] = {0}, worst = 0;
                    for (int a : addr) worst = std::max(worst, ++bank[a & 31]);
                    cost += worst;
                }
            }
        }
        if (cost < best_c) { best_c = cost; best_p = p; }
    }
    return best_p;
}

int get_lut(const LutKey& key, hipStream_t s, Lut& out) {
    std::lock_guard<std::mutex> lock(g_lut_mu);
    auto it = g_luts.find(key);
    if (it != g_luts.end()) { out = it->second; return TM_OK; }
    const int R = key.R, nt = key.n_theta;
    std::vector<double2> cs(nt);
    const double two_pi = 2.0 * M_PI;
    for (int k = 0; k < nt; ++k) {
        const double th = two_pi * k / nt;
        cs[k] = make_double2(std::cos(th), std::sin(th));
    }
    auto base_pixel = [&](int j, int k) {
        const double r = key.r0 + key.dr * j;
        const double x = key.cx + r * cs[k].x;
        const double y = key.cy + r * cs[k].y;
        double x0 = key.interp == 1 ? std::floor(x) : std::nearbyint(x);
        double y0 = key.interp == 1 ? std::floor(y) : std::nearbyint(y);
        x0 = std::fmin(std::fmax(x0, -4.0), 40000.0);
        y0 = std::fmin(std::fmax(y0, -4.0), 40000.0);
        return Sample{static_cast<int>(x0), static_cast<int>(y0)};
    };
    // a sample contributes iff its 2x2 footprint touches the image
    auto inside = [&](const Sample& q) {
        return q.x0 >= -1 && q.x0 <= key.W - 1 && q.y0 >= -1 && q.y0 <= key.H - 1;
    };
    // smallest sector / band split whose every footprint box fits the budget
    std::vector<PolarBlock> blocks;
    const size_t max_floats = kBoxBytes / sizeof(float);
    // widths divisible by 4: boxes start and end on aligned 4-pixel groups and
    // row pitches are multiples of 4 floats (16-byte aligned LDS rows)
    const bool aligned = (key.W & 3) == 0;
    int lds_floats = 0;
    for (int sk = 4, sj = 1;;) {
        blocks.clear();
        lds_floats = 0;
        bool fits = true;
        for (int bj = 0; bj < sj && fits; ++bj) {
            for (int bk = 0; bk < sk && fits; ++bk) {
                PolarBlock B{};
                B.j0 = R * bj / sj; B.j1 = R * (bj + 1) / sj;
                B.k0 = nt * bk / sk; B.k1 = nt * (bk + 1) / sk;
                if (B.j0 == B.j1 || B.k0 == B.k1) continue;
                int xl = INT32_MAX, xh = INT32_MIN, yl = INT32_MAX, yh = INT32_MIN;
                for (int j = B.j0; j < B.j1; ++j)
                    for (int k = B.k0; k < B.k1; ++k) {
                        const Sample q = base_pixel(j, k);
                        if (!inside(q)) continue;
                        xl = std::min(xl, q.x0); xh = std::max(xh, q.x0 + 1);
                        yl = std::min(yl, q.y0); yh = std::max(yh, q.y0 + 1);
                    }
                if (xl > xh) { xl = xh = yl = yh = 0; }   // block entirely outside
                if (aligned) {
                    // widen to whole aligned 4-pixel groups (xl >= -4): staged
                    // with one 16-byte LDS store per group
                    xl = (xl + 4) / 4 * 4 - 4;
                    xh = (xh + 4) / 4 * 4 - 1;
                }
                B.x_lo = xl; B.y_lo = yl; B.bw = xh - xl + 1; B.bh = yh - yl + 1;
                B.pitch = choose_pitch(B, base_pixel, inside, max_floats, aligned ? 4 : 1);
                const size_t need = static_cast<size_t>(B.pitch) * B.bh + B.pitch + 2;
                if (need > max_floats) fits = false;
                lds_floats = std::max(lds_floats, static_cast<int>(need));
                blocks.push_back(B);
            }
        }
        if (fits) break;
        if (sk < nt / 8) sk *= 2; else if (sj < R) sj *= 2;
        else { tmlib::set_error("polar grid too large for the LDS blocking"); return TM_EUNSUPPORTED; }
    }
    Lut L;
    L.n_blocks = static_cast<int>(blocks.size());
    L.lds_floats = lds_floats;
    hipError_t err = hipMalloc(&L.blocks, blocks.size() * sizeof(PolarBlock));
    if (err == hipSuccess) err = hipMalloc(&L.cs, nt * sizeof(double2));
    if (err != hipSuccess) {
        (void)hipFree(L.blocks); (void)hipFree(L.cs);
        tmlib::set_error("polar table allocation failed: %s", hipGetErrorString(err));
        return TM_ENOMEM;
    }
    TM_HIP(hipMemcpyAsync(L.blocks, blocks.data(), blocks.size() * sizeof(PolarBlock), hipMemcpyHostToDevice, s));
    TM_HIP(hipMemcpyAsync(L.cs, cs.data(), nt * sizeof(double2), hipMemcpyHostToDevice, s));
    TM_HIP(hipStreamSynchronize(s));   // host staging must outlive the copies
    g_luts[key] = L;
    out = L;
    return TM_OK;
}

constexpr int kPolarThreads = 1024;
constexpr int kPolarWaves = kPolarThreads / 64;
constexpr int kRowsPerStep = 2 * kPolarWaves;   // each half-wave owns one row per step
constexpr int kRowSteps = 4;                    // rows held per half-wave: a group of 128
constexpr int kRowGroup = kRowsPerStep * kRowSteps;
constexpr int kStageUnroll = 4;                 // independent loads in flight per thread
constexpr int kVecUnroll = 2;                   // 4-pixel groups in flight per thread

// Sum over the 32 lanes of a half-wave (fixed tree, identical in every lane
// of the half).
__device__ __forceinline__ double half_wave_sum(double v) {
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) v += __shfl_xor(v, m, 32);
    return v;
}

// One workgroup per pattern. Rows are processed in groups of 128: for each
// group every block's footprint is staged and its samples of the group's rows
// are resampled. Half-wave h of wave w owns rows g0 + 32 i + 2 w + h (i < 4)
// and its 32 lanes walk the block's columns, so stores are 128-byte runs and
// each lane keeps float32 partial row sums in registers across blocks; a row
// is reduced across its half-wave once, in float64. With a row map, polar row j is
// written to output row row_map[j] (skipped when negative); norms and
// profiles always cover all R rows.
template <typename Tin, bool BILINEAR>
__global__ void __launch_bounds__(kPolarThreads, 8)   // two workgroups per CU
polar_kernel(const Tin* __restrict__ patterns, int B, int H, int W,
             const PolarBlock* __restrict__ blocks, int n_blocks,
             const double2* __restrict__ cs, double r0, double dr, double cx, double cy,
             int R, int n_theta, float gamma, float sub, const float* __restrict__ mask,
             const int* __restrict__ row_map, int out_rows, float* __restrict__ polar,
             double* __restrict__ norm_out, float* __restrict__ prof_out) {
    extern __shared__ double smem[];
    double* partial = smem;                                   // [waves]
    float* box = reinterpret_cast<float*>(smem + kPolarWaves);
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int half = lane >> 5;
    const int col = lane & 31;
    const int wave = tmlib::uniform(tid >> 6);
    const bool pw = gamma != 1.0f;
    const Tin* img = patterns + static_cast<size_t>(b) * H * W;
    float* out = polar + static_cast<size_t>(b) * out_rows * n_theta;
    double sq = 0.0;
    for (int g0 = 0; g0 < R; g0 += kRowGroup) {
        float rs[kRowSteps];   // per-lane partial row sums (a dozen samples each)
        int orow[kRowSteps];   // output row of this lane's polar rows (-1: not written)
#pragma unroll
        for (int i = 0; i < kRowSteps; ++i) {
            rs[i] = 0.0f;
            const int j = g0 + i * kRowsPerStep + 2 * wave + half;
            const int m = j < R ? (row_map ? row_map[j] : j) : -1;
            orow[i] = (m >= 0 && m < out_rows) ? m : -1;   // entries out of range: skipped
        }
        for (int bi = 0; bi < n_blocks; ++bi) {
            const PolarBlock blk = blocks[bi];
            if (blk.j1 <= g0 || blk.j0 >= g0 + kRowGroup) continue;   // uniform
            const int bw = blk.bw, pitch = blk.pitch, total = blk.bw * blk.bh;
            __syncthreads();
            // stage the footprint (transform once per pixel, zero outside the
            // image). Image widths divisible by 4: aligned groups of 4 pixels
            // (one 16- or 8-byte load each, several in flight per thread);
            // otherwise element i = tid + 1024 m walks the box row-major.
            if ((W & 3) == 0) {
                // the box starts and ends on aligned 4-pixel groups (the
                // table is built that way for these widths) and its pitch is
                // a multiple of 4: group g = row g / ng, column g % ng is one
                // 16- or 8-byte load and one 16-byte LDS store
                const int ng = bw >> 2;
                const int ntot = ng * blk.bh;
                // row of g as trunc((g + 0.5) * fl(1 / ng)): the relative error
                // of the product is below 2^-23, so the quotient is exact
                // while g + 0.5 < 2^22 (the box holds under 2^15 groups)
                const float inv_ng = 1.0f / static_cast<float>(ng);
                for (int g0 = tid; g0 < ntot; g0 += kPolarThreads * kVecUnroll) {
                    float4 v[kVecUnroll];
                    int dst[kVecUnroll];
#pragma unroll
                    for (int u = 0; u < kVecUnroll; ++u) {
                        const int g = g0 + u * kPolarThreads;
                        const int yy = static_cast<int>((static_cast<float>(g) + 0.5f) * inv_ng);
                        const int cg = g - yy * ng;
                        const int y = blk.y_lo + yy, xs = blk.x_lo + 4 * cg;
                        dst[u] = g < ntot ? yy * pitch + 4 * cg : -1;
                        const bool in = g < ntot && y >= 0 && y < H && xs >= 0 && xs < W;
                        v[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                        if (in) {
                            const Tin* q = img + static_cast<size_t>(y) * W + xs;
                            float t[4];
                            if constexpr (sizeof(Tin) == 4) {
                                const float4 r = *reinterpret_cast<const float4*>(q);
                                t[0] = r.x; t[1] = r.y; t[2] = r.z; t[3] = r.w;
                            } else {
                                const ushort4 r = *reinterpret_cast<const ushort4*>(q);
                                t[0] = r.x; t[1] = r.y; t[2] = r.z; t[3] = r.w;
                            }
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                if (pw) t[e] = powf(fmaxf(t[e], 0.0f), gamma);
                                t[e] -= sub;
                            }
                            if (mask) {
                                const float4 m = *reinterpret_cast<const float4*>(
                                    mask + static_cast<size_t>(y) * W + xs);
                                t[0] *= m.x; t[1] *= m.y; t[2] *= m.z; t[3] *= m.w;
                            }
                            v[u] = make_float4(t[0], t[1], t[2], t[3]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kVecUnroll; ++u)
                        if (dst[u] >= 0) *reinterpret_cast<float4*>(box + dst[u]) = v[u];
                }
            } else {
                const int step_y = kPolarThreads / bw, step_x = kPolarThreads - step_y * bw;
                int yy = tid / bw, xx = tid - yy * bw;
                for (int base = tid; base < total; base += kPolarThreads * kStageUnroll) {
                    float v[kStageUnroll];
                    int dst[kStageUnroll], midx[kStageUnroll];
                    bool in[kStageUnroll];
#pragma unroll
                    for (int u = 0; u < kStageUnroll; ++u) {
                        const int y = blk.y_lo + yy, x = blk.x_lo + xx;
                        const bool live = base + u * kPolarThreads < total;
                        in[u] = live && y >= 0 && y < H && x >= 0 && x < W;
                        dst[u] = live ? yy * pitch + xx : -1;
                        midx[u] = y * W + x;
                        v[u] = in[u] ? static_cast<float>(img[y * W + x]) : 0.0f;
                        xx += step_x;
                        yy += step_y;
                        if (xx >= bw) { xx -= bw; ++yy; }
                    }
#pragma unroll
                    for (int u = 0; u < kStageUnroll; ++u) {
                        float t = v[u];
                        if (in[u]) {
                            if (pw) t = powf(fmaxf(t, 0.0f), gamma);
                            t -= sub;
                            if (mask) t *= mask[midx[u]];
                        }
                        if (dst[u] >= 0) box[dst[u]] = t;
                    }
                }
            }
            const int zero_slot = pitch * blk.bh;   // pitch + 2 zeros follow the box
            for (int i = tid; i < pitch + 2; i += kPolarThreads) box[zero_slot + i] = 0.0f;
            __syncthreads();
            const int nk = blk.k1 - blk.k0;
            const int bwm = max(bw - 2, 0), bhm = max(blk.bh - 2, 0);
            for (int c0 = 0; c0 < nk; c0 += 32) {
                const int kk = c0 + col;
                const bool col_ok = kk < nk;
                const double2 c = cs[blk.k0 + (col_ok ? kk : 0)];
#pragma unroll
                for (int i = 0; i < kRowSteps; ++i) {
                    const int j = g0 + i * kRowsPerStep + 2 * wave + half;
                    if (!(col_ok && j >= blk.j0 && j < blk.j1)) continue;
                    // x = cx + r cos, y = cy + r sin, multiply and add rounded
                    // separately (no FMA contraction), exactly as the host
                    // computed the footprint
                    double r, x, y;
                    {
#pragma clang fp contract(off)
                        r = r0 + dr * static_cast<double>(j);
                        x = cx + r * c.x;
                        y = cy + r * c.y;
                    }
                    const double xf = BILINEAR ? floor(x) : rint(x);
                    const double yf = BILINEAR ? floor(y) : rint(y);
                    // |x|, |y| < 2^21 (checked on the host), so the conversions are exact
                    const int ix = static_cast<int>(xf) - blk.x_lo;
                    const int iy = static_cast<int>(yf) - blk.y_lo;
                    // the box holds exactly the 2x2 footprints of this block's samples
                    // that touch the image (a one-pixel zero ring outside it): a sample
                    // is in the image's support iff its base pixel lies in the box
                    // minus its last row and column; every read stays in the box
                    const bool in = static_cast<unsigned>(ix) <= static_cast<unsigned>(bwm) &&
                                    static_cast<unsigned>(iy) <= static_cast<unsigned>(bhm);
                    const int o = in ? __mul24(iy, pitch) + ix : zero_slot;
                    float v;
                    if (BILINEAR) {
                        // outside the support all four taps read zeros, so the
                        // (finite) fractions need no masking
                        const float fx = static_cast<float>(x - xf);
                        const float fy = static_cast<float>(y - yf);
                        const float p00 = box[o], p01 = box[o + 1];
                        const float p10 = box[o + pitch], p11 = box[o + pitch + 1];
                        // two interpolations along x, then one along y
                        const float a = fmaf(fx, p01 - p00, p00);
                        const float e = fmaf(fx, p11 - p10, p10);
                        v = fmaf(fy, e - a, a);
                    } else {
                        v = box[o];
                    }
                    if (orow[i] >= 0)
                        out[static_cast<unsigned>(orow[i] * n_theta + blk.k0 + kk)] = v;
                    const double vd = static_cast<double>(v);
                    rs[i] += v;
                    sq += vd * vd;
                }
            }
        }
        // one reduction per row of the group
#pragma unroll
        for (int i = 0; i < kRowSteps; ++i) {
            const double t = half_wave_sum(static_cast<double>(rs[i]));
            const int j = g0 + i * kRowsPerStep + 2 * wave + half;
            if (prof_out && col == 0 && j < R) prof_out[static_cast<size_t>(j) * B + b] = static_cast<float>(t);
        }
    }
    sq = tmlib::wave_sum(sq);
    if (lane == 0) partial[wave] = sq;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < kPolarWaves; ++w) s += partial[w];
        norm_out[b] = sqrt(s);
    }
}

}  // namespace

namespace {

int polar_impl(const void* patterns, tm_dtype dtype, int32_t B, int32_t H, int32_t W,
               const tm_polar_grid* grid, float gamma, float subtract, const float* mask,
               const int32_t* row_map, int32_t out_rows, float* polar_out, double* norm_out,
               float* profile_out, void* hip_stream) {
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
    // sample coordinates must stay far inside the int range (|x|, |y| < 2^21)
    const double lim = 1048576.0;
    if (std::fabs(grid->cx) > lim || std::fabs(grid->cy) > lim ||
        std::fabs(grid->r0) + grid->dr * grid->R > lim) {
        tmlib::set_error("centre and radii must lie within +-2^20 pixels");
        return TM_EINVAL;
    }
    if (B == 0) return TM_OK;
    if (!patterns || !polar_out || !norm_out) { tmlib::set_error("patterns, polar_out and norm_out must be non-NULL"); return TM_EINVAL; }
    if (int r = tmlib::require_device()) return r;
    int dev = 0;
    TM_HIP(hipGetDevice(&dev));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    LutKey key{dev, H, W, grid->R, grid->n_theta, grid->interp, grid->r0, grid->dr, grid->cx, grid->cy};
    Lut lut;
    if (int r = get_lut(key, s, lut)) return r;
    const size_t lds = static_cast<size_t>(kPolarWaves) * sizeof(double) +
                       static_cast<size_t>(lut.lds_floats) * sizeof(float);
    auto launch = [&](auto fn, auto ptr) -> int {
        TM_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        hipLaunchKernelGGL(fn, dim3(B), dim3(kPolarThreads), lds, s, ptr, B, H, W, lut.blocks,
                           lut.n_blocks, lut.cs, grid->r0, grid->dr, grid->cx, grid->cy, grid->R,
                           grid->n_theta, gamma, subtract, mask, row_map, out_rows, polar_out,
                           norm_out, profile_out);
        return TM_OK;
    };
    int r = TM_OK;
    if (dtype == TM_F32) {
        const float* p = static_cast<const float*>(patterns);
        r = grid->interp ? launch(polar_kernel<float, true>, p) : launch(polar_kernel<float, false>, p);
    } else {
        const uint16_t* p = static_cast<const uint16_t*>(patterns);
        r = grid->interp ? launch(polar_kernel<uint16_t, true>, p) : launch(polar_kernel<uint16_t, false>, p);
    }
    if (r) return r;
    TM_HIP(hipGetLastError());
    return TM_OK;
}

}  // namespace

extern "C" int tm_polar_transform(const void* patterns, tm_dtype dtype, int32_t B, int32_t H,
                                  int32_t W, const tm_polar_grid* grid, float gamma,
                                  float subtract, float* polar_out, double* norm_out,
                                  float* profile_out, void* hip_stream) {
    tmlib::clear_error();
    return polar_impl(patterns, dtype, B, H, W, grid, gamma, subtract, nullptr, nullptr,
                      grid ? grid->R : 0, polar_out, norm_out, profile_out, hip_stream);
}

extern "C" int tm_polar_transform_rows(const void* patterns, tm_dtype dtype, int32_t B,
                                       int32_t H, int32_t W, const tm_polar_grid* grid,
                                       float gamma, float subtract, const float* mask,
                                       const int32_t* row_map, int32_t n_out_rows,
                                       float* polar_out, double* norm_out, float* profile_out,
                                       void* hip_stream) {
    tmlib::clear_error();
    if (grid && (n_out_rows < 1 || n_out_rows > grid->R)) {
        tmlib::set_error("n_out_rows=%d outside [1, R=%d]", n_out_rows, grid->R);
        return TM_EINVAL;
    }
    if (!row_map && grid && n_out_rows != grid->R) {
        tmlib::set_error("without a row map, n_out_rows must equal R");
        return TM_EINVAL;
    }
    return polar_impl(patterns, dtype, B, H, W, grid, gamma, subtract, mask, row_map,
                      n_out_rows, polar_out, norm_out, profile_out, hip_stream);
}
