// Kinematical simulation of a template library on the device (Section 2.1):
// the reciprocal lattice points up to a maximum radius, rotated by each
// orientation (phi1 = 0, Phi, phi2); the excitation error (distance to the
// Ewald sphere); spot intensity I = F F* times a shape factor of the
// excitation error; projection of the excited spots onto kx-ky.
//
//   grid_kernel      one workgroup walks the (h, k, l) box in lexicographic
//                    order, keeps 0 < |g| <= g_lim with F F* > 1e-6 (F with
//                    one constant scattering factor per atom), and appends
//                    the survivors in order (workgroup prefix sum) as
//                    (gx, gy, gz, F F*) records.
//   template_kernel  one wave per orientation (persistent grid, waves stride
//                    the orientations): lanes stride the reflections, rotate
//                    them to the sample frame g_sample = g0^T g_crystal (Bunge
//                    g0 of (0, Phi, phi2)) and keep those near the Ewald
//                    sphere (beam along -z, centre (0, 0, k)). A square-root
//                    free test |g - (0, 0, k)|^2 in ((k - s_max)^2,
//                    (k + s_max)^2) and |g_xy|^2 <= g_max^2 (slightly
//                    widened) admits a superset, appended in grid order
//                    (ballot compaction) to a wave list: the first entries in
//                    LDS, the rest in a per-wave global area. The exact
//                    s = k - |g - (0, 0, k)|, shape max(0, 1 - |s| / s_max)
//                    and projected radius tests then run on the dense list
//                    (so the square roots and the division run once per
//                    survivor, not once per 64 reflections). The wave drops
//                    spots below rel_min times the brightest, ranks the rest
//                    by (intensity desc, grid order) by counting, and writes
//                    the first max_spots, intensities divided by the
//                    brightest.
//
// float64 throughout. The work is a few dozen float64 operations per
// (orientation, reflection) pair plus the ranking of the excited spots; the
// bound is the float64 vector rate (or the spot writes for small grids).
#include <algorithm>
#include <cmath>

#include "tm_internal.h"

namespace {

constexpr int kGridThreads = 1024;
constexpr int kMaxAtoms = 32;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr int kSimWaves = 4;                 // waves per workgroup of the template kernel
constexpr int kSimThreads = 64 * kSimWaves;
constexpr int kLdsCand = 256;                // candidate entries per wave held in LDS
constexpr int kMaxBox = 1 << 20;             // (h, k, l) points the grid walk may visit

struct Crystal {
    double B[3][3];            // reciprocal basis rows b1, b2, b3 (1/Angstrom)
    double x[kMaxAtoms][3];    // fractional atom positions
    double f[kMaxAtoms];       // scattering factor per atom
    int n_atoms;
    int lim[3];                // |h|, |k|, |l| bounds of the box
    double g_lim;
};

__global__ void __launch_bounds__(kGridThreads)
grid_kernel(Crystal c, double4* __restrict__ refl, int cap, int* __restrict__ n_out) {
    __shared__ int warp_sums[kGridThreads / 64];
    __shared__ int base;
    const int nh = 2 * c.lim[0] + 1, nk = 2 * c.lim[1] + 1, nl = 2 * c.lim[2] + 1;
    const int total = nh * nk * nl;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < total; c0 += kGridThreads) {
        const int p = c0 + static_cast<int>(threadIdx.x);
        bool keep = false;
        double g[3] = {0.0, 0.0, 0.0}, f2 = 0.0;
        if (p < total) {
            const int h = p / (nk * nl) - c.lim[0];
            const int k = (p / nl) % nk - c.lim[1];
            const int l = p % nl - c.lim[2];
            if (h != 0 || k != 0 || l != 0) {
                for (int d = 0; d < 3; ++d) g[d] = h * c.B[0][d] + k * c.B[1][d] + l * c.B[2][d];
                if (sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) <= c.g_lim) {
                    double re = 0.0, im = 0.0;
                    for (int a = 0; a < c.n_atoms; ++a) {
                        const double ph = kTwoPi * (h * c.x[a][0] + k * c.x[a][1] + l * c.x[a][2]);
                        re += c.f[a] * cos(ph);
                        im += c.f[a] * sin(ph);
                    }
                    f2 = re * re + im * im;
                    keep = f2 > 1e-6;
                }
            }
        }
        // workgroup prefix sum of keep, in thread order
        const unsigned long long m = __ballot(keep);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) warp_sums[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += warp_sums[w];
        if (keep && off + before < cap) refl[off + before] = make_double4(g[0], g[1], g[2], f2);
        __syncthreads();
        if (threadIdx.x == 0) {
            int s = 0;
            for (int w = 0; w < kGridThreads / 64; ++w) s += warp_sums[w];
            base += s;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_out = min(base, cap);
}

__device__ __forceinline__ double wave_max_d(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Candidate list of one wave: entries [0, kLdsCand) in LDS, the rest in the
// wave's global overflow area.
struct CandList {
    double* li;
    int* lj;
    double* gi;
    int* gj;
    __device__ __forceinline__ void put_j(int o, int j) const {
        if (o < kLdsCand) lj[o] = j;
        else gj[o - kLdsCand] = j;
    }
    __device__ __forceinline__ void put_i(int o, double I) const {
        if (o < kLdsCand) li[o] = I;
        else gi[o - kLdsCand] = I;
    }
    __device__ __forceinline__ double I(int o) const { return o < kLdsCand ? li[o] : gi[o - kLdsCand]; }
    __device__ __forceinline__ int J(int o) const { return o < kLdsCand ? lj[o] : gj[o - kLdsCand]; }
};

__global__ void __launch_bounds__(kSimThreads)
template_kernel(const double* __restrict__ orient, int T, const double4* __restrict__ refl,
                const int* __restrict__ n_refl_p, int cap, double k, double s_max, double g_max,
                double rel_min, int max_spots, double* __restrict__ ovf_i,
                int* __restrict__ ovf_j, double* __restrict__ kx_out,
                double* __restrict__ ky_out, double* __restrict__ i_out,
                int* __restrict__ count_out) {
    __shared__ double lds_i[kSimWaves][kLdsCand];
    __shared__ int lds_j[kSimWaves][kLdsCand];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long gw = static_cast<long long>(blockIdx.x) * kSimWaves + wave;
    const long long n_waves = static_cast<long long>(gridDim.x) * kSimWaves;
    const size_t ovf = static_cast<size_t>(gw) * static_cast<size_t>(max(cap - kLdsCand, 0));
    const CandList cl{lds_i[wave], lds_j[wave], ovf_i + ovf, ovf_j + ovf};
    const int n_refl = min(*n_refl_p, cap);
    // square-root free superset of the relrod and projection tests
    const double lo = k > s_max ? (k - s_max) * (k - s_max) * (1.0 - 1e-12) : -1.0;
    const double hi = (k + s_max) * (k + s_max) * (1.0 + 1e-12);
    const double r2 = g_max * g_max * (1.0 + 1e-12);
    for (long long tl = gw; tl < T; tl += n_waves) {
        const int t = static_cast<int>(tl);
        const double Phi = orient[2 * static_cast<size_t>(t)];
        const double phi2 = orient[2 * static_cast<size_t>(t) + 1];
        double c, s, c2, s2;
        sincos(Phi, &s, &c);
        sincos(phi2, &s2, &c2);
        // crystal -> sample: transpose of Bunge g(0, Phi, phi2)
        const double m00 = c2, m01 = -s2, m02 = 0.0;
        const double m10 = s2 * c, m11 = c2 * c, m12 = -s;
        const double m20 = s2 * s, m21 = c2 * s, m22 = c;
        // 1. the cheap superset test over all reflections; survivors'
        // indices are appended in grid order
        int n_sup = 0;
        for (int j0 = 0; j0 < n_refl; j0 += 64) {
            const int j = j0 + lane;
            bool ok = false;
            if (j < n_refl) {
                const double4 r = refl[j];
                const double sx = m00 * r.x + m01 * r.y + m02 * r.z;
                const double sy = m10 * r.x + m11 * r.y + m12 * r.z;
                const double sz = m20 * r.x + m21 * r.y + m22 * r.z - k;
                const double rxy = sx * sx + sy * sy;
                const double q = rxy + sz * sz;
                ok = q > lo && q < hi && rxy <= r2;
            }
            const unsigned long long m = __ballot(ok);
            if (ok) cl.put_j(n_sup + __popcll(m & ((1ull << lane) - 1ull)), j);
            n_sup += __popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // 2. the exact tests on the dense survivor list: intensity, or -1
        // for a survivor outside the relrod or the projection radius
        double top = 0.0;
        for (int i0 = 0; i0 < n_sup; i0 += 64) {
            const int i = i0 + lane;
            if (i < n_sup) {
                const double4 r = refl[cl.J(i)];
                const double sx = m00 * r.x + m01 * r.y + m02 * r.z;
                const double sy = m10 * r.x + m11 * r.y + m12 * r.z;
                const double sz = m20 * r.x + m21 * r.y + m22 * r.z - k;
                const double rxy = sx * sx + sy * sy;
                const double q = rxy + sz * sz;
                const double err = k - sqrt(q);
                const double shape = fmax(0.0, 1.0 - fabs(err) / s_max);
                const bool ok = shape > 0.0 && sqrt(rxy) <= g_max;
                const double I = ok ? r.w * shape : -1.0;
                cl.put_i(i, I);
                top = fmax(top, I);
            }
        }
        top = wave_max_d(top);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // 3. spots at or above rel_min times the brightest, ranked by
        // (intensity desc, grid order) by counting; a counted entry has
        // I >= the lane's I >= thr >= 0, so rejected survivors (-1) never count
        const double thr = rel_min * top;
        int n_keep = 0;
        for (int i0 = 0; i0 < n_sup; i0 += 64) {
            const int i = i0 + lane;
            const bool keep = i < n_sup && cl.I(i) >= thr;
            n_keep += __popcll(__ballot(keep));
            if (!keep) continue;
            const double Ii = cl.I(i);
            int rank = 0;
            if (n_sup <= kLdsCand) {
#pragma unroll 4
                for (int q = 0; q < n_sup; ++q) {
                    const double Iq = cl.li[q];
                    rank += (Iq > Ii || (Iq == Ii && q < i)) ? 1 : 0;
                }
            } else {
                for (int q = 0; q < n_sup; ++q) {
                    const double Iq = cl.I(q);
                    rank += (Iq > Ii || (Iq == Ii && q < i)) ? 1 : 0;
                }
            }
            if (rank < max_spots) {
                const double4 r = refl[cl.J(i)];
                const size_t o = static_cast<size_t>(t) * max_spots + rank;
                kx_out[o] = m00 * r.x + m01 * r.y + m02 * r.z;
                ky_out[o] = m10 * r.x + m11 * r.y + m12 * r.z;
                i_out[o] = Ii / top;
            }
        }
        if (lane == 0) count_out[t] = min(n_keep, max_spots);
        // the list is rewritten for the next orientation
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

// 3x3 inverse (host): the real-space basis rows a_i satisfy a_i . b_j = d_ij.
bool real_basis(const double B[3][3], double A[3][3]) {
    const double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                       B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                       B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    // A = inverse(B)^T: rows of A are the columns of inverse(B)
    double inv[3][3];
    inv[0][0] = (B[1][1] * B[2][2] - B[1][2] * B[2][1]) / det;
    inv[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) / det;
    inv[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) / det;
    inv[1][0] = (B[1][2] * B[2][0] - B[1][0] * B[2][2]) / det;
    inv[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) / det;
    inv[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) / det;
    inv[2][0] = (B[1][0] * B[2][1] - B[1][1] * B[2][0]) / det;
    inv[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) / det;
    inv[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) / det;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = inv[j][i];
    return true;
}

}  // namespace

extern "C" int tm_simulate_library(const double* recip_basis, const double* atoms_frac,
                                   const double* f_atoms, int32_t n_atoms, double g_lim,
                                   const double* orientations, int32_t T, double k,
                                   double s_max, double g_max, double rel_min,
                                   int32_t max_spots, double* kx_out, double* ky_out,
                                   double* intensity_out, int32_t* count_out,
                                   void* hip_stream) {
    tmlib::clear_error();
    if (!recip_basis || !atoms_frac || !f_atoms) {
        tmlib::set_error("recip_basis, atoms_frac and f_atoms must be non-NULL");
        return TM_EINVAL;
    }
    if (n_atoms < 1 || n_atoms > kMaxAtoms) {
        tmlib::set_error("n_atoms=%d outside [1, %d]", n_atoms, kMaxAtoms);
        return TM_EINVAL;
    }
    if (T < 0) { tmlib::set_error("T=%d < 0", T); return TM_EINVAL; }
    if (max_spots < 1 || max_spots > 4096) {
        tmlib::set_error("max_spots=%d outside [1, 4096]", max_spots);
        return TM_EINVAL;
    }
    if (!(g_lim > 0.0) || !(k > 0.0) || !(s_max > 0.0) || !(g_max > 0.0) || !(rel_min >= 0.0) ||
        !std::isfinite(g_lim) || !std::isfinite(k) || !std::isfinite(s_max) ||
        !std::isfinite(g_max) || !std::isfinite(rel_min)) {
        tmlib::set_error("g_lim, k, s_max, g_max must be finite and > 0, rel_min >= 0");
        return TM_EINVAL;
    }
    if (T > 0 && (!orientations || !kx_out || !ky_out || !intensity_out || !count_out)) {
        tmlib::set_error("orientations and the outputs must be non-NULL");
        return TM_EINVAL;
    }
    Crystal c{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c.B[i][j] = recip_basis[3 * i + j];
    double A[3][3];
    if (!real_basis(c.B, A)) { tmlib::set_error("reciprocal basis is singular"); return TM_EINVAL; }
    long long box = 1;
    for (int i = 0; i < 3; ++i) {
        const double n = std::sqrt(A[i][0] * A[i][0] + A[i][1] * A[i][1] + A[i][2] * A[i][2]);
        const double lim = std::floor(g_lim * n + 1e-9);
        if (!(lim < 1024.0)) { tmlib::set_error("grid too large for g_lim=%g", g_lim); return TM_EINVAL; }
        c.lim[i] = static_cast<int>(lim);
        box *= 2 * c.lim[i] + 1;
    }
    if (box > kMaxBox) {
        tmlib::set_error("reflection grid of %lld points exceeds %d", box, kMaxBox);
        return TM_EUNSUPPORTED;
    }
    for (int a = 0; a < n_atoms; ++a) {
        for (int d = 0; d < 3; ++d) c.x[a][d] = atoms_frac[3 * a + d];
        c.f[a] = f_atoms[a];
    }
    c.n_atoms = n_atoms;
    c.g_lim = g_lim;
    // Scratch sizing: the grid points inside a slightly larger sphere bound
    // the reflection count from above (the device applies the exact radius
    // and the structure-factor test).
    long long cap = 0;
    {
        const double r2 = g_lim * g_lim * (1.0 + 1e-9);
        for (int h = -c.lim[0]; h <= c.lim[0]; ++h)
            for (int kk = -c.lim[1]; kk <= c.lim[1]; ++kk)
                for (int l = -c.lim[2]; l <= c.lim[2]; ++l) {
                    double g2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const double v = h * c.B[0][d] + kk * c.B[1][d] + l * c.B[2][d];
                        g2 += v * v;
                    }
                    cap += g2 <= r2 ? 1 : 0;
                }
        cap = std::max<long long>(cap, 1);
    }
    if (int r = tmlib::require_device()) return r;
    if (T == 0) return TM_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int dev = 0, cus = 0;
    TM_HIP(hipGetDevice(&dev));
    TM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const long long blocks = std::min<long long>((static_cast<long long>(T) + kSimWaves - 1) / kSimWaves,
                                                 static_cast<long long>(std::max(cus, 1)) * 8);
    const long long ovf_n = blocks * kSimWaves * std::max<long long>(cap - kLdsCand, 0);
    double4* refl = nullptr;
    int* n_refl = nullptr;
    double* ovf_i = nullptr;
    int* ovf_j = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&refl), static_cast<size_t>(cap) * sizeof(double4), s);
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&n_refl), sizeof(int), s);
    if (e == hipSuccess && ovf_n > 0) {
        e = hipMallocAsync(reinterpret_cast<void**>(&ovf_i), static_cast<size_t>(ovf_n) * sizeof(double), s);
        if (e == hipSuccess)
            e = hipMallocAsync(reinterpret_cast<void**>(&ovf_j), static_cast<size_t>(ovf_n) * sizeof(int), s);
    }
    int r = TM_OK;
    if (e != hipSuccess) {
        r = e == hipErrorOutOfMemory ? (tmlib::set_error("simulation scratch: out of memory"), TM_ENOMEM)
                                     : tmlib::hip_fail(e, "hipMallocAsync");
    } else {
        hipLaunchKernelGGL(grid_kernel, dim3(1), dim3(kGridThreads), 0, s, c, refl,
                           static_cast<int>(cap), n_refl);
        hipLaunchKernelGGL(template_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kSimThreads),
                           0, s, orientations, T, refl, n_refl, static_cast<int>(cap), k, s_max,
                           g_max, rel_min, max_spots, ovf_i, ovf_j, kx_out, ky_out,
                           intensity_out, count_out);
        e = hipGetLastError();
        if (e != hipSuccess) r = tmlib::hip_fail(e, "simulation kernel launch");
    }
    if (refl) (void)hipFreeAsync(refl, s);
    if (n_refl) (void)hipFreeAsync(n_refl, s);
    if (ovf_i) (void)hipFreeAsync(ovf_i, s);
    if (ovf_j) (void)hipFreeAsync(ovf_j, s);
    return r;
}
