// Orientation of each match as Bunge Euler angles, and the angular deviation
// of Eq. (2) between two orientation maps.
//
// Section 2.1: the library samples (Phi, phi2) with phi1 = 0; the in-plane
// search finds phi1. Section 2.2: a mirrored template (spots reflected
// across y = 0) stands for a further orientation. Section 4.1, Eq. (2): the
// deviation between two maps is the angle between the crystal directions
// their inverse-pole-figure (IPF) maps show in each pixel.
//
// Sample frame: x along image columns, y along image rows, z = x cross y.
// Bunge's g maps sample to crystal coordinates, g = Z(phi2) X(Phi) Z(phi1)
// (frame rotations). A match at in-plane shift phi (counter-clockwise) of
// template (Phi, phi2) has crystal -> sample matrix Rz(phi) g0^T, which is
// Bunge (phi, Phi, phi2). A mirrored template is read as a rotation by pi
// about the sample x axis before the in-plane rotation; since
// X(Phi) X(pi) = Z(pi) X(pi - Phi) Z(pi), that orientation is Bunge
// (phi + pi, pi - Phi, phi2 + pi). Angles come out with phi1, phi2 in
// [0, 2 pi) and Phi in [0, pi]; where sin(Phi) = 0 only phi1 +- phi2 is
// defined and the angles are returned as (phi1 +- phi2, Phi, 0).
//
// Both kernels are element-wise (one thread per match or per pixel) and
// bound by latency, not by bandwidth: the work is a few dozen float64
// operations per element.
#include <cmath>

#include "tm_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

__device__ __forceinline__ double wrap_2pi(double a) {
    double r = a - kTwoPi * floor(a / kTwoPi);
    return r >= kTwoPi ? 0.0 : r;
}

__global__ void __launch_bounds__(kThreads)
orient_kernel(const double* __restrict__ lib_euler, int T, int n_total, int n_theta,
              const int* __restrict__ top_t, const int* __restrict__ top_s,
              const float* __restrict__ angle_deg, long long n, double* __restrict__ out) {
    const long long i = static_cast<long long>(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= n) return;
    const int t = top_t[i];
    double e0 = NAN, e1 = NAN, e2 = NAN;
    if (t >= 0 && t < n_total) {
        const bool mirrored = t >= T;
        const int base = mirrored ? t - T : t;
        const double Phi = lib_euler[2 * static_cast<long long>(base)];
        const double phi2 = lib_euler[2 * static_cast<long long>(base) + 1];
        const double phi = angle_deg ? static_cast<double>(angle_deg[i]) * (kPi / 180.0)
                                     : static_cast<double>(top_s[i]) * (kTwoPi / n_theta);
        if (!mirrored) {
            e0 = phi;
            e1 = Phi;
            e2 = phi2;
        } else {
            e0 = phi + kPi;
            e1 = kPi - Phi;
            e2 = phi2 + kPi;
        }
        if (fabs(sin(e1)) <= 1e-12) {
            // Phi = 0: g = Z(phi1 + phi2); Phi = pi: g depends on phi1 - phi2
            e0 = cos(e1) > 0.0 ? e0 + e2 : e0 - e2;
            e2 = 0.0;
        }
        e0 = wrap_2pi(e0);
        e2 = wrap_2pi(e2);
    }
    out[3 * i] = e0;
    out[3 * i + 1] = e1;
    out[3 * i + 2] = e2;
}

// Column d of Bunge's g: the crystal coordinates of sample axis d.
__device__ __forceinline__ void sample_axis_in_crystal(const double* e, int d, double v[3]) {
    const double c1 = cos(e[0]), s1 = sin(e[0]);
    const double c = cos(e[1]), s = sin(e[1]);
    const double c2 = cos(e[2]), s2 = sin(e[2]);
    if (d == 0) {
        v[0] = c1 * c2 - s1 * s2 * c;
        v[1] = -c1 * s2 - s1 * c2 * c;
        v[2] = s1 * s;
    } else if (d == 1) {
        v[0] = s1 * c2 + c1 * s2 * c;
        v[1] = -s1 * s2 + c1 * c2 * c;
        v[2] = -c1 * s;
    } else {
        v[0] = s2 * s;
        v[1] = c2 * s;
        v[2] = c;
    }
}

// Reduce a crystal direction to the fundamental sector of the Laue group.
__device__ __forceinline__ void to_sector(int laue, double v[3]) {
    double x = fabs(v[0]), y = fabs(v[1]), z = fabs(v[2]);
    if (laue == TM_LAUE_M3M) {
        // z >= x >= y >= 0: the largest magnitude on z, the smallest on y
        double lo = fmin(x, fmin(y, z)), hi = fmax(x, fmax(y, z));
        double mid = x + y + z - lo - hi;
        v[0] = mid;
        v[1] = lo;
        v[2] = hi;
    } else if (laue == TM_LAUE_MMM) {
        v[0] = x;
        v[1] = y;
        v[2] = z;
    } else {
        // 6/mmm: azimuth folded into [0, pi/6], z >= 0
        const double rho = hypot(v[0], v[1]);
        double az = atan2(v[1], v[0]);
        az = az - (kPi / 3.0) * floor(az / (kPi / 3.0));
        if (az > kPi / 6.0) az = kPi / 3.0 - az;
        v[0] = rho * cos(az);
        v[1] = rho * sin(az);
        v[2] = z;
    }
}

__global__ void __launch_bounds__(kThreads)
ipf_kernel(const double* __restrict__ ea, long long sa, const double* __restrict__ eb,
           long long sb, int B, int laue, double* __restrict__ out) {
    const int b = blockIdx.x * kThreads + threadIdx.x;
    if (b >= B) return;
    double a[3], p[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = ea[b * sa + k];
        p[k] = eb[b * sb + k];
    }
    for (int d = 0; d < 3; ++d) {
        double va[3], vp[3];
        sample_axis_in_crystal(a, d, va);
        sample_axis_in_crystal(p, d, vp);
        to_sector(laue, va);
        to_sector(laue, vp);
        const double dot = va[0] * vp[0] + va[1] * vp[1] + va[2] * vp[2];
        const double na = sqrt(va[0] * va[0] + va[1] * va[1] + va[2] * va[2]);
        const double np = sqrt(vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2]);
        const double c = fmin(1.0, fmax(-1.0, dot / (na * np)));
        out[3 * static_cast<long long>(b) + d] = fabs(acos(c));
    }
}

}  // namespace

extern "C" int tm_orientations(const double* lib_euler, int32_t T, int32_t mirrors,
                               int32_t n_theta, const int32_t* top_template,
                               const int32_t* top_angle, const float* angle_deg, int32_t B,
                               int32_t N, double* euler_out, void* hip_stream) {
    tmlib::clear_error();
    if (T < 1) { tmlib::set_error("T=%d < 1", T); return TM_EINVAL; }
    if (mirrors != 0 && mirrors != 1) { tmlib::set_error("mirrors=%d is not 0 or 1", mirrors); return TM_EINVAL; }
    if (n_theta < 1) { tmlib::set_error("n_theta=%d < 1", n_theta); return TM_EINVAL; }
    if (B < 0 || N < 1) { tmlib::set_error("B=%d, N=%d: need B >= 0, N >= 1", B, N); return TM_EINVAL; }
    if (!lib_euler || !top_template || !euler_out) {
        tmlib::set_error("lib_euler, top_template and euler_out must be non-NULL");
        return TM_EINVAL;
    }
    if ((top_angle == nullptr) == (angle_deg == nullptr)) {
        tmlib::set_error("exactly one of top_angle and angle_deg must be given");
        return TM_EINVAL;
    }
    if (static_cast<long long>(T) * (mirrors ? 2 : 1) > INT32_MAX) {
        tmlib::set_error("T=%d too large", T);
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    const long long n = static_cast<long long>(B) * N;
    if (n == 0) return TM_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int n_total = T * (mirrors ? 2 : 1);
    const long long blocks = (n + kThreads - 1) / kThreads;
    if (blocks > INT32_MAX) { tmlib::set_error("B*N too large"); return TM_EINVAL; }
    hipLaunchKernelGGL(orient_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s,
                       lib_euler, T, n_total, n_theta, top_template, top_angle, angle_deg, n,
                       euler_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TM_OK : tmlib::hip_fail(e, "orient_kernel launch");
}

extern "C" int tm_ipf_deviation(const double* euler_a, int32_t stride_a, const double* euler_b,
                                int32_t stride_b, int32_t B, int32_t laue, double* deviation_out,
                                void* hip_stream) {
    tmlib::clear_error();
    if (B < 0) { tmlib::set_error("B=%d < 0", B); return TM_EINVAL; }
    if (stride_a < 3 || stride_b < 3) {
        tmlib::set_error("strides %d, %d must be >= 3", stride_a, stride_b);
        return TM_EINVAL;
    }
    if (laue != TM_LAUE_M3M && laue != TM_LAUE_MMM && laue != TM_LAUE_6MMM) {
        tmlib::set_error("unknown Laue group %d", laue);
        return TM_EINVAL;
    }
    if (!euler_a || !euler_b || !deviation_out) {
        tmlib::set_error("euler_a, euler_b and deviation_out must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;
    if (B == 0) return TM_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(ipf_kernel, dim3((B + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       euler_a, static_cast<long long>(stride_a), euler_b,
                       static_cast<long long>(stride_b), B, laue, deviation_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TM_OK : tmlib::hip_fail(e, "ipf_kernel launch");
}
