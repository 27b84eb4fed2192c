// Internal declarations shared by the libtm translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "tm.h"

namespace tmlib {

// Thread-local error message for tm_last_error().
void set_error(const char* fmt, ...);
void clear_error();

// TM_ENODEV if no HIP device is visible, TM_OK otherwise (cached).
int require_device();

// Map a HIP error to TM_EHIP with a message naming the failing call.
int hip_fail(hipError_t e, const char* what);

#define TM_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return tmlib::hip_fail(e_, #call); \
    } while (0)

// Shared validation of a tm_polar_grid (TM_OK or TM_EINVAL with a message).
int validate_grid(const tm_polar_grid* g);

constexpr int kMaxN = TM_MAX_N;
constexpr int kWave = 64;

// Number of 64-lane shift slots per lane for a given polar width.
inline int slots_for(int n_theta) { return (n_theta + kWave - 1) / kWave; }

// Width of an LDS polar row: n_theta columns plus a wraparound halo long
// enough that lane l of slot k reading column (k0 + l + 64 k) never wraps
// (k0 < n_theta, l < 64, k < K).
inline int lds_row_width(int n_theta) { return n_theta + kWave * slots_for(n_theta) - 1; }

}  // namespace tmlib

// Device-resident library (opaque to callers).
struct tm_library {
    int32_t T = 0;          // base templates
    int32_t Tp = 0;         // total templates (2T with mirrors)
    int32_t R = 0, n_theta = 0;
    double r0 = 0, dr = 1, px_per = 1;
    uint32_t flags = 0;
    int device = 0;

    // polar rows that any template touches, grouped into LDS bands
    int32_t n_rows = 0;         // touched rows
    int32_t n_bands = 0;
    int32_t band_rows = 0;      // max rows per band
    int32_t row_width = 0;      // LDS row width in floats
    int64_t n_spots = 0;        // merged pixels over all T' templates

    // device arrays
    int32_t* d_rows = nullptr;      // [n_rows] global row of each touched row
    int32_t* d_band_off = nullptr;  // [n_bands + 1] first touched-row index of each band
    uint2* d_spots = nullptr;       // [n_spots] (LDS float offset within band, weight bits)
    int32_t* d_seg = nullptr;       // [Tp * (n_bands + 1)] spot ranges per (template, band)
    float* d_prof = nullptr;        // [T, R] radial profiles of base templates (float32)
    float* d_prof_norm = nullptr;   // [T] L2 norm of each profile (float32 of float64)
    size_t device_bytes = 0;

    // host copies used for validation and info
    std::vector<double> tnorm;      // [Tp]
};
