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

// Pre-filter (azimuthally integrated profiles, Fig. 3): per pattern the n_keep
// base templates with the highest profile correlation, ties to the lower
// index, written ascending to items [B, n_items]; with mirrors, entries
// n_keep.. hold the kept templates' mirrors (t + T). The score matrix [B, T]
// float32 lives in S when given, else in stream-ordered scratch. Enqueued on s.
int prefilter_kept(const tm_library* lib, const float* profiles, int32_t B, int32_t n_keep,
                   int32_t precision, int32_t* items, int32_t n_items, bool mirror, hipStream_t s,
                   float* S = nullptr);

// tm_match_batch with its pre-filter scratch taken from [scratch, scratch +
// scratch_bytes) when scratch is given (then nothing is allocated), else
// from the stream-ordered allocator.
int match_batch_impl(const tm_library* lib, const float* polar, const double* norms,
                     const float* profiles, int32_t B, const tm_match_opts* opts, int32_t N,
                     int32_t* top_template, int32_t* top_angle, float* top_score,
                     float* best_score, int16_t* best_angle, void* hip_stream, void* scratch,
                     size_t scratch_bytes);

// A split launch of the match kernel, planned on the device (tm_certify.hip):
// workgroups claim tasks in order from a counter; task x = pattern, [y, z) =
// its range of items (groups, or entries of its candidate row), w = the slot
// of its partial top-N list (-1: the pattern's own output rows). meta[0]
// holds the task count and meta[2] the claim counter (zeroed by the
// planner). grid: workgroups launched.
struct SplitWork {
    const int4* tasks;
    int32_t* meta;
    int32_t* part_t;
    int32_t* part_s;
    float* part_q;
    int32_t grid;
};

// Exact rescoring launch of the match kernel (tm_match.hip): all templates
// (cand == nullptr) or per-pattern candidate lists of up to n_items ids;
// cand_count (optional, [B]) limits each pattern's list; pat_mask (optional,
// [B]) skips patterns whose entry is 0; compact: polar holds only the
// library's touched rows, in order ([B, n_rows, n_theta]); split (optional)
// runs the planned tasks instead of one workgroup per pattern (cand_count,
// pat_mask and best_* unused). Enqueued on s.
int launch_match(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                 int32_t N, int32_t* top_template, int32_t* top_angle, float* top_score,
                 float* best_score, int16_t* best_angle, const int32_t* cand, int32_t n_items,
                 const int32_t* cand_count, const int32_t* pat_mask, bool compact,
                 hipStream_t s, const SplitWork* split = nullptr);

// Top-N over per-template scores [B, T] (tm_topn's kernel); best_angle may be
// null (angles reported as 0). Enqueued on s.
int launch_topn(const float* best_score, const int16_t* best_angle, int32_t B, int32_t T,
                int32_t N, int32_t* top_template, int32_t* top_angle, float* top_score,
                hipStream_t s);

// Per row of S [B, n], the n_keep largest entries (ties to the lower index),
// written ascending to items [B, n_keep]. Enqueued on s.
int select_top(const float* S, int32_t B, int32_t n, int32_t n_keep, int32_t* items,
               hipStream_t s);

// Template pixel on the polar grid (host, float64 weight).
struct HostPixel {
    int32_t j, k;
    double w;
};

// Fourier-route data of a library (tm_fft.hip): template spectra, inverse
// transform tables and the error bound; host pixels are per base template.
int fft_prepare(tm_library* L, const std::vector<std::vector<HostPixel>>& pix, hipStream_t s,
                size_t& bytes);
void fft_release(tm_library* L);
// Certified or keep-fraction rescoring after the Fourier-route coarse scorer.
int fft_match(const tm_library* lib, const float* polar, const double* norms, int32_t B,
              int32_t N, int32_t policy, double keep, int32_t* n_rescored, int32_t* top_template,
              int32_t* top_angle, float* top_score, bool compact, hipStream_t s);
// Fill a device int32 array with a value. Enqueued on s.
int fill_i32(int32_t* dst, int64_t n, int32_t value, hipStream_t s);

// Exact float32 top-N from per-template estimates Qt [B, T'] of each
// template's best exact score, every estimate either within `margin` of it
// or (margin 0) at least that score (tm_certify.hip): the n_first (N <=
// n_first <= 64) best estimates are scored exactly, then every template
// whose estimate reaches the N-th best of those exact scores minus the
// margin; a pattern with more than `cap` such templates is scored in full.
// n_rescored (optional, [B]) receives the number of templates scored
// exactly in the second pass. Enqueued on s.
// With map (optional) the estimates come in another column order: Qt is
// [B, n_cols] and column c holds template map[c] (c < T'; the columns from
// T' on hold none, map -1); without it n_cols = T'.
// With first_q / first_col (optional, device [B, n_list]) the first pass
// scores the columns first_col of the n_first largest first_q values
// instead of Qt's n_first largest (any choice keeps the result exact;
// columns -1 are none).
int certified_rescore(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                      int32_t N, int32_t n_first, const float* Qt, int32_t n_cols,
                      const int32_t* map, double margin, int32_t cap, int32_t* n_rescored,
                      int32_t* top_template, int32_t* top_angle, float* top_score, bool compact,
                      hipStream_t s, const float* first_q = nullptr,
                      const int32_t* first_col = nullptr, int32_t n_list = 0);

// Window upper bounds (tm_bound.hip): library data built at load (only when
// every template weight is non-negative and the window image fits the LDS
// budget), its release, the bounds of a batch, and the exact search built
// on them (certified rescoring with margin 0).
int bound_prepare(tm_library* L, const std::vector<std::vector<HostPixel>>& pix,
                  const std::vector<int32_t>& row_index, hipStream_t s, size_t& bytes);
void bound_release(tm_library* L);
// Bounds in chunk-slot order (Qc [B, bnd_chunks * 64], -inf for empty
// slots; d_bnd_tid maps slots to templates) or, with template_order, in
// template order (Qt [B, T']).
// lane_q, lane_c (optional, device, B x 1024): each lane's largest bound
// and its chunk-slot column (-inf / -1 for none), in rows of *n_list
// entries (the workgroup's lanes).
int bound_scores_impl(const tm_library* L, const float* polar, const double* norms, int32_t B,
                      float* out, bool template_order, bool compact, hipStream_t s,
                      float* lane_q = nullptr, int32_t* lane_c = nullptr, int* n_list = nullptr);
int bound_match(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                int32_t N, double cap_frac, int32_t* n_rescored, int32_t* top_template,
                int32_t* top_angle, float* top_score, bool compact, hipStream_t s);

constexpr int kMaxN = TM_MAX_N;
constexpr int kWave = 64;

// Number of 64-lane shift slots per lane for a given polar width.
inline int slots_for(int n_theta) { return (n_theta + kWave - 1) / kWave; }

// LDS polar row widths. Wide: n_theta columns plus a wraparound halo long
// enough that lane l of slot k reading column (k0 + l + 64 k) never wraps
// (k0 < n_theta, l < 64, k < K). Narrow: a halo of one wave, enough for any
// read of 64 consecutive columns starting below n_theta.
inline int wide_row_width(int n_theta) { return n_theta + kWave * slots_for(n_theta) - 1; }
inline int narrow_row_width(int n_theta) { return n_theta + kWave - 1; }
// Narrow rows are used up to this many slots (n_theta <= 384).
constexpr int kMaxNarrowSlots = 6;

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
    bool narrow = false;        // narrow rows with per-pixel wrap classes
    int32_t n_cls = 1;          // record classes per (group, band): K if narrow, else 1
    int64_t n_spots = 0;        // merged pixels over all T' templates
    int32_t group = 1;          // templates per group (1 or 3)
    int32_t n_groups = 0;
    int64_t n_records = 0;      // union pixels over all groups and bands

    // device arrays
    int32_t* d_rows = nullptr;      // [n_rows] global row of each touched row
    int32_t* d_row_map = nullptr;   // [R] compact index of polar row j, -1 if untouched
    int32_t* d_band_off = nullptr;  // [n_bands + 1] first touched-row index of each band
    uint32_t* d_recs = nullptr;     // [n_records * (group + 1)]: LDS float offset within the
                                    // band, then one float32 weight per group member
    int32_t* d_seg = nullptr;       // [n_groups * n_bands * n_cls + 1] first record of each
                                    // (group, band, class) segment; the next entry ends it
    int32_t* d_members = nullptr;   // [n_groups * group] template index of each member, -1 = none
    // per-template records and segments (layout of group = 1), used to rescore
    // candidate lists; null when group == 1 (then d_recs / d_seg serve)
    uint32_t* d_recs1 = nullptr;
    int32_t* d_seg1 = nullptr;
    const uint32_t* recs_single() const { return d_recs1 ? d_recs1 : d_recs; }
    const int32_t* seg_single() const { return d_seg1 ? d_seg1 : d_seg; }
    float* d_prof = nullptr;        // [T, R] radial profiles of base templates, unit L2 norm
    float* d_prof_max = nullptr;    // [T] largest entry of each normalised profile
    size_t device_bytes = 0;

    // Fourier route (TM_LIB_FFT)
    bool fft = false;
    int32_t fft_F = 0;          // frequencies 0..n_theta/2
    int32_t fft_Fp = 0;         // padded to a multiple of 16 (8 per parity)
    int32_t fft_Rp = 0;         // touched polar rows padded to a multiple of 16
    int32_t fft_Tpad = 0;       // base templates padded to a multiple of 32
    int32_t fft_Sh = 0;         // shifts of half a turn padded to a multiple of 32
    int32_t fft_sc = 0;         // power of two applied to C(k) before float16 storage
    double fft_eps = 0.0;       // certified bound |Q~ - Q32|
    uint16_t* d_fft_t = nullptr;    // [Fp][2 Tpad][Rp] float16 template spectra (x 2^8),
                                    // rows = the touched polar rows in order
    uint16_t* d_fft_w = nullptr;    // [2 parities][Sh][Fp + 8] float16 inverse tables (x 2^12)
    double* d_fft_dft = nullptr;    // [n_theta][2] cos, sin of 2 pi m / n_theta

    // window upper bounds (tm_bound.hip)
    bool bound = false;
    int32_t bnd_win = 0;        // polar columns per coarse shift window
    int32_t bnd_shifts = 0;     // coarse shifts per template
    int32_t bnd_L = 0;          // window-image row length (dwords: pairs of halves) in LDS
    int32_t bnd_chunks = 0;     // chunks of 64 templates (one per lane) scored by one wave
    int64_t bnd_units = 0;      // record units per pattern (all chunks)
    float bnd_dfac = 1.0f;      // 1 / (1 - gamma_n), rounded up, for the bound's float32 sums
    uint32_t* d_bnd_recs = nullptr;   // units of 4 steps x 64 lanes: LDS half offset | float16
                                      // weight << 16, 16 bytes per lane
    int32_t* d_bnd_end = nullptr;     // [bnd_chunks]: first unit after each chunk
    int32_t* d_bnd_slots = nullptr;   // [bnd_chunks][4]: first unit after each quarter slot
    int32_t* d_bnd_rowat = nullptr;   // [n_rows]: the compact row held at each image row place
    int32_t* d_bnd_tid = nullptr;     // [bnd_chunks * 64]: template of each chunk slot, -1 none
    std::vector<int32_t> bnd_tid;     // host copy
    float* d_bnd_cfac = nullptr;      // [bnd_chunks * 64]: margin factor, -1 for no template
    int32_t* d_bnd_part = nullptr;    // [9 + 17]: chunk ranges of 8 and of 16 waves

    // host copies used for validation and info
    std::vector<double> tnorm;      // [Tp]
    std::vector<int32_t> row_index; // [R] compact index of polar row j, -1 if untouched
};
