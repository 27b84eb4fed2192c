/*
 * tm.h - C ABI of libtm, template-matching orientation mapping on MI355X (gfx950).
 *
 * The library indexes 4D-STEM diffraction patterns against a library of
 * simulated templates, following Cautaerts et al., "Free, flexible and fast:
 * orientation mapping using the multi-core and GPU-accelerated template
 * matching capabilities in the Python-based open source 4D-STEM analysis
 * toolbox Pyxem" (Ultramicroscopy; arXiv 2111.07347):
 *
 *   - a template is a list of Bragg spots (kx, ky) with intensities, one per
 *     out-of-plane orientation (Section 2.1);
 *   - each pattern is resampled to polar coordinates about the direct beam
 *     (Section 2.2, Fig. 2 c);
 *   - every template, and its mirror across y = 0, is slid along the
 *     azimuthal axis with wraparound and scored at every shift by the
 *     correlation index Q of Eq. (1), with template spots rounded to integer
 *     polar pixels (Section 2.2, Fig. 2 d-e);
 *   - the best Q per template and its angle are kept and the N best
 *     templates are returned per pattern (Section 2.2, end);
 *   - optionally the library is first pre-filtered by correlating
 *     azimuthally integrated profiles (Section 2.2, Fig. 3).
 *
 * Conventions shared by every call
 *   - Template indices: base templates are 0..T-1; with mirrors enabled the
 *     mirror of base template t has index T + t, so T' = 2T.
 *   - Angles are bins s in [0, n_theta); the in-plane rotation in degrees is
 *     s * 360 / n_theta (Section 2.2: 360 polar columns give 1 degree).
 *     Shift s means the template read at polar column (k + s) mod n_theta,
 *     i.e. the template rotated counter-clockwise (from +x toward +y, x being
 *     the image column and y the image row) by s bins.
 *   - Scores are Q of Eq. (1) as float32.
 *   - Device buffers are owned by the caller (e.g. torch tensors); the
 *     library only reads or writes them during the work it enqueues.
 *   - Every call that touches the device enqueues its work asynchronously on
 *     the given HIP stream (NULL = the default stream) and returns; results
 *     are valid once that stream has synchronised. Arguments are validated
 *     before anything is enqueued.
 *   - Every call returns a tm_status. Nothing aborts or throws across the
 *     ABI. On failure tm_last_error() describes the cause (per thread).
 *   - With no HIP device present, every call that needs one returns
 *     TM_ENODEV.
 */
#ifndef TM_H
#define TM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TM_OK = 0,
    TM_EINVAL = -1,          /* an argument is invalid (null, out of range, mismatched) */
    TM_ENOMEM = -2,          /* device or host allocation failed */
    TM_EHIP = -3,            /* a HIP runtime call failed; message in tm_last_error() */
    TM_ENODEV = -4,          /* no HIP device is available */
    TM_EUNSUPPORTED = -5,    /* valid request the library does not implement */
    TM_ENOMEM_BUDGET = -6    /* request larger than a caller-given memory budget */
} tm_status;

typedef enum { TM_U16 = 0, TM_F32 = 1 } tm_dtype;

typedef enum {
    TM_PREC_FP32 = 0,        /* plain float32 */
    TM_PREC_BF16 = 1,
    TM_PREC_FP16 = 2,
    TM_PREC_FP8 = 3          /* e4m3 with per-template scale */
} tm_precision;

/* Polar sampling grid (Section 2.2, Fig. 2 c).
 *   radii   r_j = r0 + j*dr, j in [0, R)                   (pixels)
 *   angles  theta_k = 2*pi*k/n_theta, k in [0, n_theta)
 *   sample  (x, y) = (cx + r_j cos theta_k, cy + r_j sin theta_k), where x is
 *           the image column and y the image row (pixel (row i, column j)
 *           sits at x = j, y = i), (cx, cy) is the direct-beam centre.
 * interp: 1 = bilinear with zero padding outside the image (default),
 *         0 = nearest pixel (round half to even), zero outside.
 * Limits: 1 <= R <= 4096, 64 <= n_theta <= 768, dr > 0. */
typedef struct {
    int32_t R;
    int32_t n_theta;
    double r0;
    double dr;
    double cx;
    double cy;
    int32_t interp;
} tm_polar_grid;

/* Library flags. */
enum {
    TM_LIB_MIRROR = 1u,            /* add mirrored templates (Section 2.2, Fig. 2 f) */
    TM_LIB_UNIT_INTENSITY = 2u,    /* all spot weights 1 (Section 4.3) */
    TM_LIB_KEEP_DIRECT_BEAM = 4u,  /* keep spots at (0, 0); dropped by default */
    TM_LIB_NO_GROUPING = 8u,       /* score every template on its own; by default
                                      templates sharing polar pixels are scored
                                      together (same results up to float32
                                      summation order) */
    TM_LIB_FFT = 16u               /* also keep the templates' spectra along theta
                                      for the Fourier-route coarse scorer
                                      (tm_fft_scores; needs an even n_theta) */
};

/* Coarse scorer and rescoring policy of tm_match_batch. */
enum {
    TM_COARSE_NONE = 0,            /* no coarse scorer */
    TM_COARSE_FFT = 1,             /* Fourier route along theta (tm_fft_scores) */
    TM_COARSE_BOUND = 2            /* window upper bounds (tm_bound_scores): an
                                      exact search with the plain path's result */
};
enum {
    TM_RESCORE_CERTIFIED = 0,      /* rescore every template the coarse scorer's
                                      error bound cannot rule out: the result
                                      is the exact float32 top-N */
    TM_RESCORE_KEEP = 1            /* rescore a fixed fraction of the templates
                                      with the best coarse scores */
};

/* Options of tm_match_batch. A NULL options pointer (or all fields zero)
 * means the plain float32 path: every template scored exactly.
 *   prefilter_keep    fraction f of base templates kept by the azimuthal
 *                     pre-filter (Section 2.2, Fig. 3), 0 = no pre-filter;
 *                     the kept ceil(f*T) base templates (and their mirrors)
 *                     are then scored exactly in float32 (tm_prefilter
 *                     followed by tm_match_candidates).
 *   prefilter_prec    arithmetic of the pre-filter's profile correlation
 *                     (FP32, BF16, FP16 or FP8 on the matrix cores with
 *                     float32 accumulation).
 *   coarse            TM_COARSE_NONE, or TM_COARSE_FFT: score every template
 *                     approximately through the Fourier route (Section 2.2;
 *                     tm_fft_scores; the library needs TM_LIB_FFT), then
 *                     rescore candidates exactly in float32; or
 *                     TM_COARSE_BOUND: bound every template's best score
 *                     from above over windows of shifts (tm_bound_scores)
 *                     and score exactly every template whose bound reaches
 *                     the N-th best exact score: the same top-N as the plain
 *                     path, usually after scoring a small fraction of the
 *                     library exactly. Exclusive with the pre-filter.
 *   rescore_policy    with a coarse scorer: TM_RESCORE_CERTIFIED (default)
 *                     or TM_RESCORE_KEEP.
 *   rescore_keep      TM_RESCORE_KEEP: fraction of the T' templates rescored
 *                     (those with the best coarse scores, ties to the lower
 *                     index). TM_RESCORE_CERTIFIED: largest fraction of T'
 *                     rescored from the candidate list (0 = 0.1); a pattern
 *                     whose certified set is larger is scored in full.
 *   n_rescored        optional device [B] int32 output: templates scored
 *                     exactly per pattern (T' for a full scan), or NULL.
 *   compact_rows      0: polar is [B, R, n_theta]; 1: polar holds only the
 *                     library's touched rows in increasing order,
 *                     [B, n_rows, n_theta] (tm_polar_transform_rows with the
 *                     map of tm_library_rows). */
typedef struct {
    double prefilter_keep;
    int32_t prefilter_prec;
    int32_t coarse;
    int32_t rescore_policy;
    int32_t compact_rows;
    double rescore_keep;
    int32_t* n_rescored;
} tm_match_opts;

typedef struct tm_library tm_library;   /* opaque; immutable after load */

/* Largest N accepted by tm_match_batch and tm_topn. */
#define TM_MAX_N 64

/* tm_load_library - build a device-resident template library.
 *
 * Section 2.1: each template is a list of Bragg spots (kx, ky)_i in
 * reciprocal-space units (1/Angstrom) with intensities I_i; the library is a
 * list of templates. Section 2.2: spot polar coordinates are rounded to the
 * nearest integer pixel of the polar grid; mirrors reflect spots across
 * y = 0; template norms are precomputed so Eq. (1) becomes a dot product.
 *
 * Per spot, in float64 on the host (one-time set-up):
 *   rho = px_per_inv_angstrom * hypot(kx, ky)
 *   j   = rint((rho - grid->r0) / grid->dr)                (half to even)
 *   k   = rint(atan2(ky, kx) * n_theta / (2 pi)) mod n_theta
 *   spots with j outside [0, R) are dropped; spots at (0, 0) are dropped
 *   unless TM_LIB_KEEP_DIRECT_BEAM; spots of one template falling on the
 *   same (j, k) are merged by summing their weights (weight = intensity, or
 *   1 with TM_LIB_UNIT_INTENSITY); ||T|| = sqrt(sum of merged weights^2);
 *   device weights are w / ||T|| rounded to float32. A mirror uses
 *   (j, (-k) mod n_theta).
 *
 * Arguments
 *   kx, ky, intensity  host float64 arrays of length offsets[n_templates],
 *                      read during the call only.
 *   offsets            host int64 array [n_templates + 1], CSR offsets
 *                      (offsets[0] = 0, non-decreasing).
 *   n_templates        T >= 1 base templates.
 *   px_per_inv_angstrom  detector calibration (pixels per 1/Angstrom), > 0.
 *   grid               polar grid the patterns will be resampled on (R,
 *                      n_theta, r0, dr are used; cx, cy, interp are not).
 *   flags              TM_LIB_* bits.
 *   hip_stream         stream used for the uploads; the call synchronises it
 *                      before returning.
 *   out                receives the handle; free with tm_free_library.
 * Errors: TM_EINVAL (null pointer, T < 1, bad offsets, bad grid),
 *         TM_ENOMEM, TM_EHIP, TM_ENODEV. On error *out is set to NULL. */
int tm_load_library(const double* kx, const double* ky, const double* intensity,
                    const int64_t* offsets, int32_t n_templates,
                    double px_per_inv_angstrom, const tm_polar_grid* grid, uint32_t flags,
                    void* hip_stream, tm_library** out);

/* tm_free_library - release a library's device memory. The caller must make
 * sure no enqueued work still uses it (synchronise the streams first).
 * NULL is accepted and ignored. */
int tm_free_library(tm_library* lib);

/* tm_library_info - sizes of a loaded library (any pointer may be NULL).
 *   n_templates_total  T' (2T with mirrors)
 *   n_spots            merged polar pixels over all T' templates
 *   device_bytes       device memory held by the handle */
int tm_library_info(const tm_library* lib, int32_t* n_templates_total, int64_t* n_spots,
                    size_t* device_bytes);

/* tm_library_layout - how a loaded library is laid out for the match kernel
 * (any pointer may be NULL).
 *   group      templates scored together per group (1 = no grouping)
 *   n_bands    LDS bands the touched polar rows are split into (1 = all at once)
 *   n_rows     polar rows touched by any template
 *   n_records  union pixels stored over all groups and bands
 *   row_width  floats per LDS row: n_theta + 64*ceil(n_theta/64) - 1 (wide rows,
 *              no wrap handling) or n_theta + 63 (narrow rows, wrap handled
 *              per pixel) */
int tm_library_layout(const tm_library* lib, int32_t* group, int32_t* n_bands, int32_t* n_rows,
                      int64_t* n_records, int32_t* row_width);

/* tm_library_rows - the polar rows any template of lib touches: their number
 * and a library-owned device map [R] (int32: compact index of polar row j in
 * increasing row order, -1 if no template touches row j), valid until
 * tm_free_library. Errors: TM_EINVAL (null library). */
int tm_library_rows(const tm_library* lib, int32_t* n_rows, const int32_t** row_map);

/* tm_polar_transform - intensity transform, polar resampling, norms and
 * azimuthal profiles of a batch of patterns (Section 2.2: gamma correction
 * and constant subtraction of the pattern; polar transform about the
 * direct-beam centre; Eq. (1) image norm; Fig. 3 azimuthal integration).
 *
 *   x~ = (gamma != 1 ? max(x, 0)^gamma : x) - subtract   per Cartesian pixel
 *   P[b, j, k] = interp(x~_b; sample point of (j, k))    zero outside image
 *   norm_out[b] = sqrt(sum_{j,k} P[b,j,k]^2)              float64 sum
 *   profile_out[j*B + b] = sum_k P[b, j, k]               float64 sum, stored float32
 *
 * Arguments
 *   patterns     device, [B, H, W] row-major, uint16 or float32 (dtype).
 *   B, H, W      B >= 0 (0 is a no-op), 1 <= H, W <= 32767.
 *   grid         sampling grid (all fields used).
 *   gamma        > 0; 1 disables the power (and the clamp at zero).
 *   subtract     constant removed after the power.
 *   polar_out    device, [B, R, n_theta] float32, written.
 *   norm_out     device, [B] float64, written.
 *   profile_out  device, [R, B] float32 (note: radius-major), or NULL.
 * Polar look-up tables (float64-built base pixel and float32 fractions) are
 * built on first use for each (H, W, grid) and cached for the process.
 * Errors: TM_EINVAL (null required pointer, bad sizes or grid, gamma <= 0),
 *         TM_EHIP, TM_ENODEV, TM_ENOMEM. */
int tm_polar_transform(const void* patterns, tm_dtype dtype, int32_t B, int32_t H, int32_t W,
                       const tm_polar_grid* grid, float gamma, float subtract,
                       float* polar_out, double* norm_out, float* profile_out,
                       void* hip_stream);

/* tm_polar_transform_rows - tm_polar_transform with an optional pattern mask,
 * writing only selected polar rows.
 *
 * Mask (Section 4.3, custom indexation procedures: the dominant phase's
 * reflections are masked before the second phase is indexed): the
 * transformed pattern is multiplied pixel by pixel by mask[y*W + x] before
 * resampling, P~ = mask * (max(x, 0)^gamma - c), so a masked pixel is 0 and
 * contributes neither to Q nor to ||P|| (see tm_mask_from_mean).
 *
 * Rows: every row is still sampled (||P|| and the profiles cover the whole
 * polar image, Eq. 1); polar row j goes to output row row_map[j], or is not
 * stored when row_map[j] < 0 (entries outside [0, n_out_rows) are not
 * stored either). With a library's map (tm_library_rows) the output holds
 * exactly the rows its templates touch, which is all the search reads
 * (Section 2.2: the template is non-zero only at its spots).
 *
 * Arguments as in tm_polar_transform, plus
 *   mask         device, [H, W] float32, 16-byte aligned, or NULL (no mask).
 *   row_map      device, [R] int32, or NULL (then n_out_rows must be R).
 *   n_out_rows   1 <= n_out_rows <= R.
 *   polar_out    device, [B, n_out_rows, n_theta] float32, written.
 * Errors as tm_polar_transform. */
int tm_polar_transform_rows(const void* patterns, tm_dtype dtype, int32_t B, int32_t H,
                            int32_t W, const tm_polar_grid* grid, float gamma, float subtract,
                            const float* mask, const int32_t* row_map, int32_t n_out_rows,
                            float* polar_out, double* norm_out, float* profile_out,
                            void* hip_stream);

/* tm_mask_from_mean - the mask of the dominant phase for two-stage indexing
 * (Section 4.3, custom indexation procedures): average all patterns, threshold
 * the average, then erode and dilate to remove small noise-like features and
 * the tails of intense peaks.
 *
 *   bright[y, x] = (1/B) sum_b pattern_b[y, x] > threshold   (float64)
 *   bright       = dilate^n_open(erode^n_open(bright))          (opening)
 *   bright       = dilate^n_grow(bright)
 *   mask_out     = 0 where bright, 1 elsewhere
 * Erosion / dilation: 3x3 square neighbourhood, pixels outside the image
 * count as not bright.
 *
 * Arguments
 *   patterns   device, [B, H, W] uint16 or float32 (dtype), B >= 1.
 *   threshold  finite; n_open, n_grow in [0, 64].
 *   mask_out   device, [H, W] float32, written.
 * Scratch (chunk sums, two byte images) from the stream-ordered allocator.
 * Errors: TM_EINVAL, TM_ENOMEM, TM_EHIP, TM_ENODEV. */
int tm_mask_from_mean(const void* patterns, tm_dtype dtype, int32_t B, int32_t H, int32_t W,
                      double threshold, int32_t n_open, int32_t n_grow, float* mask_out,
                      void* hip_stream);

/* tm_match_batch - score every template of lib against every pattern at every
 * in-plane shift and keep the N best templates per pattern (Eq. 1; Section
 * 2.2: sliding with wraparound, best Q and angle per template, top-N).
 *
 *   Q(b, t, s) = sum_{(j,k,w) in t} w * P[b, j, (k+s) mod n_theta]
 *                / (norms[b] * ||T_t||)           (0 if either norm is 0)
 *   best(b, t) = max_s Q, angle = smallest maximising s
 *   top rows: N distinct templates by best descending, ties to the lower
 *   template index, each with its best angle. Accumulation is float32 in a
 *   fixed order per (pattern, template), independent of the batch.
 *   A pattern whose norm is not finite (its polar image holds a NaN or an
 *   infinity) is not ranked: its N rows are template -1, angle -1, score NaN
 *   (per-template outputs: NaN and -1). This holds on every path below.
 *
 * Arguments
 *   lib          loaded library; its grid defines R and n_theta.
 *   polar        device, [B, R, n_theta] float32 (tm_polar_transform output).
 *   norms        device, [B] float64 image norms.
 *   profiles     device, [R, B] float32 azimuthal profiles; required only
 *                when opts->prefilter_keep > 0, else may be NULL.
 *                With opts->coarse = TM_COARSE_FFT (certified policy), the
 *                result equals the plain path's top-N: every template whose
 *                approximate score, widened by tm_fft_error_bound(), could
 *                reach the N-th best exact score is rescored exactly.
 *   B            >= 0 (0 is a no-op).
 *   opts         NULL for the plain path, or options (see tm_match_opts).
 *   N            1 <= N <= min(TM_MAX_N, T'); with a pre-filter, N must not
 *                exceed the number of kept templates.
 *   top_template, top_angle  device, [B, N] int32, written, best first.
 *   top_score    device, [B, N] float32, written.
 *   best_score   device, [B, T'] float32 per-template best Q, or NULL.
 *   best_angle   device, [B, T'] int16 per-template best angle, or NULL;
 *                best_score and best_angle must be both NULL or both set,
 *                and are only available without pre-filter or coarse
 *                scorer.
 * Errors: TM_EINVAL, TM_EUNSUPPORTED (unknown options), TM_EHIP, TM_ENODEV. */
int tm_match_batch(const tm_library* lib, const float* polar, const double* norms,
                   const float* profiles, int32_t B, const tm_match_opts* opts, int32_t N,
                   int32_t* top_template, int32_t* top_angle, float* top_score,
                   float* best_score, int16_t* best_angle, void* hip_stream);

/* Size of the static scratch array of tm_match_batch_static (per GPU). */
#define TM_STATIC_SCRATCH_BYTES (64u << 20)

/* tm_match_batch_static - tm_match_batch for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation during a run. It takes the same arguments and gives
 * the same results; it calls no hipMalloc, hipFree or allocating routine.
 *
 * The pre-filter's scratch (kept lists [B, n_items] int32, then the score
 * matrix [B, T] float32 at the next 256-byte boundary) lives in a static
 * device array of TM_STATIC_SCRATCH_BYTES (64 MiB) that each GPU the library
 * runs on holds until the process ends. Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race and must be serialised by the caller. Everything the kernels read
 * from it is written first in the same call, so no clearing is needed.
 * The plain path uses no scratch.
 *
 * Errors: as tm_match_batch, plus TM_EINVAL when the pre-filter's scratch
 * exceeds the array (e.g. with T = 20000 base templates and keep 0.1,
 * B <= 699 patterns per call) and TM_EUNSUPPORTED for the Fourier route
 * (TM_COARSE_FFT), whose scratch is far larger. */
int tm_match_batch_static(const tm_library* lib, const float* polar, const double* norms,
                          const float* profiles, int32_t B, const tm_match_opts* opts, int32_t N,
                          int32_t* top_template, int32_t* top_angle, float* top_score,
                          float* best_score, int16_t* best_angle, void* hip_stream);

/* tm_prefilter - the library pre-filter of Section 2.2 (Fig. 3): pattern and
 * template are integrated over the azimuth and correlated by one matrix
 * product; the best-correlating templates are kept for the full search.
 *
 *   score[b, t] = sum_j prof_T[t, j] * profiles[j*B + b]
 *
 * prof_T is template t's radial profile (per polar row, the sum of its merged
 * pixel weights) scaled to unit length, so ranking a pattern's scores ranks
 * the cosine between the two profiles. The product runs in `precision`
 * (TM_PREC_FP32, BF16, FP16 or FP8 e4m3 with every template profile and every
 * pattern profile scaled to maximum 1) with float32 accumulation. Per pattern
 * the n_keep base templates with the largest scores are kept, ties to the
 * lower template index, and written in ascending index order.
 *
 * Arguments
 *   lib        loaded library (its base templates 0..T-1 are ranked; mirrors
 *              share their base template's profile).
 *   profiles   device, [R, B] float32 (tm_polar_transform's profile_out).
 *   B          >= 0 (0 is a no-op).
 *   n_keep     1 <= n_keep <= T.
 *   precision  a tm_precision.
 *   kept       device, [B, n_keep] int32, written.
 * Scratch of B*T*4 bytes is taken from the stream-ordered allocator.
 * Errors: TM_EINVAL, TM_ENOMEM, TM_EHIP, TM_ENODEV. */
int tm_prefilter(const tm_library* lib, const float* profiles, int32_t B, int32_t n_keep,
                 int32_t precision, int32_t* kept, void* hip_stream);

/* tm_match_candidates - the exact search of tm_match_batch restricted to a
 * per-pattern candidate list (rescoring after a pre-filter or another coarse
 * scorer): Q of Eq. (1) at every shift for each listed template, best shift
 * per template, N best by Q descending, ties to the lower template index.
 *
 * Arguments
 *   candidates device, [B, n_cand] int32 template indices in [0, T') (mirrors
 *              are T..T'-1); entries outside that range are ignored; a row
 *              must not list a template twice.
 *   n_cand     >= 1; 1 <= N <= min(TM_MAX_N, n_cand).
 *   other arguments as in tm_match_batch (a pattern with a non-finite norm
 *   gets template -1, angle -1, score NaN).
 * Errors: TM_EINVAL, TM_EHIP, TM_ENODEV. */
int tm_match_candidates(const tm_library* lib, const float* polar, const double* norms,
                        int32_t B, const int32_t* candidates, int32_t n_cand, int32_t N,
                        int32_t* top_template, int32_t* top_angle, float* top_score,
                        void* hip_stream);

/* tm_refine_angles - sub-bin in-plane angles of reported matches (Section 5,
 * discussion: improving the optimisation of the in-plane angle phi1).
 *
 * For row i of pattern b with template t = top_template[b, i] and shift
 * s = top_angle[b, i]: q-, q0, q+ = Q(b, t, s-1), Q(b, t, s), Q(b, t, s+1)
 * (Eq. 1, shifts mod n_theta, float32 as in tm_match_batch); when the
 * parabola through them is a maximum (q- - 2 q0 + q+ < 0) its vertex offset
 * d = (q- - q+) / (2 (q- - 2 q0 + q+)) clipped to [-1/2, 1/2], else d = 0;
 *   refined_deg[b, i] = ((s + d) * 360 / n_theta) mod 360.
 * Templates outside [0, T') give s * 360 / n_theta.
 *
 * Arguments
 *   lib, polar, norms, B    as in tm_match_batch (B >= 0; 0 is a no-op).
 *   compact_rows            layout of polar (tm_match_opts.compact_rows).
 *   N                       >= 1, columns of the top arrays.
 *   top_template, top_angle device, [B, N] int32 (tm_match_batch output).
 *   refined_deg             device, [B, N] float32, written.
 * Errors: TM_EINVAL, TM_EHIP, TM_ENODEV. */
int tm_refine_angles(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                     int32_t compact_rows, int32_t N, const int32_t* top_template,
                     const int32_t* top_angle, float* refined_deg, void* hip_stream);

/* Laue groups for the inverse-pole-figure reduction of tm_ipf_deviation
 * (Cartesian crystal frame; hexagonal with a along x). */
enum {
    TM_LAUE_M3M = 0,    /* cubic m-3m: sector z >= x >= y >= 0 */
    TM_LAUE_MMM = 1,    /* orthorhombic mmm: x, y, z >= 0 */
    TM_LAUE_6MMM = 2    /* hexagonal 6/mmm: z >= 0, azimuth in [0, 30 degrees] */
};

/* tm_orientations - Bunge Euler angles (phi1, Phi, phi2) of reported matches
 * (Section 2.1: the library samples (Phi, phi2) with phi1 = 0 and phi1 is
 * found by the in-plane search; Section 2.2: mirrored templates stand for
 * further orientations).
 *
 * Frames: sample x along image columns, y along image rows, z = x cross y;
 * g = Z(phi2) X(Phi) Z(phi1) (frame rotations) maps sample to crystal
 * coordinates. A match of base template t at in-plane angle phi (the
 * counter-clockwise rotation of the matching convention) is
 * (phi, Phi_t, phi2_t). A mirrored match is read as the template's
 * orientation rotated by pi about the sample x axis, then by phi about z,
 * i.e. (phi + pi, pi - Phi_t, phi2_t + pi). Output ranges: phi1, phi2 in
 * [0, 2 pi), Phi in [0, pi]; where sin(Phi) = 0 the pair is returned as
 * (phi1 +- phi2, Phi, 0). Entries whose template is outside [0, T') are NaN.
 *
 * Arguments
 *   lib_euler      device, [T, 2] float64: (Phi, phi2) of each base template,
 *                  radians.
 *   T              >= 1, base templates.
 *   mirrors        1 if template ids T..2T-1 are mirrors (TM_LIB_MIRROR), else 0.
 *   n_theta        polar columns (angle bin s is s * 2 pi / n_theta).
 *   top_template   device, [B, N] int32 (tm_match_batch output).
 *   top_angle      device, [B, N] int32 angle bins, or NULL;
 *   angle_deg      device, [B, N] float32 degrees (tm_refine_angles), or NULL;
 *                  exactly one of the two is given.
 *   B, N           B >= 0 (0 is a no-op), N >= 1.
 *   euler_out      device, [B, N, 3] float64 radians, written.
 * Errors: TM_EINVAL, TM_EHIP, TM_ENODEV. */
int tm_orientations(const double* lib_euler, int32_t T, int32_t mirrors, int32_t n_theta,
                    const int32_t* top_template, const int32_t* top_angle,
                    const float* angle_deg, int32_t B, int32_t N, double* euler_out,
                    void* hip_stream);

/* tm_ipf_deviation - angular deviation between two orientation maps, Eq. (2)
 * (Section 4.1): for each sample direction d in (x, y, z), v = g d is the
 * crystal direction an IPF-d map shows, reduced to the fundamental sector of
 * the Laue group; theta = |arccos(v_A . v_P / (|v_A| |v_P|))|.
 *
 * Arguments
 *   euler_a, euler_b  device float64 Bunge triples (radians); pattern b's
 *                     triple starts at element b * stride (stride >= 3, e.g.
 *                     3 * N to take the best match of a [B, N, 3] array).
 *   B                 >= 0 (0 is a no-op).
 *   laue              TM_LAUE_*.
 *   deviation_out     device, [B, 3] float64 radians (IPF-x, IPF-y, IPF-z),
 *                     written.
 * Errors: TM_EINVAL, TM_EHIP, TM_ENODEV. */
int tm_ipf_deviation(const double* euler_a, int32_t stride_a, const double* euler_b,
                     int32_t stride_b, int32_t B, int32_t laue, double* deviation_out,
                     void* hip_stream);

/* tm_simulate_library - kinematical template library on the device
 * (Section 2.1): the reciprocal lattice points up to a maximum radius are rotated
 * by each orientation (phi1 = 0, Phi, phi2); each point's excitation error
 * (distance to the Ewald sphere) sets a shape factor; spot intensity is
 * F F* times the shape factor; the excited spots are projected onto kx-ky.
 *
 *   grid       all hkl != 000 with |g| <= g_lim, g = h b1 + k b2 + l b3,
 *              lexicographic in (h, k, l); F = sum_a f_a exp(2 pi i h.x_a),
 *              reflections with F F* <= 1e-6 dropped;
 *   rotation   g_sample = g0^T g_crystal, g0 the Bunge matrix of
 *              (0, Phi, phi2) (tm_orientations' frames);
 *   Ewald      beam along -z: s = k - |g_sample - (0, 0, k)|;
 *   shape      max(0, 1 - |s| / s_max) (linear relrod);
 *   kept       shape > 0 and sqrt(gx^2 + gy^2) <= g_max, then intensity
 *              >= rel_min * the template's brightest; ordered by intensity
 *              (descending, ties in grid order), at most max_spots;
 *              intensities divided by the brightest.
 *
 * Arguments
 *   recip_basis   host, [3][3] float64, rows b1, b2, b3 in 1/Angstrom
 *                 (Cartesian crystal frame, no factor 2 pi).
 *   atoms_frac    host, [n_atoms][3] float64 fractional positions.
 *   f_atoms       host, [n_atoms] float64 scattering factor per atom (1 for
 *                 unit scattering factors).
 *   n_atoms       1..32.
 *   g_lim         > 0, grid radius (1/Angstrom); the (h, k, l) box it spans
 *                 may hold at most 2^20 points.
 *   orientations  device, [T, 2] float64 (Phi, phi2) radians.
 *   T             >= 0 (0 is a no-op).
 *   k             > 0, 1 / wavelength (1/Angstrom).
 *   s_max, g_max  > 0 (1/Angstrom). rel_min >= 0. max_spots 1..4096.
 *   kx_out, ky_out, intensity_out  device, [T, max_spots] float64, written
 *                 up to count_out[t] entries per row (the rest untouched).
 *   count_out     device, [T] int32, written.
 * Scratch (the reflection list, and spill space for orientations that excite
 * more than 256 reflections: about 12 bytes x reflections x 8 x 4 x CUs)
 * comes from the stream-ordered allocator.
 * Errors: TM_EINVAL, TM_EUNSUPPORTED (box too large), TM_ENOMEM, TM_EHIP,
 *         TM_ENODEV. */
int tm_simulate_library(const double* recip_basis, const double* atoms_frac,
                        const double* f_atoms, int32_t n_atoms, double g_lim,
                        const double* orientations, int32_t T, double k, double s_max,
                        double g_max, double rel_min, int32_t max_spots, double* kx_out,
                        double* ky_out, double* intensity_out, int32_t* count_out,
                        void* hip_stream);

/* Options of tm_preprocess (Section 4.1: direct beam centred, diffuse
 * background removed by a difference of Gaussians, Gaussian blur, low
 * intensities set to zero). */
typedef struct {
    int32_t r_box;       /* centre search half-width in px around (W/2, H/2); < 0: no centring */
    double frac;         /* box pixels >= frac * box maximum enter the centroid */
    double sigma_min;    /* difference of Gaussians G(sigma_min) - G(sigma_max), px; */
    double sigma_max;    /*   sigma_max = 0 skips it; else 0 <= sigma_min < sigma_max */
    double sigma_blur;   /* Gaussian blur of the result, px; 0 skips it */
    double threshold;    /* values below it become 0; -inf skips it */
} tm_preprocess_opts;

/* tm_preprocess - the preprocessing the paper applies before indexing, in
 * its order, on the device (Section 4.1; the discussion lists moving these
 * steps off the CPU as an open optimisation).
 *
 *   centre    (cx, cy) = intensity-weighted centroid (float64) of the pixels
 *             of the box |x - W/2| <= r_box, |y - H/2| <= r_box whose value
 *             is >= frac * the box maximum (the direct beam); a box whose
 *             maximum is <= 0 gives (W/2, H/2). The pattern is resampled
 *             as c(x, y) = p(x + cx - W/2, y + cy - H/2), bilinear, zero
 *             outside, which puts the beam on (W/2, H/2);
 *   DoG       d = G(sigma_min) c - G(sigma_max) c;
 *   blur      e = G(sigma_blur) d;  threshold: e < threshold -> 0.
 * G(sigma): separable correlation with exp(-t^2 / 2 sigma^2) on
 * |t| <= floor(4 sigma + 0.5) (at most 64), normalised to sum 1, mirror
 * boundary (... c b a | a b c ...); G(0) is the identity. Arithmetic in
 * float32 (centroid in float64). The output feeds tm_polar_transform as a
 * TM_F32 pattern stack (its gamma step follows, as in the paper).
 *
 * Arguments
 *   patterns     device, [B, H, W] uint16 or float32 (dtype).
 *   B, H, W      B >= 0 (0 is a no-op), 1 <= H, W <= 8192.
 *   opts         host, read during the call.
 *   out          device, [B, H, W] float32, written (may not alias patterns).
 *   centre_out   device, [B, 2] float64 (cx, cy), written, or NULL.
 * Scratch (two float32 images per pattern of a chunk, at most 1 GiB) comes
 * from the stream-ordered allocator.
 * Errors: TM_EINVAL, TM_ENOMEM, TM_EHIP, TM_ENODEV. */
int tm_preprocess(const void* patterns, tm_dtype dtype, int32_t B, int32_t H, int32_t W,
                  const tm_preprocess_opts* opts, float* out, double* centre_out,
                  void* hip_stream);

/* tm_fft_scores - approximate best score and angle of every template for every
 * pattern through the Fourier route (Section 2.2: the azimuthal sliding is a
 * circular cross-correlation along theta, evaluated with Fourier transforms).
 *
 *   spectra  P^[b, j, k] = sum_theta P[b, j, theta] e^{-2 pi i k theta / n}
 *            / norms[b], and T^[t, j, k] of template t's merged weights / ||T||,
 *            frequencies k = 0 .. n/2 (n = n_theta);
 *   C(k)     = sum_j conj(T^[t, j, k]) P^[b, j, k] (mirror: T^ instead of
 *            conj(T^));
 *   Q~(s)    = (1/n) sum_k c_k Re(C(k) e^{2 pi i k s / n}), c_k = 1 at k = 0
 *            and k = n/2, else 2; approx_score = max_s Q~, approx_angle =
 *            the smallest maximising s of the computed values.
 * Exact arithmetic would give Q of Eq. (1). Here the spectra are float16,
 * the contraction over rows and the inverse transform run on the matrix
 * cores with float32 accumulation, and C(k) is stored as float16 between
 * them; |approx_score - best Q| never exceeds tm_fft_error_bound().
 *
 * Arguments
 *   lib           library loaded with TM_LIB_FFT.
 *   polar, norms  as in tm_match_batch.
 *   B             >= 0 (0 is a no-op).
 *   compact_rows  0: polar is [B, R, n_theta]; 1: [B, n_rows, n_theta] holding
 *                 the library's touched rows (as tm_match_opts.compact_rows).
 *   approx_score  device, [B, T'] float32, written.
 *   approx_angle  device, [B, T'] int16, written, or NULL.
 * Scratch (spectra of a chunk of patterns; about 2 GiB) is taken from
 * the stream-ordered allocator.
 * Errors: TM_EINVAL (null pointer, library without TM_LIB_FFT), TM_ENOMEM,
 *         TM_EHIP, TM_ENODEV. */
int tm_fft_scores(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                  int32_t compact_rows, float* approx_score, int16_t* approx_angle,
                  void* hip_stream);

/* tm_bound_scores - an upper bound of every template's best Q for every
 * pattern (an exact-search aid, not part of the paper's procedure: it
 * lets the certified rescoring skip templates that cannot reach the top-N).
 *
 * With non-negative template weights, for the window of win = ceil(n_theta
 * / 4) consecutive shifts starting at S win (S = 0..3, columns mod n_theta):
 *   C(s) = sum_i w_i P[j_i, k_i + s] <= sum_i w_i M[j_i, k_i + S win - e_iS],
 *   M[j, x] = max(0, max_{0 <= d < wlen} P[j, x + d]),
 * where dl = 4 win - n_theta, wlen = min(win + dl, n_theta), and e_iS = dl
 * when floor(k_i / win) + S >= 4, else 0 (the window image holds a pixel's
 * 4 maxima at columns k_i mod win + q win, q = 0..3; with 4 | n_theta,
 * dl = 0 and wlen = win). The
 * largest of the 4 window sums bounds max_s Q(b, t, s) of Eq. (1).
 * The window maxima and weights are rounded up to float16 (scaled), summed
 * in float32, and the stored bound is widened by the worst-case float32
 * rounding of both the bound and the plain path's own sum, so that
 *   bound_out[b, t] >= the float32 Q that tm_match_batch computes.
 *
 * Arguments
 *   lib           loaded library (all weights >= 0, n_theta >= 16; the
 *                 window image of the touched rows plus one, (rows + 1) x
 *                 2 win pairs of float16, must fit 128 KiB of LDS, else
 *                 TM_EUNSUPPORTED).
 *   polar, norms  as in tm_match_batch; compact_rows as in tm_fft_scores.
 *   B             >= 0 (0 is a no-op).
 *   bound_out     device, [B, T'] float32, written. A pattern with a
 *                 non-finite norm gets 0 (tm_match_batch flags it).
 * Errors: TM_EINVAL, TM_EUNSUPPORTED, TM_EHIP, TM_ENODEV. */
int tm_bound_scores(const tm_library* lib, const float* polar, const double* norms, int32_t B,
                    int32_t compact_rows, float* bound_out, void* hip_stream);

/* tm_bound_scores_slots - the bounds of tm_bound_scores in the order the
 * kernel produces them (no reordering pass): chunk-slot order, slot
 * c * 64 + l holding template slot_template[c * 64 + l].
 *   bound_out      device, [B, chunks * 64] float32 (chunks from
 *                  tm_bound_layout), written; slots without a template
 *                  (slot_template -1) get the bound of an empty template, 0.
 *   slot_template  host, nullable, [chunks * 64] int32, written: the
 *                  template of each slot, -1 for none.
 * Other arguments and errors as tm_bound_scores. */
int tm_bound_scores_slots(const tm_library* lib, const float* polar, const double* norms,
                          int32_t B, int32_t compact_rows, float* bound_out,
                          int32_t* slot_template, void* hip_stream);

/* tm_bound_layout - the window-bound data of a library, for work accounting
 * (the same exact-search aid as tm_bound_scores).
 *   chunks  out (nullable): chunks of 64 templates, one template per lane.
 *   units   out (nullable): record units per pattern (each 4 records per
 *           lane, 1 KiB per wave; in a chunk each template's four
 *           quarter-turns of pixels, the margin record joining the smallest,
 *           are padded to the chunk's largest, in whole units).
 *   win     out (nullable): shifts per coarse window, ceil(n_theta / 4).
 * Errors: TM_EINVAL (lib NULL), TM_EUNSUPPORTED (no window bounds for this
 * library: a negative weight, n_theta < 16 or an image over the LDS
 * budget). */
int tm_bound_layout(const tm_library* lib, int32_t* chunks, int64_t* units, int32_t* win);

/* tm_fft_error_bound - a-priori bound eps with |Q~ - Q32| <= eps for every
 * template and shift, where Q~ is tm_fft_scores' arithmetic and Q32 the exact
 * float32 path's score (both for the same float32 polar image). It adds the
 * worst-case effect of every float16 rounding (spectra, stored C(k), cosine
 * tables, with subnormals possibly flushed) and of float32 accumulation,
 * bounded through Parseval's identity, and the float32 path's own error.
 * The certified rescoring of tm_match_batch relies on it.
 * Errors: TM_EINVAL (null pointer, library without TM_LIB_FFT). */
int tm_fft_error_bound(const tm_library* lib, double* eps);

/* tm_topn - sort per-template best scores and keep the N best per pattern
 * (Section 2.2, end: sorting the per-template correlations gives the N
 * best templates rather than only the best one).
 *
 * Arguments
 *   best_score   device, [B, T] float32.
 *   best_angle   device, [B, T] int16.
 *   B, T, N      B >= 0, T >= 1, 1 <= N <= min(TM_MAX_N, T).
 *   top_template, top_angle  device, [B, N] int32, written.
 *   top_score    device, [B, N] float32, written.
 * Order: score descending, ties to the lower template index.
 * Errors: TM_EINVAL, TM_EHIP, TM_ENODEV. */
int tm_topn(const float* best_score, const int16_t* best_angle, int32_t B, int32_t T, int32_t N,
            int32_t* top_template, int32_t* top_angle, float* top_score, void* hip_stream);

/* tm_last_error - message of the last failing call on this thread ("" if
 * none). The pointer stays valid until the next call on the same thread. */
const char* tm_last_error(void);

/* tm_version - library version string, e.g. "tm 0.1.0 gfx950". */
const char* tm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
