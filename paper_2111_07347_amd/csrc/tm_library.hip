// tm_load_library / tm_free_library / tm_library_info.
//
// One-time host set-up of a template library (Section 2.1 template format;
// Section 2.2 rounding of spot polar coordinates to integer pixels, mirrors
// across y = 0, precomputed template norms that turn Eq. (1) into a dot
// product). The float64 geometry runs once per library on the host; the
// result is uploaded in the layout the match kernels read:
//
//   * touched rows: the sorted set of polar rows any template has a pixel
//     in. Only these rows are staged into LDS by the match kernels.
//   * bands: touched rows are grouped into bands that fit the LDS budget; a
//     library whose rows fit at once has a single band.
//   * spots: per template (base 0..T-1, then mirrors T..2T-1) its merged
//     pixels as (LDS float offset = local_row * row_width + column, float32
//     weight w/||T||), sorted by (band, offset).
//   * seg: per (template, band) the start of that band's spots, plus the end.
#include <algorithm>
#include <cmath>
#include <cfenv>
#include <cstring>

#include "tm_internal.h"

namespace {

// LDS budget: all touched rows in one band up to this many bytes ...
constexpr size_t kSingleBandBytes = 96 * 1024;
// ... otherwise bands of at most this many bytes.
constexpr size_t kBandBytes = 80 * 1024;

struct Pixel {
    int32_t j, k;
    double w;
};

// Merged polar pixels of one template, sorted by (j, k).
void template_pixels(const double* kx, const double* ky, const double* inten, int64_t a,
                     int64_t b, double px_per, const tm_polar_grid& g, uint32_t flags,
                     std::vector<Pixel>& out) {
    out.clear();
    const double two_pi = 2.0 * M_PI;
    for (int64_t i = a; i < b; ++i) {
        const double x = kx[i], y = ky[i];
        if (!(flags & TM_LIB_KEEP_DIRECT_BEAM) && x == 0.0 && y == 0.0) continue;
        const double rho = px_per * std::hypot(x, y);
        const double jf = std::nearbyint((rho - g.r0) / g.dr);   // round half to even
        if (!(jf >= 0.0 && jf < static_cast<double>(g.R))) continue;
        double kf = std::nearbyint(std::atan2(y, x) * g.n_theta / two_pi);
        long long kk = static_cast<long long>(kf) % g.n_theta;
        if (kk < 0) kk += g.n_theta;
        const double w = (flags & TM_LIB_UNIT_INTENSITY) ? 1.0 : inten[i];
        out.push_back({static_cast<int32_t>(jf), static_cast<int32_t>(kk), w});
    }
    // merge pixels with equal (j, k) by summing weights in spot order
    std::stable_sort(out.begin(), out.end(), [](const Pixel& p, const Pixel& q) {
        return p.j != q.j ? p.j < q.j : p.k < q.k;
    });
    size_t n = 0;
    for (size_t i = 0; i < out.size(); ++i) {
        if (n > 0 && out[n - 1].j == out[i].j && out[n - 1].k == out[i].k)
            out[n - 1].w += out[i].w;
        else
            out[n++] = out[i];
    }
    out.resize(n);
}

}  // namespace

int tmlib::validate_grid(const tm_polar_grid* g) {
    if (!g) { tmlib::set_error("grid is NULL"); return TM_EINVAL; }
    if (g->R < 1 || g->R > 4096) { tmlib::set_error("grid R=%d outside [1, 4096]", g->R); return TM_EINVAL; }
    if (g->n_theta < 64 || g->n_theta > 768) {
        tmlib::set_error("grid n_theta=%d outside [64, 768]", g->n_theta);
        return TM_EINVAL;
    }
    if (!(g->dr > 0.0) || !std::isfinite(g->r0)) { tmlib::set_error("grid needs dr > 0 and finite r0"); return TM_EINVAL; }
    return TM_OK;
}

namespace {

template <typename T>
int upload(T** dst, const std::vector<T>& src, hipStream_t s, size_t& bytes) {
    *dst = nullptr;
    const size_t n = std::max<size_t>(src.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), n);
    if (e != hipSuccess) {
        *dst = nullptr;
        tmlib::set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
        return TM_ENOMEM;
    }
    bytes += n;
    if (!src.empty()) TM_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return TM_OK;
}

void release(tm_library* L) {
    if (!L) return;
    hipFree(L->d_rows);
    hipFree(L->d_band_off);
    hipFree(L->d_spots);
    hipFree(L->d_seg);
    hipFree(L->d_prof);
    hipFree(L->d_prof_norm);
    delete L;
}

}  // namespace

extern "C" int tm_load_library(const double* kx, const double* ky, const double* intensity,
                               const int64_t* offsets, int32_t n_templates,
                               double px_per_inv_angstrom, const tm_polar_grid* grid,
                               uint32_t flags, void* hip_stream, tm_library** out) {
    tmlib::clear_error();
    if (out) *out = nullptr;
    if (!out || !offsets) { tmlib::set_error("out and offsets must be non-NULL"); return TM_EINVAL; }
    if (n_templates < 1 || n_templates > (1 << 29)) { tmlib::set_error("n_templates=%d outside [1, 2^29]", n_templates); return TM_EINVAL; }
    if (int r = tmlib::validate_grid(grid)) return r;
    if (!(px_per_inv_angstrom > 0.0) || !std::isfinite(px_per_inv_angstrom)) {
        tmlib::set_error("px_per_inv_angstrom must be positive and finite");
        return TM_EINVAL;
    }
    if (flags & ~7u) { tmlib::set_error("unknown library flags 0x%x", flags); return TM_EINVAL; }
    if (offsets[0] != 0) { tmlib::set_error("offsets[0] must be 0"); return TM_EINVAL; }
    for (int32_t t = 0; t < n_templates; ++t)
        if (offsets[t + 1] < offsets[t]) { tmlib::set_error("offsets decrease at template %d", t); return TM_EINVAL; }
    const int64_t n_in = offsets[n_templates];
    if (n_in > 0 && (!kx || !ky || (!intensity && !(flags & TM_LIB_UNIT_INTENSITY)))) {
        tmlib::set_error("kx, ky and intensity must be non-NULL");
        return TM_EINVAL;
    }
    if (int r = tmlib::require_device()) return r;

    const tm_polar_grid g = *grid;
    const bool mirror = flags & TM_LIB_MIRROR;
    const int32_t T = n_templates;
    const int32_t Tp = mirror ? 2 * T : T;
    const int n_theta = g.n_theta;

    // 1. merged pixels and norms of the base templates (float64)
    std::fesetround(FE_TONEAREST);
    std::vector<std::vector<Pixel>> pix(T);
    std::vector<Pixel> tmp;
    std::vector<double> tnorm(Tp, 0.0);
    std::vector<char> row_used(g.R, 0);
    for (int32_t t = 0; t < T; ++t) {
        template_pixels(kx, ky, intensity, offsets[t], offsets[t + 1], px_per_inv_angstrom, g,
                        flags, tmp);
        pix[t] = tmp;
        double s = 0.0;
        for (const Pixel& p : tmp) {
            s += p.w * p.w;
            row_used[p.j] = 1;
        }
        tnorm[t] = std::sqrt(s);
        if (mirror) tnorm[T + t] = tnorm[t];
    }

    // 2. touched rows and bands
    std::vector<int32_t> rows;
    std::vector<int32_t> row_index(g.R, -1);
    for (int j = 0; j < g.R; ++j)
        if (row_used[j]) { row_index[j] = static_cast<int32_t>(rows.size()); rows.push_back(j); }
    const int32_t n_rows = static_cast<int32_t>(rows.size());
    const int row_width = tmlib::lds_row_width(n_theta);
    const size_t row_bytes = static_cast<size_t>(row_width) * sizeof(float);
    int32_t n_bands = 1, band_rows = std::max<int32_t>(n_rows, 1);
    if (static_cast<size_t>(n_rows) * row_bytes > kSingleBandBytes) {
        const int32_t max_rows = static_cast<int32_t>(kBandBytes / row_bytes);
        if (max_rows < 1) { tmlib::set_error("n_theta=%d too wide for an LDS band", n_theta); return TM_EUNSUPPORTED; }
        n_bands = (n_rows + max_rows - 1) / max_rows;
        band_rows = (n_rows + n_bands - 1) / n_bands;
    }
    std::vector<int32_t> band_off(n_bands + 1);
    for (int b = 0; b <= n_bands; ++b) band_off[b] = std::min(n_rows, b * band_rows);

    // 3. packed spots per (template, band)
    struct Spot { int32_t band; uint32_t off; float w; };
    std::vector<uint2> spots;
    std::vector<int32_t> seg(static_cast<size_t>(Tp) * (n_bands + 1));
    std::vector<Spot> ts;
    for (int32_t tt = 0; tt < Tp; ++tt) {
        const int32_t t = tt < T ? tt : tt - T;
        const bool is_mirror = tt >= T;
        const double nrm = tnorm[t];
        ts.clear();
        for (const Pixel& p : pix[t]) {
            const int32_t ri = row_index[p.j];
            const int32_t band = ri / band_rows;
            const int32_t local = ri - band * band_rows;
            const int32_t k = is_mirror ? (n_theta - p.k) % n_theta : p.k;
            const float w = nrm > 0.0 ? static_cast<float>(p.w / nrm) : 0.0f;
            ts.push_back({band, static_cast<uint32_t>(local * row_width + k), w});
        }
        std::sort(ts.begin(), ts.end(), [](const Spot& a, const Spot& b) {
            return a.band != b.band ? a.band < b.band : a.off < b.off;
        });
        size_t base = static_cast<size_t>(tt) * (n_bands + 1);
        size_t i = 0;
        for (int b = 0; b < n_bands; ++b) {
            seg[base + b] = static_cast<int32_t>(spots.size() + i);
            while (i < ts.size() && ts[i].band == b) ++i;
        }
        seg[base + n_bands] = static_cast<int32_t>(spots.size() + ts.size());
        for (const Spot& s : ts) {
            uint32_t wb;
            std::memcpy(&wb, &s.w, 4);
            spots.push_back(make_uint2(s.off, wb));
        }
        if (spots.size() > static_cast<size_t>(INT32_MAX)) { tmlib::set_error("library too large"); return TM_EINVAL; }
    }

    // 4. radial profiles of the base templates, normalised (Fig. 3)
    std::vector<float> prof(static_cast<size_t>(T) * g.R, 0.0f), prof_norm(T, 0.0f);
    std::vector<double> acc(g.R);
    for (int32_t t = 0; t < T; ++t) {
        std::fill(acc.begin(), acc.end(), 0.0);
        for (const Pixel& p : pix[t]) acc[p.j] += p.w;
        double s = 0.0;
        for (int j = 0; j < g.R; ++j) s += acc[j] * acc[j];
        s = std::sqrt(s);
        prof_norm[t] = static_cast<float>(s);
        for (int j = 0; j < g.R; ++j)
            prof[static_cast<size_t>(t) * g.R + j] = s > 0.0 ? static_cast<float>(acc[j] / s) : 0.0f;
    }

    // 5. upload
    auto* L = new tm_library();
    L->T = T;
    L->Tp = Tp;
    L->R = g.R;
    L->n_theta = n_theta;
    L->r0 = g.r0;
    L->dr = g.dr;
    L->px_per = px_per_inv_angstrom;
    L->flags = flags;
    hipGetDevice(&L->device);
    L->n_rows = n_rows;
    L->n_bands = n_bands;
    L->band_rows = band_rows;
    L->row_width = row_width;
    L->n_spots = static_cast<int64_t>(spots.size());
    L->tnorm = tnorm;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int r = TM_OK;
    size_t bytes = 0;
    if (!r) r = upload(&L->d_rows, rows, s, bytes);
    if (!r) r = upload(&L->d_band_off, band_off, s, bytes);
    if (!r) r = upload(&L->d_spots, spots, s, bytes);
    if (!r) r = upload(&L->d_seg, seg, s, bytes);
    if (!r) r = upload(&L->d_prof, prof, s, bytes);
    if (!r) r = upload(&L->d_prof_norm, prof_norm, s, bytes);
    if (!r) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) r = tmlib::hip_fail(e, "hipStreamSynchronize");
    }
    if (r) {
        release(L);
        return r;
    }
    L->device_bytes = bytes;
    *out = L;
    return TM_OK;
}

extern "C" int tm_free_library(tm_library* lib) {
    tmlib::clear_error();
    release(lib);
    return TM_OK;
}

extern "C" int tm_library_info(const tm_library* lib, int32_t* n_templates_total, int64_t* n_spots,
                               size_t* device_bytes) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (n_templates_total) *n_templates_total = lib->Tp;
    if (n_spots) *n_spots = lib->n_spots;
    if (device_bytes) *device_bytes = lib->device_bytes;
    return TM_OK;
}
