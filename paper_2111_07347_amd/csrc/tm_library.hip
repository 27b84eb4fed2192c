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
#include <unordered_map>

#include "tm_internal.h"

namespace {

// LDS budgets: a band small enough for two workgroups per CU, the most a
// single workgroup may stage, and the band size when rows must be streamed.
constexpr size_t kSharedCuBytes = 76 * 1024;
constexpr size_t kSingleBandBytes = 160 * 1024;   // all of a CU's LDS
constexpr size_t kBandBytes = 76 * 1024;

using Pixel = tmlib::HostPixel;

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


// Greedy grouping of templates into groups of G that share polar pixels
// (pixel key = band << 32 | LDS offset). Each group starts from the lowest
// unassigned template and repeatedly adds the unassigned template sharing
// the most pixels with the group's union (lowest index on ties; the next
// unassigned template if none shares any). Returns the total union size;
// members holds G entries per group, -1 for empty slots.
template <typename SpotVecs>
int64_t group_templates(const SpotVecs& tsp, int G, std::vector<int32_t>& members) {
    const int32_t Tp = static_cast<int32_t>(tsp.size());
    std::unordered_map<uint64_t, std::vector<int32_t>> inv;
    for (int32_t t = 0; t < Tp; ++t)
        for (const auto& s : tsp[t]) inv[(static_cast<uint64_t>(s.band) << 32) | s.off].push_back(t);
    std::vector<char> used(Tp, 0);
    std::vector<int32_t> cnt(Tp, 0), touched;
    std::vector<uint64_t> uni;
    members.clear();
    int64_t total = 0;
    int32_t next_free = 0;
    for (int32_t t0 = 0; t0 < Tp; ++t0) {
        if (used[t0]) continue;
        used[t0] = 1;
        members.push_back(t0);
        uni.clear();
        for (const auto& s : tsp[t0]) uni.push_back((static_cast<uint64_t>(s.band) << 32) | s.off);
        for (int g = 1; g < G; ++g) {
            touched.clear();
            for (uint64_t key : uni)
                for (int32_t v : inv[key])
                    if (!used[v]) {
                        if (cnt[v] == 0) touched.push_back(v);
                        ++cnt[v];
                    }
            int32_t best = -1;
            for (int32_t v : touched)
                if (best < 0 || cnt[v] > cnt[best] || (cnt[v] == cnt[best] && v < best)) best = v;
            for (int32_t v : touched) cnt[v] = 0;
            if (best < 0) {
                while (next_free < Tp && used[next_free]) ++next_free;
                if (next_free < Tp) best = next_free;
            }
            if (best < 0) { members.push_back(-1); continue; }
            used[best] = 1;
            members.push_back(best);
            for (const auto& s : tsp[best]) uni.push_back((static_cast<uint64_t>(s.band) << 32) | s.off);
            std::sort(uni.begin(), uni.end());
            uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
        }
        std::sort(uni.begin(), uni.end());
        uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
        total += static_cast<int64_t>(uni.size());
    }
    return total;
}

// Estimated match cost (CU clocks) of scoring all templates from `records`
// union pixels with groups of G: per union pixel the larger of the LDS time
// (K wave-wide 4-byte reads at ~110 B/clk/CU) and the VALU time (one address
// add and G*K FMAs at ~1.5 wave instructions per clock per CU), plus a fixed
// per-template cost for the maximum and the top-N test.
double group_cost(int64_t records, int32_t Tp, int G, int K, int n_bands) {
    const double lds = 256.0 * K / 110.0;
    const double valu = (1.0 + G * K) / 1.5;
    (void)n_bands;
    return static_cast<double>(records) * std::max(lds, valu) + Tp * 14.0;
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
    (void)hipFree(L->d_rows);
    (void)hipFree(L->d_row_map);
    (void)hipFree(L->d_band_off);
    (void)hipFree(L->d_recs);
    (void)hipFree(L->d_members);
    (void)hipFree(L->d_recs1);
    (void)hipFree(L->d_seg1);
    (void)hipFree(L->d_seg);
    (void)hipFree(L->d_prof);
    (void)hipFree(L->d_prof_max);
    tmlib::fft_release(L);
    tmlib::bound_release(L);
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
    if (flags & ~31u) { tmlib::set_error("unknown library flags 0x%x", flags); return TM_EINVAL; }
    if ((flags & TM_LIB_FFT) && (grid->n_theta % 2)) {
        tmlib::set_error("TM_LIB_FFT needs an even n_theta (got %d)", grid->n_theta);
        return TM_EUNSUPPORTED;
    }
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
    // Row layout. Wide rows carry a halo long enough that every shift slot
    // reads past the row end without wrapping; narrow rows carry only one
    // wave of halo, and each pixel records how many of its K slot reads come
    // before the wrap (its class), the rest reading one period back.
    const int K = tmlib::slots_for(n_theta);
    const size_t wide_bytes = static_cast<size_t>(tmlib::wide_row_width(n_theta)) * sizeof(float);
    const size_t narrow_bytes = static_cast<size_t>(tmlib::narrow_row_width(n_theta)) * sizeof(float);
    bool narrow = false;
    size_t budget = kSingleBandBytes;
    if (static_cast<size_t>(n_rows) * wide_bytes <= kSharedCuBytes) {
        narrow = false;
    } else if (K <= tmlib::kMaxNarrowSlots) {
        narrow = true;
        if (static_cast<size_t>(n_rows) * narrow_bytes > kSingleBandBytes) budget = kBandBytes;
    } else if (static_cast<size_t>(n_rows) * wide_bytes > kSingleBandBytes) {
        budget = kBandBytes;
    }
    const int row_width = narrow ? tmlib::narrow_row_width(n_theta) : tmlib::wide_row_width(n_theta);
    const size_t row_bytes = static_cast<size_t>(row_width) * sizeof(float);
    const int n_cls = narrow ? K : 1;
    int32_t n_bands = 1, band_rows = std::max<int32_t>(n_rows, 1);
    if (static_cast<size_t>(n_rows) * row_bytes > budget) {
        const int32_t max_rows = static_cast<int32_t>(budget / row_bytes);
        if (max_rows < 1) { tmlib::set_error("n_theta=%d too wide for an LDS band", n_theta); return TM_EUNSUPPORTED; }
        n_bands = (n_rows + max_rows - 1) / max_rows;
        band_rows = (n_rows + n_bands - 1) / n_bands;
    }
    std::vector<int32_t> band_off(n_bands + 1);
    for (int b = 0; b <= n_bands; ++b) band_off[b] = std::min(n_rows, b * band_rows);
    // class of a pixel at column q: slot reads k with q + 64 k < n_theta
    auto pixel_class = [&](uint32_t off) -> int {
        if (!narrow) return 0;
        const int q = static_cast<int>(off % static_cast<uint32_t>(row_width));
        return std::min(K, (n_theta - q + 63) / 64) - 1;
    };

    // 3. per template its pixels as (band, LDS float offset, weight w/||T||)
    struct Spot { int32_t band; uint32_t off; float w; };
    std::vector<std::vector<Spot>> tsp(Tp);
    for (int32_t tt = 0; tt < Tp; ++tt) {
        const int32_t t = tt < T ? tt : tt - T;
        const bool is_mirror = tt >= T;
        const double nrm = tnorm[t];
        auto& ts = tsp[tt];
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
    }
    int64_t n_pixels = 0;
    for (const auto& ts : tsp) n_pixels += static_cast<int64_t>(ts.size());

    // 4. group templates that share pixels: a group's union pixel is read
    // from LDS once and applied to every member (zero weight if absent)
    std::vector<int32_t> members;
    int G = 1;
    if (!(flags & TM_LIB_NO_GROUPING)) {
        std::vector<int32_t> m3;
        const int64_t u3 = group_templates(tsp, 3, m3);
        const double c1 = group_cost(n_pixels, Tp, 1, K, n_bands);
        const double c3 = group_cost(u3, Tp, 3, K, n_bands);
        if (c3 < c1) { G = 3; members.swap(m3); }
    }
    if (G == 1) {
        members.resize(Tp);
        for (int32_t t = 0; t < Tp; ++t) members[t] = t;
    }
    const int32_t n_groups = static_cast<int32_t>(members.size() / G);

    // 5. records per (group, band, class): union pixel offset + one weight
    // per member (zero when the member lacks the pixel)
    auto build_records = [&](int G, const std::vector<int32_t>& members,
                             std::vector<uint32_t>& recs, std::vector<int32_t>& seg) -> int {
        const int32_t n_groups = static_cast<int32_t>(members.size() / G);
        const size_t n_seg = static_cast<size_t>(n_groups) * n_bands * n_cls;
        recs.clear();
        seg.assign(n_seg + 1, 0);
        struct UEnt { uint64_t key; int g; float w; };
        std::vector<UEnt> u;   // key = (band << 40 | class << 32 | off), member, weight
        std::vector<float> w_of;
        const size_t rec_words = static_cast<size_t>(G) + 1;
        for (int32_t gi = 0; gi < n_groups; ++gi) {
            u.clear();
            for (int g = 0; g < G; ++g) {
                const int32_t tt = members[static_cast<size_t>(gi) * G + g];
                if (tt < 0) continue;
                for (const Spot& s : tsp[tt])
                    u.push_back({(static_cast<uint64_t>(s.band) << 40) |
                                     (static_cast<uint64_t>(pixel_class(s.off)) << 32) | s.off,
                                 g, s.w});
            }
            std::sort(u.begin(), u.end(), [](const UEnt& a, const UEnt& b) {
                return a.key != b.key ? a.key < b.key : a.g < b.g;
            });
            const size_t base = static_cast<size_t>(gi) * n_bands * n_cls;
            size_t next = 0;   // next segment of this group to open
            for (size_t i = 0; i < u.size();) {
                const uint64_t key = u[i].key;
                const size_t sidx = static_cast<size_t>(key >> 40) * n_cls + ((key >> 32) & 0xff);
                while (next <= sidx) seg[base + next++] = static_cast<int32_t>(recs.size() / rec_words);
                w_of.assign(G, 0.0f);
                for (; i < u.size() && u[i].key == key; ++i) w_of[u[i].g] = u[i].w;
                recs.push_back(static_cast<uint32_t>(key & 0xffffffffu));
                for (int g = 0; g < G; ++g) {
                    uint32_t wb;
                    std::memcpy(&wb, &w_of[g], 4);
                    recs.push_back(wb);
                }
            }
            while (next < static_cast<size_t>(n_bands) * n_cls)
                seg[base + next++] = static_cast<int32_t>(recs.size() / rec_words);
            if (recs.size() / rec_words > static_cast<size_t>(INT32_MAX)) {
                tmlib::set_error("library too large");
                return TM_EINVAL;
            }
        }
        seg[n_seg] = static_cast<int32_t>(recs.size() / rec_words);
        return TM_OK;
    };
    std::vector<uint32_t> recs, recs1;
    std::vector<int32_t> seg, seg1;
    if (int r = build_records(G, members, recs, seg)) return r;
    // per-template records (one template per "group") for rescoring an
    // arbitrary candidate list; the same arrays when G = 1
    if (G != 1) {
        std::vector<int32_t> ident(Tp);
        for (int32_t t = 0; t < Tp; ++t) ident[t] = t;
        if (int r = build_records(1, ident, recs1, seg1)) return r;
    }

    // 6. radial profiles of the base templates, normalised (Fig. 3)
    std::vector<float> prof(static_cast<size_t>(T) * g.R, 0.0f), prof_max(T, 0.0f);
    std::vector<double> acc(g.R);
    for (int32_t t = 0; t < T; ++t) {
        std::fill(acc.begin(), acc.end(), 0.0);
        for (const Pixel& p : pix[t]) acc[p.j] += p.w;
        double s = 0.0;
        for (int j = 0; j < g.R; ++j) s += acc[j] * acc[j];
        s = std::sqrt(s);
        float mx = 0.0f;
        for (int j = 0; j < g.R; ++j) {
            const float v = s > 0.0 ? static_cast<float>(acc[j] / s) : 0.0f;
            prof[static_cast<size_t>(t) * g.R + j] = v;
            mx = std::max(mx, std::fabs(v));
        }
        prof_max[t] = mx;
    }

    // 7. upload
    auto* L = new tm_library();
    L->T = T;
    L->Tp = Tp;
    L->R = g.R;
    L->n_theta = n_theta;
    L->r0 = g.r0;
    L->dr = g.dr;
    L->px_per = px_per_inv_angstrom;
    L->flags = flags;
    (void)hipGetDevice(&L->device);
    L->n_rows = n_rows;
    L->n_bands = n_bands;
    L->band_rows = band_rows;
    L->row_width = row_width;
    L->narrow = narrow;
    L->n_cls = n_cls;
    L->n_spots = n_pixels;
    L->group = G;
    L->n_groups = n_groups;
    L->n_records = static_cast<int64_t>(recs.size() / (G + 1));
    L->tnorm = tnorm;
    L->row_index = row_index;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int r = TM_OK;
    size_t bytes = 0;
    if (!r) r = upload(&L->d_rows, rows, s, bytes);
    if (!r) r = upload(&L->d_row_map, row_index, s, bytes);
    if (!r) r = upload(&L->d_band_off, band_off, s, bytes);
    if (!r) r = upload(&L->d_recs, recs, s, bytes);
    if (!r) r = upload(&L->d_seg, seg, s, bytes);
    if (!r) r = upload(&L->d_members, members, s, bytes);
    if (!r && G != 1) r = upload(&L->d_recs1, recs1, s, bytes);
    if (!r && G != 1) r = upload(&L->d_seg1, seg1, s, bytes);
    if (!r) r = upload(&L->d_prof, prof, s, bytes);
    if (!r) r = upload(&L->d_prof_max, prof_max, s, bytes);
    if (!r && (flags & TM_LIB_FFT)) r = tmlib::fft_prepare(L, pix, s, bytes);
    if (!r) r = tmlib::bound_prepare(L, pix, row_index, s, bytes);
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

extern "C" int tm_library_rows(const tm_library* lib, int32_t* n_rows,
                               const int32_t** row_map) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (n_rows) *n_rows = lib->n_rows;
    if (row_map) *row_map = lib->d_row_map;
    return TM_OK;
}

extern "C" int tm_library_layout(const tm_library* lib, int32_t* group, int32_t* n_bands,
                                 int32_t* n_rows, int64_t* n_records, int32_t* row_width) {
    tmlib::clear_error();
    if (!lib) { tmlib::set_error("library is NULL"); return TM_EINVAL; }
    if (group) *group = lib->group;
    if (n_bands) *n_bands = lib->n_bands;
    if (n_rows) *n_rows = lib->n_rows;
    if (n_records) *n_records = lib->n_records;
    if (row_width) *row_width = lib->row_width;
    return TM_OK;
}
