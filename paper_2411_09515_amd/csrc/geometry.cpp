// Host-side geometry: the CSR pixel-to-bin matrix and the packed radial
// coordinate of every pixel (Sec. 2.2 "Azimuthal averaging", Sec. 3).
//
// Angles are computed in float64; the bin of an angle a is floor(a / w) with
// w = 2theta_max / n_bins, the last bin closed at 2theta_max.  Bounding-box
// splitting shares a pixel between the bins its corner-angle interval
// overlaps, in proportion to the overlap.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

#include "sigsep.h"

namespace {

constexpr double kDeg = 180.0 / 3.14159265358979323846;

inline double angle_deg(double dy, double dx, double pixel_m, double dist_m) {
    return std::atan(pixel_m * std::sqrt(dy * dy + dx * dx) / dist_m) * kDeg;
}

struct Corners {
    int32_t h, w;
    std::vector<double> a;  // [(h + 1) * (w + 1)]
    double max = 0.0;
    Corners(int32_t height, int32_t width, double pixel_m, double dist_m, double cy, double cx)
        : h(height), w(width), a(size_t(height + 1) * size_t(width + 1)) {
        for (int32_t y = 0; y <= h; ++y)
            for (int32_t x = 0; x <= w; ++x) {
                double v = angle_deg(double(y) - cy, double(x) - cx, pixel_m, dist_m);
                a[size_t(y) * size_t(w + 1) + size_t(x)] = v;
                max = std::max(max, v);
            }
    }
    double at(int32_t y, int32_t x) const { return a[size_t(y) * size_t(w + 1) + size_t(x)]; }
};

// Calls fn(bin, coef) for every bin that pixel (y, x) contributes to.
template <class Fn>
inline void pixel_entries(const Corners &cn, int32_t y, int32_t x, double cy, double cx,
                          double pixel_m, double dist_m, int32_t n_bins, int32_t split, Fn &&fn) {
    const double tmax = cn.max;
    const double w = tmax / n_bins;
    if (split == SS_SPLIT_NONE) {
        double t = angle_deg(y + 0.5 - cy, x + 0.5 - cx, pixel_m, dist_m);
        int64_t b = int64_t(std::floor(t / w));
        if (b > n_bins - 1) b = n_bins - 1;
        if (b < 0) b = 0;
        fn(int32_t(b), 1.0);
        return;
    }
    double c00 = cn.at(y, x), c01 = cn.at(y, x + 1), c10 = cn.at(y + 1, x), c11 = cn.at(y + 1, x + 1);
    double lo = std::min(std::min(c00, c01), std::min(c10, c11));
    double hi = std::max(std::max(c00, c01), std::max(c10, c11));
    if (y == int32_t(std::floor(cy)) && x == int32_t(std::floor(cx))) lo = 0.0;
    const double span = hi - lo;
    int64_t r0 = int64_t(std::floor(lo / w)) - 1, r1 = int64_t(std::floor(hi / w)) + 1;
    r0 = std::max<int64_t>(r0, 0);
    r1 = std::min<int64_t>(r1, n_bins - 1);
    for (int64_t r = r0; r <= r1; ++r) {
        double lower = double(r) * w;
        double upper = (r == n_bins - 1) ? tmax : double(r + 1) * w;
        double ov = std::min(hi, upper) - std::max(lo, lower);
        if (ov > 0.0) fn(int32_t(r), ov / span);
    }
}

bool geometry_ok(int32_t height, int32_t width, double pixel_m, double dist_m, int32_t n_bins) {
    return height > 0 && width > 0 && pixel_m > 0.0 && dist_m > 0.0 && n_bins > 0 &&
           std::isfinite(pixel_m) && std::isfinite(dist_m);
}

}  // namespace

extern "C" int ss_build_csr(int32_t height, int32_t width, double pixel_m, double dist_m,
                            double centre_row, double centre_col, int32_t n_bins, int32_t split,
                            const uint8_t *mask, const float *norm, int64_t *indptr,
                            int32_t *indices, float *weight, int64_t capacity, int64_t *nnz,
                            int32_t *max_row, double *tth_max) {
    if (!nnz || !max_row || !tth_max) return SS_EINVAL;
    if (split != SS_SPLIT_NONE && split != SS_SPLIT_BBOX) return SS_EINVAL;
    if (!std::isfinite(centre_row) || !std::isfinite(centre_col)) return SS_EINVAL;
    if (!geometry_ok(height, width, pixel_m, dist_m, n_bins)) return SS_ESIZE;
    const int64_t n_pix = int64_t(height) * int64_t(width);
    if (n_pix >= (int64_t(1) << 31) || n_bins > SS_MAX_BINS) return SS_ESIZE;

    Corners cn(height, width, pixel_m, dist_m, centre_row, centre_col);
    *tth_max = cn.max;
    std::vector<int64_t> count(size_t(n_bins), 0);
    for (int32_t y = 0; y < height; ++y)
        for (int32_t x = 0; x < width; ++x) {
            int64_t i = int64_t(y) * width + x;
            if (mask && mask[i]) continue;
            pixel_entries(cn, y, x, centre_row, centre_col, pixel_m, dist_m, n_bins, split,
                          [&](int32_t r, double) { ++count[size_t(r)]; });
        }
    int64_t total = 0, longest = 0;
    for (int64_t c : count) {
        total += c;
        longest = std::max(longest, c);
    }
    *nnz = total;
    *max_row = int32_t(longest);
    if (!indices) return SS_OK;
    if (!indptr || !weight) return SS_EINVAL;
    if (capacity < total || total >= (int64_t(1) << 31)) return SS_ESIZE;

    indptr[0] = 0;
    for (int32_t r = 0; r < n_bins; ++r) indptr[r + 1] = indptr[r] + count[size_t(r)];
    std::vector<int64_t> fill(indptr, indptr + n_bins);
    // pixels are visited in ascending index, so every row comes out sorted
    for (int32_t y = 0; y < height; ++y)
        for (int32_t x = 0; x < width; ++x) {
            int64_t i = int64_t(y) * width + x;
            if (mask && mask[i]) continue;
            double nrm = norm ? double(norm[i]) : 1.0;
            pixel_entries(cn, y, x, centre_row, centre_col, pixel_m, dist_m, n_bins, split,
                          [&](int32_t r, double c) {
                              int64_t j = fill[size_t(r)]++;
                              indices[j] = int32_t(i);
                              weight[j] = float(c * nrm);
                          });
        }
    return SS_OK;
}

extern "C" int ss_radial_coords(int32_t height, int32_t width, double pixel_m, double dist_m,
                                double centre_row, double centre_col, int32_t n_bins,
                                double tth_max, const uint8_t *mask, uint32_t *rcoord,
                                double *centre0, double *width_out) {
    if (!rcoord || !centre0 || !width_out) return SS_EINVAL;
    if (!std::isfinite(centre_row) || !std::isfinite(centre_col) || !(tth_max > 0.0))
        return SS_EINVAL;
    if (!geometry_ok(height, width, pixel_m, dist_m, n_bins)) return SS_ESIZE;
    if (n_bins > SS_MAX_BINS || int64_t(height) * width >= (int64_t(1) << 31)) return SS_ESIZE;
    const double w = tth_max / n_bins;
    const double c0 = 0.5 * w;
    const double scale = double(1u << SS_RC_FRAC_BITS);
    const uint32_t fmax = (1u << SS_RC_FRAC_BITS) - 1u;
    *centre0 = c0;
    *width_out = w;
    for (int32_t y = 0; y < height; ++y)
        for (int32_t x = 0; x < width; ++x) {
            int64_t i = int64_t(y) * width + x;
            if (mask && mask[i]) {
                rcoord[i] = SS_RC_MASKED;
                continue;
            }
            double pos = angle_deg(y + 0.5 - centre_row, x + 0.5 - centre_col, pixel_m, dist_m);
            double s = (pos - c0) / w;
            int64_t t = int64_t(std::floor(s));
            if (t < -1) t = -1;
            if (t > n_bins - 1) t = n_bins - 1;
            uint32_t frac = 0;
            if (t >= 0 && t <= n_bins - 2) {
                double f = (s - double(t)) * scale;
                frac = f <= 0.0 ? 0u : (f >= double(fmax) ? fmax : uint32_t(f));
            }
            rcoord[i] = (uint32_t(t + 1) << SS_RC_FRAC_BITS) | frac;
        }
    return SS_OK;
}

namespace {
// Longest row of each class but the last (which takes any length); the clip
// sizes its work-groups to these (work-group threads x values per thread).
constexpr int32_t kClassRows[SS_N_CLASSES - 1] = {1024, 2048, 4096, 8192, 16384, 24576, 51200};
}  // namespace

extern "C" int32_t ss_class_rows(int32_t c) {
    return (c >= 0 && c < SS_N_CLASSES - 1) ? kClassRows[c] : 0;
}

extern "C" int ss_csr_schedule(const int64_t *indptr, int32_t n_bins, int32_t *bin_order, int32_t *class_count) {
    if (!indptr || !bin_order || !class_count) return SS_EINVAL;
    if (n_bins <= 0 || n_bins > SS_MAX_BINS) return SS_ESIZE;
    std::vector<int32_t> cls(static_cast<size_t>(n_bins), 0);
    for (int32_t c = 0; c < SS_N_CLASSES; ++c) class_count[c] = 0;
    for (int32_t r = 0; r < n_bins; ++r) {
        const int64_t len = indptr[r + 1] - indptr[r];
        if (len < 0) return SS_EINVAL;
        int32_t c = 0;
        while (c < SS_N_CLASSES - 1 && len > kClassRows[c]) ++c;
        cls[size_t(r)] = c;
        ++class_count[c];
    }
    int32_t at = 0;
    for (int32_t c = SS_N_CLASSES - 1; c >= 0; --c)
        for (int32_t r = 0; r < n_bins; ++r)
            if (cls[size_t(r)] == c) bin_order[at++] = r;
    return SS_OK;
}

namespace {

bool pow2(int32_t v) { return v > 0 && (v & (v - 1)) == 0; }

int64_t tiles_x_of(const ss_layout &l) { return (int64_t(l.width) + l.tile_w - 1) / l.tile_w; }

// Word of pixel (y, x) in a layout (the formula of ss_layout).
int64_t word_of(const ss_layout &l, int64_t tiles_x, int64_t y, int64_t x) {
    if (l.tile_w == 0) return y * l.width + x;
    return ((y / l.tile_h) * tiles_x + x / l.tile_w) * (int64_t(l.tile_w) * l.tile_h) + (y % l.tile_h) * l.tile_w +
           x % l.tile_w;
}

}  // namespace

extern "C" int64_t ss_layout_words(const ss_layout *l) {
    if (!l) return SS_EINVAL;
    if (l->height <= 0 || l->width <= 0) return SS_ESIZE;
    const int64_t n = int64_t(l->height) * l->width;
    if (n >= (int64_t(1) << 31)) return SS_ESIZE;
    if (l->tile_w == 0 && l->tile_h == 0) return n;
    if (!pow2(l->tile_w) || !pow2(l->tile_h) || l->tile_w < 4 || l->tile_w > 64 || l->tile_h > 64) return SS_ESIZE;
    const int64_t ty = (int64_t(l->height) + l->tile_h - 1) / l->tile_h;
    const int64_t words = tiles_x_of(*l) * ty * l->tile_w * l->tile_h;
    return words >= (int64_t(1) << 31) ? SS_ESIZE : words;
}

extern "C" int ss_csr_relayout(const ss_layout *layout, int32_t n_bins, const int64_t *indptr, int32_t *indices,
                               float *weight) {
    if (!layout || !indptr) return SS_EINVAL;
    const int64_t words = ss_layout_words(layout);
    if (words < 0) return int(words);
    if (n_bins <= 0 || n_bins > SS_MAX_BINS) return SS_ESIZE;
    if (indptr[0] != 0) return SS_EINVAL;
    for (int32_t r = 0; r < n_bins; ++r)
        if (indptr[r + 1] < indptr[r]) return SS_EINVAL;
    const int64_t nnz = indptr[n_bins];
    if (nnz == 0) return SS_OK;
    if (!indices || !weight) return SS_EINVAL;
    const int64_t n_pix = int64_t(layout->height) * layout->width;
    for (int64_t j = 0; j < nnz; ++j)
        if (indices[j] < 0 || indices[j] >= n_pix) return SS_EINVAL;  // checked before anything is rewritten
    const int64_t tx = layout->tile_w == 0 ? 1 : tiles_x_of(*layout);
    std::vector<std::pair<int32_t, float>> row;
    for (int32_t r = 0; r < n_bins; ++r) {
        row.clear();
        for (int64_t j = indptr[r]; j < indptr[r + 1]; ++j) {
            const int64_t p = indices[j];
            row.emplace_back(int32_t(word_of(*layout, tx, p / layout->width, p % layout->width)), weight[j]);
        }
        std::stable_sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
        int64_t j = indptr[r];
        for (const auto &e : row) {
            indices[j] = e.first;
            weight[j] = e.second;
            ++j;
        }
    }
    return SS_OK;
}

extern "C" int ss_layout_scatter(const ss_layout *layout, const float *src, float fill, float *dst) {
    if (!layout || !src || !dst) return SS_EINVAL;
    const int64_t words = ss_layout_words(layout);
    if (words < 0) return int(words);
    for (int64_t o = 0; o < words; ++o) dst[o] = fill;
    const int64_t tx = layout->tile_w == 0 ? 1 : tiles_x_of(*layout);
    for (int64_t y = 0; y < layout->height; ++y)
        for (int64_t x = 0; x < layout->width; ++x) dst[word_of(*layout, tx, y, x)] = src[y * layout->width + x];
    return SS_OK;
}

extern "C" const char *ss_strerror(int code) {
    switch (code) {
        case SS_OK: return "ok";
        case SS_EINVAL: return "invalid argument";
        case SS_ESIZE: return "size out of range";
        case SS_EHIP: return "HIP runtime error";
        default: return "unknown error";
    }
}

extern "C" int ss_version(void) { return 100; }
