// Host checks of the geometry entry points (CSR builder, radial codes, row
// schedule, error strings), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_geometry_sanitizers.py.  Every
// buffer is sized exactly to what the call may touch, so an overrun is a
// sanitizer report; a failed property prints its name and exits 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sigsep.h"

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);    \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

struct Scene {
    int32_t h, w, n_bins, split;
    double pixel_m, dist_m, cy, cx;
    bool masked, normed;
};

static uint32_t lcg(uint32_t &s) { return s = s * 1664525u + 1013904223u; }

static void check_scene(const Scene &s) {
    const int64_t n = int64_t(s.h) * s.w;
    uint32_t seed = uint32_t(n * 2654435761u) ^ uint32_t(s.n_bins);
    std::vector<uint8_t> mask(size_t(n), 0);
    std::vector<float> norm(size_t(n), 1.0f);
    for (int64_t i = 0; i < n; ++i) {
        if (s.masked) mask[size_t(i)] = (lcg(seed) >> 24) < 20 ? 1 : 0;
        if (s.normed) norm[size_t(i)] = 0.5f + float(lcg(seed) >> 8) / float(1u << 24);
    }
    const uint8_t *mp = s.masked ? mask.data() : nullptr;
    const float *np = s.normed ? norm.data() : nullptr;

    // sizes, then an exactly sized fill
    int64_t nnz = -1;
    int32_t max_row = -1;
    double tth = -1.0;
    CHECK(ss_build_csr(s.h, s.w, s.pixel_m, s.dist_m, s.cy, s.cx, s.n_bins, s.split, mp, np, nullptr, nullptr,
                       nullptr, 0, &nnz, &max_row, &tth) == SS_OK);
    CHECK(nnz >= 0 && max_row >= 0 && tth > 0.0);
    std::vector<int64_t> indptr(static_cast<size_t>(s.n_bins) + 1);
    std::vector<int32_t> indices(static_cast<size_t>(nnz));
    std::vector<float> weight(static_cast<size_t>(nnz));
    if (nnz > 0)
        CHECK(ss_build_csr(s.h, s.w, s.pixel_m, s.dist_m, s.cy, s.cx, s.n_bins, s.split, mp, np, indptr.data(),
                           indices.data(), weight.data(), nnz - 1, &nnz, &max_row, &tth) == SS_ESIZE);
    int64_t nnz2 = -1;
    CHECK(ss_build_csr(s.h, s.w, s.pixel_m, s.dist_m, s.cy, s.cx, s.n_bins, s.split, mp, np, indptr.data(),
                       nnz ? indices.data() : reinterpret_cast<int32_t *>(indptr.data()), weight.data(), nnz, &nnz2,
                       &max_row, &tth) == SS_OK);
    CHECK(nnz2 == nnz);
    CHECK(indptr[0] == 0 && indptr[size_t(s.n_bins)] == nnz);
    int64_t longest = 0;
    std::vector<double> per_pixel(size_t(n), 0.0);
    std::vector<int32_t> entries(size_t(n), 0);
    for (int32_t r = 0; r < s.n_bins; ++r) {
        CHECK(indptr[size_t(r) + 1] >= indptr[size_t(r)]);
        longest = std::max<int64_t>(longest, indptr[size_t(r) + 1] - indptr[size_t(r)]);
        for (int64_t j = indptr[size_t(r)]; j < indptr[size_t(r) + 1]; ++j) {
            const int32_t i = indices[size_t(j)];
            CHECK(i >= 0 && i < n);
            if (i < 0 || i >= n) continue;
            if (j > indptr[size_t(r)]) CHECK(indices[size_t(j) - 1] < i);  // rows sorted, no repeats
            CHECK(!mask[size_t(i)] || !s.masked);
            CHECK(weight[size_t(j)] > 0.0f);
            per_pixel[size_t(i)] += double(weight[size_t(j)]) / double(norm[size_t(i)]);
            ++entries[size_t(i)];
        }
    }
    CHECK(longest == max_row);
    // every unmasked pixel's coefficients sum to one (one entry without splitting)
    for (int64_t i = 0; i < n; ++i) {
        if (s.masked && mask[size_t(i)]) {
            CHECK(entries[size_t(i)] == 0);
            continue;
        }
        CHECK(std::fabs(per_pixel[size_t(i)] - 1.0) < 1e-5);
        if (s.split == SS_SPLIT_NONE) CHECK(entries[size_t(i)] == 1);
    }

    // the same CSR in an 8 x 4 tiled layout: rows ascend in word offsets
    // inside the frame, and the per-pixel norm scattered to its words
    {
        const ss_layout lay{s.h, s.w, 8, 4};
        const int64_t words = ss_layout_words(&lay);
        CHECK(words >= n);
        std::vector<int32_t> ti(indices);
        std::vector<float> tw(weight);
        if (nnz > 0) CHECK(ss_csr_relayout(&lay, s.n_bins, indptr.data(), ti.data(), tw.data()) == SS_OK);
        for (int32_t r = 0; r < s.n_bins; ++r)
            for (int64_t j = indptr[size_t(r)]; j < indptr[size_t(r) + 1]; ++j) {
                CHECK(ti[size_t(j)] >= 0 && ti[size_t(j)] < words);
                if (j > indptr[size_t(r)]) CHECK(ti[size_t(j) - 1] < ti[size_t(j)]);
            }
        std::vector<float> dst(static_cast<size_t>(words));
        CHECK(ss_layout_scatter(&lay, norm.data(), -1.0f, dst.data()) == SS_OK);
        int64_t filled = 0;
        for (float v : dst) filled += v == -1.0f ? 1 : 0;
        CHECK(filled == words - n);
    }

    // radial codes
    std::vector<uint32_t> rc(static_cast<size_t>(n));
    double c0 = 0.0, width = 0.0;
    CHECK(ss_radial_coords(s.h, s.w, s.pixel_m, s.dist_m, s.cy, s.cx, s.n_bins, tth, mp, rc.data(), &c0, &width) ==
          SS_OK);
    CHECK(std::fabs(width * s.n_bins - tth) <= 1e-12 * tth && std::fabs(c0 - 0.5 * width) <= 1e-15 * tth);
    for (int64_t i = 0; i < n; ++i) {
        if (s.masked && mask[size_t(i)]) {
            CHECK(rc[size_t(i)] == SS_RC_MASKED);
            continue;
        }
        const uint32_t t1 = rc[size_t(i)] >> SS_RC_FRAC_BITS;  // interval + 1, 0 below the first centre
        CHECK(t1 <= uint32_t(s.n_bins));
    }

    // row schedule: a permutation of the bins, classes from the longest down
    std::vector<int32_t> order(size_t(s.n_bins), -1);
    int32_t counts[SS_N_CLASSES];
    CHECK(ss_csr_schedule(indptr.data(), s.n_bins, order.data(), counts) == SS_OK);
    std::vector<int32_t> seen(size_t(s.n_bins), 0);
    int32_t sum = 0;
    for (int c = 0; c < SS_N_CLASSES; ++c) sum += counts[c];
    CHECK(sum == s.n_bins);
    int prev_class = SS_N_CLASSES;
    for (int32_t k = 0; k < s.n_bins; ++k) {
        const int32_t r = order[size_t(k)];
        CHECK(r >= 0 && r < s.n_bins);
        if (r < 0 || r >= s.n_bins) continue;
        ++seen[size_t(r)];
        const int64_t len = indptr[size_t(r) + 1] - indptr[size_t(r)];
        int c = 0;
        while (c < SS_N_CLASSES - 1 && len > ss_class_rows(c)) ++c;
        CHECK(c <= prev_class);
        prev_class = c;
    }
    for (int32_t r = 0; r < s.n_bins; ++r) CHECK(seen[size_t(r)] == 1);
}

static void check_errors() {
    int64_t nnz;
    int32_t max_row;
    double tth;
    CHECK(ss_build_csr(8, 8, 75e-6, 0.1, 4, 4, 4, 7, nullptr, nullptr, nullptr, nullptr, nullptr, 0, &nnz, &max_row,
                       &tth) == SS_EINVAL);
    CHECK(ss_build_csr(0, 8, 75e-6, 0.1, 4, 4, 4, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0, &nnz, &max_row,
                       &tth) == SS_ESIZE);
    CHECK(ss_build_csr(8, 8, 75e-6, 0.1, 4, 4, SS_MAX_BINS + 1, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                       &nnz, &max_row, &tth) == SS_ESIZE);
    CHECK(ss_build_csr(8, 8, 75e-6, 0.1, NAN, 4, 4, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0, &nnz,
                       &max_row, &tth) == SS_EINVAL);
    CHECK(ss_build_csr(8, 8, -1.0, 0.1, 4, 4, 4, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0, &nnz, &max_row,
                       &tth) == SS_ESIZE);
    CHECK(ss_build_csr(8, 8, 75e-6, 0.1, 4, 4, 4, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr,
                       &max_row, &tth) == SS_EINVAL);
    CHECK(ss_build_csr(1 << 16, 1 << 15, 75e-6, 0.1, 4, 4, 4, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0, &nnz,
                       &max_row, &tth) == SS_ESIZE);
    uint32_t rc[4];
    double c0, w;
    CHECK(ss_radial_coords(2, 2, 75e-6, 0.1, 1, 1, 4, 0.0, nullptr, rc, &c0, &w) == SS_EINVAL);
    CHECK(ss_radial_coords(2, 2, 75e-6, 0.1, 1, 1, 0, 1.0, nullptr, rc, &c0, &w) == SS_ESIZE);
    CHECK(ss_radial_coords(2, 2, 75e-6, 0.1, 1, 1, 4, 1.0, nullptr, nullptr, &c0, &w) == SS_EINVAL);
    const int64_t bad_ptr[3] = {0, 5, 3};  // a row of negative length
    int32_t order[2], counts[SS_N_CLASSES];
    CHECK(ss_csr_schedule(bad_ptr, 2, order, counts) == SS_EINVAL);
    CHECK(ss_csr_schedule(bad_ptr, 0, order, counts) == SS_ESIZE);
    CHECK(ss_csr_schedule(nullptr, 2, order, counts) == SS_EINVAL);
    for (int c = -2; c <= SS_N_CLASSES + 1; ++c) {
        const int32_t rows = ss_class_rows(c);
        CHECK(rows >= 0);
        if (c >= 1 && c < SS_N_CLASSES - 1) CHECK(rows > ss_class_rows(c - 1));
    }
    const ss_layout bad_tiles{8, 8, 3, 4};
    CHECK(ss_layout_words(&bad_tiles) == SS_ESIZE);
    CHECK(ss_layout_words(nullptr) == SS_EINVAL);
    CHECK(ss_csr_relayout(nullptr, 2, bad_ptr, order, nullptr) == SS_EINVAL);
    float one = 1.0f;
    CHECK(ss_layout_scatter(&bad_tiles, &one, 0.0f, &one) == SS_ESIZE);
    for (int code = -5; code <= 1; ++code) CHECK(ss_strerror(code) != nullptr);
    CHECK(ss_version() > 0);
}

int main() {
    const Scene scenes[] = {
        {37, 53, 17, SS_SPLIT_BBOX, 75e-6, 0.1, 10.3, 40.7, true, true},
        {37, 53, 17, SS_SPLIT_NONE, 75e-6, 0.1, 10.3, 40.7, true, true},
        {1, 1, 1, SS_SPLIT_BBOX, 75e-6, 0.1, 0.5, 0.5, false, false},
        {5, 300, 64, SS_SPLIT_BBOX, 75e-6, 0.05, -40.0, 900.0, false, true},  // centre outside the detector
        {256, 256, 1000, SS_SPLIT_BBOX, 75e-6, 0.12, 131.2, 120.9, true, false},
        {64, 48, SS_MAX_BINS, SS_SPLIT_BBOX, 75e-6, 0.1, 30.0, 20.0, false, false},  // more bins than pixels per ring
    };
    for (const Scene &s : scenes) check_scene(s);
    check_errors();
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("geometry checks ok\n");
    return 0;
}
