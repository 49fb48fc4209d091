// Jungfrau pre-processing and normalisation (Sec. 1.2, eq. norm).
//
// One thread owns 4 consecutive pixels and walks all frames of the batch: the
// pedestals and gains of all three levels and the normalisation of its
// pixels are read once per batch into registers, while the raw words stream
// through with 8-byte loads, several frames in flight.  No word causes a
// gather, whatever its gain level.
//
// The arithmetic is float64 and each stored value is rounded once to
// float32: signal = f32((adc - ped) / gain), out = f32(signal / norm).
//
// Output frames are row-major or tiled (ss_layout).  Threads walk the
// output in word order, 4 words (one quad of pixels in one image row) each,
// so every store is 16 contiguous bytes of a fully written line; the raw
// words and calibration of the quad are read at its row-major pixels.

#include "common.h"

namespace ss {

bool make_layout(int32_t height, int32_t width, int32_t tile_w, int32_t tile_h, Layout &out) {
    const ss_layout l{height, width, tile_w, tile_h};
    const int64_t words = ss_layout_words(&l);
    if (words < 0) return false;
    out.height = height;
    out.width = width;
    out.words = words;
    out.sw = tile_w == 0 ? -1 : __builtin_ctz(uint32_t(tile_w));
    out.sh = tile_w == 0 ? -1 : __builtin_ctz(uint32_t(tile_h));
    out.tiles_x = tile_w == 0 ? 1 : (width + tile_w - 1) / tile_w;
    return true;
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t value) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = value;
}

namespace {

constexpr int kVec = 4;
#ifndef SS_CORRECT_BLOCK
#define SS_CORRECT_BLOCK 256
#endif
constexpr int kCorrectBlock = SS_CORRECT_BLOCK;

// float32(a / b) rounded to nearest, for a and b exact in float64, given
// r = float64(1 / b).  The product q = a * r lies within 2^-52 |a / b| (1 +
// 2^-52) of a / b: two units in q's last place.  Rounding to float32 keeps
// q's top 24 significant bits and decides on the 29 fraction bits below,
// whose only rounding boundary is the half-way pattern 2^28 (values just
// either side of a float32 itself round to it).  So when those 29 bits lie
// more than 8 from 2^28, a / b rounds as q does; otherwise (about one value
// in 3 * 10^7) the exact quotient is formed.
__device__ __noinline__ float div_exact32(double a, float b) { return float(a / double(b)); }

__device__ inline float div_round32(double a, float b, double r) {
    const double q = a * r;
    const uint32_t below = uint32_t(uint64_t(__double_as_longlong(q))) & 0x1FFFFFFFu;
    if (__builtin_expect(below - (0x10000000u - 8u) > 16u, 1)) return float(q);
    return div_exact32(a, b);
}

// Calibration of one pixel held in registers for the whole batch: the three
// pedestals and gains and the reciprocals of the gains and of the norm, so
// that every gain level takes the certified reciprocal product (the level
// of a word costs selects, not a divergent division).  Scalar fields keep
// it in registers.
struct PixelCal {
    float p0, p1, p2;
    float g0, g1, g2;
    double r0, r1, r2;  // 1 / gain of levels 0, 1, 2
    float norm;
    double rnorm;       // 1 / norm
};

__device__ inline PixelCal load_cal(const float *__restrict__ ped, const float *__restrict__ gain,
                                    const float *__restrict__ norm, int64_t i, int64_t n_pix) {
    PixelCal c;
    c.p0 = ped[i];
    c.p1 = ped[n_pix + i];
    c.p2 = ped[2 * n_pix + i];
    c.g0 = gain[i];
    c.g1 = gain[n_pix + i];
    c.g2 = gain[2 * n_pix + i];
    c.r0 = 1.0 / double(c.g0);
    c.r1 = 1.0 / double(c.g1);
    c.r2 = 1.0 / double(c.g2);
    c.norm = norm ? norm[i] : 1.0f;
    c.rnorm = 1.0 / double(c.norm);
    return c;
}

// Corrected intensity of one raw word: f32(f32((adc - ped) / gain) / norm).
// Gain codes 0, 1 and 3 select levels 0, 1 and 2; code 2 is invalid (NaN,
// counted).  Branch free apart from the rare exact division.
__device__ inline float correct_one(uint32_t word, const PixelCal c, bool has_norm, int &invalid) {
    const uint32_t code = (word >> 14) & 3u;
    const bool bad = code == 2u;
    const bool l0 = code == 0u, l1 = code == 1u;
    const double adc = double(word & 0x3FFFu);
    const float pg = l0 ? c.p0 : (l1 ? c.p1 : c.p2);
    const float gg = l0 ? c.g0 : (l1 ? c.g1 : c.g2);
    const double rg = l0 ? c.r0 : (l1 ? c.r1 : c.r2);
    const float s = div_round32(adc - double(pg), gg, rg);
    const float v = has_norm ? div_round32(double(s), c.norm, c.rnorm) : s;
    invalid += bad ? 1 : 0;
    return bad ? __builtin_nanf("") : v;
}

// Raw words of frame f: frame f of the batch, or, with a frame index, frame
// frame_index[f] of a ring of ring_frames frames.  An index outside the ring
// reads as invalid words (gain code 10: NaN, counted) instead of memory.
struct RawFrames {
    const uint16_t *raw;
    const int64_t *frame_index;  // [n_frames] or null
    int64_t ring_frames;
};

__device__ inline const uint16_t *frame_words(const RawFrames &r, int f, int64_t n_pix, bool &ok) {
    int64_t fi = f;
    if (r.frame_index) fi = r.frame_index[f];
    ok = uint64_t(fi) < uint64_t(r.ring_frames);
    return r.raw + (ok ? fi : 0) * n_pix;
}

constexpr uint32_t kInvalidPair = 0x80008000u;  // two words with gain code 10

// Raster index p of the first pixel of output quad i (words 4i .. 4i + 3,
// pixels p .. p + 3 of one image row), or false for a quad past the image
// edge.  Row-major: p = 4i.  Tiled (tile width >= 4): quads run through
// a tile row by row.
__device__ inline bool quad_site(int64_t i, const Layout &L, int64_t &p) {
    if (!L.tiled()) {
        p = i * 4;
        return p < L.words;
    }
    const int tq = L.sw + L.sh - 2;  // log2 of the quads of a tile
    const int64_t t = i >> tq;
    const int q = int(i & ((int64_t(1) << tq) - 1));
    const int64_t ty = t / L.tiles_x, tx = t - ty * L.tiles_x;
    const int64_t y = (ty << L.sh) + (q >> (L.sw - 2));
    const int64_t x = (tx << L.sw) + int64_t(q & ((1 << (L.sw - 2)) - 1)) * 4;
    p = y * L.width + x;
    return y < L.height && x < L.width;
}

// Raster index of the pixel at output word o, or false past the image edge.
__device__ inline bool word_site(int64_t o, const Layout &L, int64_t &p) {
    if (!L.tiled()) {
        p = o;
        return o < L.words;
    }
    const int64_t t = o >> (L.sw + L.sh);
    const int w = int(o & ((int64_t(1) << (L.sw + L.sh)) - 1));
    const int64_t ty = t / L.tiles_x, tx = t - ty * L.tiles_x;
    const int64_t y = (ty << L.sh) + (w >> L.sw), x = (tx << L.sw) + (w & ((1 << L.sw) - 1));
    p = y * L.width + x;
    return y < L.height && x < L.width;
}

#ifndef SS_CORRECT_UNROLL
#define SS_CORRECT_UNROLL 4
#endif
constexpr int kFrameUnroll = SS_CORRECT_UNROLL;

// Vector path: quads of pixels within image rows (row-major: n_pix % 4 ==
// 0; tiled: width % 4 == 0) and 16-byte aligned buffers.
__global__ __launch_bounds__(kCorrectBlock) void k_correct_vec(
    const RawFrames raw, int n_frames, const Layout L, const float *__restrict__ ped,
    const float *__restrict__ gain, const float *__restrict__ norm, float *__restrict__ out,
    int64_t *__restrict__ n_invalid) {
    const int64_t qi = int64_t(blockIdx.x) * kCorrectBlock + threadIdx.x;
    if (qi * kVec >= L.words) return;
    const int64_t n_pix = int64_t(L.height) * L.width;
    int64_t p0;
    if (!quad_site(qi, L, p0)) {
        const float nan = __builtin_nanf("");
        for (int f = 0; f < n_frames; ++f)
            *reinterpret_cast<float4 *>(out + int64_t(f) * L.words + qi * kVec) = make_float4(nan, nan, nan, nan);
        return;
    }
    PixelCal cal[kVec];
#pragma unroll
    for (int k = 0; k < kVec; ++k) cal[k] = load_cal(ped, gain, norm, p0 + k, n_pix);
    for (int f0 = 0; f0 < n_frames; f0 += kFrameUnroll) {
        uint2 w[kFrameUnroll];
#pragma unroll
        for (int u = 0; u < kFrameUnroll; ++u) {
            const int f = min(f0 + u, n_frames - 1);
            bool ok;
            const uint16_t *fr = frame_words(raw, f, n_pix, ok);
            w[u] = ok ? *reinterpret_cast<const uint2 *>(fr + p0) : make_uint2(kInvalidPair, kInvalidPair);
        }
#pragma unroll
        for (int u = 0; u < kFrameUnroll; ++u) {
            const int f = f0 + u;
            if (f >= n_frames) break;
            const uint32_t words[kVec] = {w[u].x & 0xFFFFu, w[u].x >> 16, w[u].y & 0xFFFFu, w[u].y >> 16};
            int invalid = 0;
            float o[kVec];
#pragma unroll
            for (int k = 0; k < kVec; ++k) o[k] = correct_one(words[k], cal[k], norm != nullptr, invalid);
            *reinterpret_cast<float4 *>(out + int64_t(f) * L.words + qi * kVec) = make_float4(o[0], o[1], o[2], o[3]);
            if (invalid && n_invalid)
                atomicAdd(reinterpret_cast<unsigned long long *>(n_invalid + f), (unsigned long long)invalid);
        }
    }
}

// Vector path for one or two frames (a single frame waits for it): the
// calibration of a word's own gain level only, gathered per word, instead
// of all three levels per pixel -- 8 bytes of pedestal and gain per word
// against 24 per pixel.  The same arithmetic as k_correct_vec.
constexpr int kFewFrames = 2;

__global__ __launch_bounds__(kCorrectBlock) void k_correct_few(
    const RawFrames raw, int n_frames, const Layout L, const float *__restrict__ ped,
    const float *__restrict__ gain, const float *__restrict__ norm, float *__restrict__ out,
    int64_t *__restrict__ n_invalid) {
    const int64_t qi = int64_t(blockIdx.x) * kCorrectBlock + threadIdx.x;
    if (qi * kVec >= L.words) return;
    const int64_t n_pix = int64_t(L.height) * L.width;
    int64_t p0;
    if (!quad_site(qi, L, p0)) {
        const float nan = __builtin_nanf("");
        for (int f = 0; f < n_frames; ++f)
            *reinterpret_cast<float4 *>(out + int64_t(f) * L.words + qi * kVec) = make_float4(nan, nan, nan, nan);
        return;
    }
    float nm[kVec];
    double rn[kVec];
#pragma unroll
    for (int k = 0; k < kVec; ++k) {
        nm[k] = norm ? norm[p0 + k] : 1.0f;
        rn[k] = 1.0 / double(nm[k]);
    }
    for (int f = 0; f < n_frames; ++f) {
        bool ok;
        const uint16_t *fr = frame_words(raw, f, n_pix, ok);
        const uint2 w = ok ? *reinterpret_cast<const uint2 *>(fr + p0) : make_uint2(kInvalidPair, kInvalidPair);
        const uint32_t words[kVec] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
        int invalid = 0;
        float o[kVec];
#pragma unroll
        for (int k = 0; k < kVec; ++k) {
            // gain codes 0, 1, 3 -> levels 0, 1, 2 (code 2, invalid, reads level 0)
            const uint32_t code = (words[k] >> 14) & 3u;
            const int64_t at = int64_t(code == 3u ? 2 : (code == 1u ? 1 : 0)) * n_pix + p0 + k;
            const float pg = ped[at], gg = gain[at];
            const double rg = 1.0 / double(gg);
            const PixelCal c{pg, pg, pg, gg, gg, gg, rg, rg, rg, nm[k], rn[k]};
            o[k] = correct_one(words[k], c, norm != nullptr, invalid);
        }
        *reinterpret_cast<float4 *>(out + int64_t(f) * L.words + qi * kVec) = make_float4(o[0], o[1], o[2], o[3]);
        if (invalid && n_invalid)
            atomicAdd(reinterpret_cast<unsigned long long *>(n_invalid + f), (unsigned long long)invalid);
    }
}

// Scalar path for any size and alignment: one thread per output word, all
// frames.
__global__ __launch_bounds__(kCorrectBlock) void k_correct_scalar(
    const RawFrames raw, int n_frames, const Layout L, const float *__restrict__ ped,
    const float *__restrict__ gain, const float *__restrict__ norm, float *__restrict__ out,
    int64_t *__restrict__ n_invalid) {
    const int64_t o = int64_t(blockIdx.x) * kCorrectBlock + threadIdx.x;
    if (o >= L.words) return;
    const int64_t n_pix = int64_t(L.height) * L.width;
    int64_t i;
    if (!word_site(o, L, i)) {
        for (int f = 0; f < n_frames; ++f) out[int64_t(f) * L.words + o] = __builtin_nanf("");
        return;
    }
    const PixelCal cal = load_cal(ped, gain, norm, i, n_pix);
    for (int f = 0; f < n_frames; ++f) {
        const int64_t at = int64_t(f) * L.words + o;
        int invalid = 0;
        bool ok;
        const uint16_t *fr = frame_words(raw, f, n_pix, ok);
        out[at] = correct_one(ok ? fr[i] : 0x8000u, cal, norm != nullptr, invalid);
        if (invalid && n_invalid) atomicAdd(reinterpret_cast<unsigned long long *>(n_invalid + f),
                                            (unsigned long long)invalid);
    }
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace
}  // namespace ss

namespace {

// Row-major frames of n_pix pixels (one row of n_pix for the indexing).
ss::Layout raster_layout(int64_t n_pix) {
    ss::Layout L{};
    L.height = 1;
    L.width = int32_t(n_pix);
    L.sw = L.sh = -1;
    L.tiles_x = 1;
    L.words = n_pix;
    return L;
}

int correct_entry(const ss::RawFrames &rf, int32_t n_frames, const ss::Layout &L, const float *pedestal,
                  const float *gain, const float *norm, float *out, int64_t *n_invalid, hipStream_t stream) {
    using namespace ss;
    if (n_frames == 0) return SS_OK;
    if (!rf.raw || !pedestal || !gain || !out) return SS_EINVAL;
    if (n_invalid) {
        k_fill_i64<<<1, 64, 0, stream>>>(n_invalid, n_frames, 0);
        SS_RETURN_IF_LAUNCH_FAILED();
    }
    const int64_t n_pix = int64_t(L.height) * L.width;
    if (n_pix == 0) return SS_OK;
    // quads stay inside image rows: row-major needs n_pix % 4 == 0, tiled
    // layouts width % 4 == 0 (their tiles are at least 4 wide)
    const bool quads = L.tiled() ? (L.width % kVec == 0) : (n_pix % kVec == 0);
    const bool vec = quads && aligned16(rf.raw) && aligned16(out);
    if (vec) {
        const int64_t threads = L.words / kVec;
        const int64_t blocks = (threads + kCorrectBlock - 1) / kCorrectBlock;
        if (n_frames <= kFewFrames)
            k_correct_few<<<dim3(uint32_t(blocks)), kCorrectBlock, 0, stream>>>(rf, n_frames, L, pedestal, gain,
                                                                                norm, out, n_invalid);
        else
            k_correct_vec<<<dim3(uint32_t(blocks)), kCorrectBlock, 0, stream>>>(rf, n_frames, L, pedestal, gain,
                                                                                norm, out, n_invalid);
    } else {
        const int64_t blocks = (L.words + kCorrectBlock - 1) / kCorrectBlock;
        k_correct_scalar<<<dim3(uint32_t(blocks)), kCorrectBlock, 0, stream>>>(rf, n_frames, L, pedestal, gain,
                                                                              norm, out, n_invalid);
    }
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}

int layout_arg(const ss_layout *layout, ss::Layout &L) {
    if (!layout) return SS_EINVAL;
    return ss::make_layout(layout->height, layout->width, layout->tile_w, layout->tile_h, L) ? SS_OK : SS_ESIZE;
}

}  // namespace

extern "C" int ss_correct(const uint16_t *raw, int32_t n_frames, int64_t n_pix, const float *pedestal,
                          const float *gain, const float *norm, float *out, int64_t *n_invalid,
                          hipStream_t stream) {
    if (n_frames < 0 || n_pix < 0 || n_pix >= (int64_t(1) << 31)) return SS_ESIZE;
    return correct_entry(ss::RawFrames{raw, nullptr, int64_t(n_frames)}, n_frames, raster_layout(n_pix), pedestal,
                         gain, norm, out, n_invalid, stream);
}

extern "C" int ss_correct_tiled(const uint16_t *raw, int32_t n_frames, const ss_layout *layout,
                                const float *pedestal, const float *gain, const float *norm, float *out,
                                int64_t *n_invalid, hipStream_t stream) {
    ss::Layout L;
    const int rc = layout_arg(layout, L);
    if (rc != SS_OK) return rc;
    if (n_frames < 0) return SS_ESIZE;
    return correct_entry(ss::RawFrames{raw, nullptr, int64_t(n_frames)}, n_frames, L, pedestal, gain, norm, out,
                         n_invalid, stream);
}

extern "C" int ss_correct_indexed(const uint16_t *ring, int64_t ring_frames, const int64_t *frame_index,
                                  int32_t n_frames, int64_t n_pix, const float *pedestal, const float *gain,
                                  const float *norm, float *out, int64_t *n_invalid, hipStream_t stream) {
    if (ring_frames < 0 || n_frames < 0 || n_pix < 0 || n_pix >= (int64_t(1) << 31)) return SS_ESIZE;
    if (n_frames > 0 && !frame_index) return SS_EINVAL;
    return correct_entry(ss::RawFrames{ring, frame_index, ring_frames}, n_frames, raster_layout(n_pix), pedestal,
                         gain, norm, out, n_invalid, stream);
}

extern "C" int ss_correct_indexed_tiled(const uint16_t *ring, int64_t ring_frames, const int64_t *frame_index,
                                        int32_t n_frames, const ss_layout *layout, const float *pedestal,
                                        const float *gain, const float *norm, float *out, int64_t *n_invalid,
                                        hipStream_t stream) {
    ss::Layout L;
    const int rc = layout_arg(layout, L);
    if (rc != SS_OK) return rc;
    if (ring_frames < 0 || n_frames < 0) return SS_ESIZE;
    if (n_frames > 0 && !frame_index) return SS_EINVAL;
    return correct_entry(ss::RawFrames{ring, frame_index, ring_frames}, n_frames, L, pedestal, gain, norm, out,
                         n_invalid, stream);
}
