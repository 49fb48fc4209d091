// Per-pixel classification against the clipped profile: sparsification
// (Sec. 3) and the peak finder (Sec. 4) in one pass over the pixels.
//
// k_profile_table (one work-group per frame) turns the per-bin profile into a
// lookup table over the n_bins + 1 intervals between bin centres: for each
// interval the bracketing non-empty bins and their mean/std, so that the
// background of a pixel is one table read plus a linear interpolation.  It
// also clears the output counts.
//
// k_pixel_state stages 2-D tiles of pixels (plus a halo of half a patch) in
// LDS and computes, once per pixel and frame, four bits: valid, kept
// (v - mu > n_pick sigma_eff), peak candidate (v - mu >= snr sigma_eff) and
// peak (the patch test of the peak finder, evaluated from LDS).
//
// Ordered output: the pixel pass also counts the kept pixels and peaks of
// every compaction tile (consecutive pixels of one frame, 256 threads x 32
// pixels; x 8 for one or two frames; integer sums, so the order of the
// additions does not matter), one work-group per frame turns the counts
// into exclusive offsets (k_tile_scan), and the tiles write their entries
// in pixel order at those offsets (k_tile_write), computing peak records on
// the way.
//
// The inverse direction (Sec. 3.2): k_densify rebuilds dense frames from the
// same background table -- noise free, or with noise drawn from a
// counter-based generator -- and k_densify_scatter puts the kept pixels
// back.  k_veto turns per-frame peak counts into the hit decision of Sec. 4
// and accumulates the counters a live veto threshold is chosen from.

#include <cmath>
#include <mutex>

#include "common.h"

namespace ss {
namespace {

constexpr int kBlock = 256;
// consecutive pixels per thread of the compaction: 32 for batches, 8 for one
// or two frames (four times the tiles, so that a single frame still fills
// the device); the workspace holds counts for the smaller tiles
constexpr int kPPT = 32;
constexpr int kPPTFew = 8;
constexpr int kFewFrames = 2;
constexpr int kNW = kBlock / kWave;
constexpr int kTableBlock = 256;

constexpr int kScanBlock = 1024;

struct Seg {
    double m_lo, dm, s_lo, ds, inv_span;
    int32_t lo, pad;
};

// The same interpolation in float32 for the fast path, as a line in the
// pixel's fraction of its interval: mu = a + b frac, sigma = c + d frac
// (a, b, c, d computed in float64 per interval and rounded once).
struct alignas(16) SegF {
    float a, b, c, d;
};

struct Workspace {
    SegF *tablef;       // [n_frames][n_bins + 1]
    SegF *tablet;       // [n_frames][n_bins + 1] threshold lines (noise 0), or null
    float *tolf;        // [n_frames] tolerance of the threshold lines, or null
    uint32_t *counts;   // per tile: kept | peaks << 16, [n_frames][tiles]
    uint64_t *offsets;  // per tile: kept offset | peak offset << 32, [n_frames][tiles]
    Seg *table;         // [n_frames][n_bins + 1]
    uint8_t *bits;      // pixel state [n_frames][n_pix]
};

constexpr uint8_t kValid = 1, kKeep = 2, kCand = 4, kPeak = 8;

size_t tiles_of(int64_t n_pix, int ppt = kPPTFew) {
    return size_t((n_pix + int64_t(kBlock) * ppt - 1) / (int64_t(kBlock) * ppt));
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

size_t workspace_bytes(int32_t n_frames, int64_t n_pix, int32_t n_bins) {
    const size_t tiles = size_t(n_frames) * tiles_of(n_pix);
    return 256 + 2 * align256(size_t(n_frames) * size_t(n_bins + 1) * sizeof(SegF)) +
           align256(size_t(n_frames) * sizeof(float)) + align256(tiles * sizeof(uint32_t)) +
           align256(tiles * sizeof(uint64_t)) + align256(size_t(n_frames) * size_t(n_bins + 1) * sizeof(Seg)) +
           align256(size_t(n_frames) * size_t(n_pix));
}

Workspace carve(void *base, int32_t n_frames, int64_t n_pix, int32_t n_bins) {
    const size_t tiles = size_t(n_frames) * tiles_of(n_pix);
    uintptr_t p = (reinterpret_cast<uintptr_t>(base) + 255) & ~uintptr_t(255);
    Workspace w;
    w.tablef = reinterpret_cast<SegF *>(p);
    p += align256(size_t(n_frames) * size_t(n_bins + 1) * sizeof(SegF));
    w.tablet = reinterpret_cast<SegF *>(p);
    p += align256(size_t(n_frames) * size_t(n_bins + 1) * sizeof(SegF));
    w.tolf = reinterpret_cast<float *>(p);
    p += align256(size_t(n_frames) * sizeof(float));
    w.counts = reinterpret_cast<uint32_t *>(p);
    p += align256(tiles * sizeof(uint32_t));
    w.offsets = reinterpret_cast<uint64_t *>(p);
    p += align256(tiles * sizeof(uint64_t));
    w.table = reinterpret_cast<Seg *>(p);
    p += align256(size_t(n_frames) * size_t(n_bins + 1) * sizeof(Seg));
    w.bits = reinterpret_cast<uint8_t *>(p);
    return w;
}

// ---- table ---------------------------------------------------------------

__global__ __launch_bounds__(kTableBlock) void k_profile_table(
    const double *__restrict__ mean, const double *__restrict__ stdv, const int32_t *__restrict__ members,
    int32_t n_bins, Workspace ws, int32_t tiles, int64_t *n_kept, int64_t *n_peaks, double n_pick, double snr) {
    __shared__ int32_t lo_s[SS_MAX_BINS + 1];
    __shared__ int32_t hi_s[SS_MAX_BINS + 1];
    __shared__ int32_t chunk_lo[kTableBlock];
    __shared__ int32_t chunk_hi[kTableBlock];
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    const int32_t *mem = members + int64_t(f) * n_bins;
    const double *mf = mean + int64_t(f) * n_bins;
    const double *sf = stdv + int64_t(f) * n_bins;

    // last non-empty bin <= r (prefix max) and first non-empty bin >= r
    // (suffix min), each thread scanning one contiguous chunk
    const int per = (n_bins + kTableBlock - 1) / kTableBlock;
    const int a0 = tid * per, a1 = min(n_bins, a0 + per);
    int run = -1;
    for (int r = a0; r < a1; ++r) {
        if (mem[r] > 0) run = r;
        lo_s[r] = run;
    }
    chunk_lo[tid] = run;
    run = n_bins;
    for (int r = a1 - 1; r >= a0; --r) {
        if (mem[r] > 0) run = r;
        hi_s[r] = run;
    }
    chunk_hi[tid] = run;
    // inclusive prefix max / suffix min over the chunks, log2(kTableBlock)
    // steps (a single frame waits for this table, so no serial scan)
    int in_lo = chunk_lo[tid], in_hi = chunk_hi[tid];
    for (int off = 1; off < kTableBlock; off <<= 1) {
        __syncthreads();
        const int plo = tid >= off ? chunk_lo[tid - off] : -1;
        const int phi = tid + off < kTableBlock ? chunk_hi[tid + off] : n_bins;
        __syncthreads();
        in_lo = max(in_lo, plo);
        in_hi = min(in_hi, phi);
        chunk_lo[tid] = in_lo;
        chunk_hi[tid] = in_hi;
    }
    __syncthreads();
    // exclusive: the chunks before (after) this one
    const int ex_lo = tid > 0 ? chunk_lo[tid - 1] : -1;
    const int ex_hi = tid + 1 < kTableBlock ? chunk_hi[tid + 1] : n_bins;
    for (int r = a0; r < a1; ++r) {
        if (lo_s[r] < 0) lo_s[r] = ex_lo;
        if (hi_s[r] >= n_bins) hi_s[r] = ex_hi;
    }
    __syncthreads();

    // interval t (stored at t + 1) lies between centres t and t + 1
    Seg *tab = ws.table + int64_t(f) * (n_bins + 1);
    double scale = 0.0;
    for (int t1 = tid; t1 <= n_bins; t1 += kTableBlock) {
        const int t = t1 - 1;
        const int lo = t >= 0 ? lo_s[t] : -1;
        const int hi = t + 1 < n_bins ? hi_s[t + 1] : n_bins;
        Seg s{0.0, 0.0, 0.0, 0.0, 0.0, 0, 0};
        if (lo >= 0 && hi < n_bins) {
            s.m_lo = mf[lo];
            s.dm = mf[hi] - mf[lo];
            s.s_lo = sf[lo];
            s.ds = sf[hi] - sf[lo];
            s.inv_span = 1.0 / double(hi - lo);
            s.lo = lo;
        } else if (lo >= 0 || hi < n_bins) {
            const int b = lo >= 0 ? lo : hi;
            s.m_lo = mf[b];
            s.s_lo = sf[b];
        }
        tab[t1] = s;
        // u = (t1 - 1 - lo + frac) inv_span, so mu = m_lo + dm u is a line in frac
        const double u0 = double(t1 - 1 - s.lo) * s.inv_span;
        const double ma = s.m_lo + s.dm * u0, mb = s.dm * s.inv_span;
        const double sa = s.s_lo + s.ds * u0, sb = s.ds * s.inv_span;
        ws.tablef[int64_t(f) * (n_bins + 1) + t1] = SegF{float(ma), float(mb), float(sa), float(sb)};
        if (ws.tablet) {
            // Without a noise level sigma_eff = sigma, which the interpolation
            // keeps non-negative, so both thresholds mu + n sigma are lines in
            // frac too: keep = v > ka + kb frac, candidate = v >= ca + cb frac
            const double ka = ma + n_pick * sa, kb = mb + n_pick * sb;
            const double ca = ma + snr * sa, cb = mb + snr * sb;
            ws.tablet[int64_t(f) * (n_bins + 1) + t1] = SegF{float(ka), float(kb), float(ca), float(cb)};
            scale = fmax(scale, fmax(fabs(ka) + fabs(kb), fabs(ca) + fabs(cb)));
        }
    }
    if (ws.tolf) {
        // A line evaluated in float32 from its rounded coefficients is within
        // 2^-23 (|a| + |b|) of the exact threshold (0 <= frac < 1, one fma),
        // so a value whose float32 compare could differ from the exact one
        // lies within that of the float32 threshold; pixels within 1e-6 of
        // the frame's largest |a| + |b| are decided again in float64.
        __shared__ double red[kTableBlock];
        red[tid] = scale;
        __syncthreads();
        for (int off = kTableBlock / 2; off > 0; off >>= 1) {
            if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
            __syncthreads();
        }
        if (tid == 0) ws.tolf[f] = float(1e-6 * red[0]) + 1e-30f;
    }
    if (tid == 0) {
        if (n_kept) n_kept[f] = 0;
        if (n_peaks) n_peaks[f] = 0;
    }
    // the pixel pass adds every compaction tile's kept pixels and peaks
    for (int t = tid; t < tiles; t += kTableBlock) ws.counts[int64_t(f) * tiles + t] = 0;
}

// ---- classification ----------------------------------------------------------

struct ClassArgs {
    const float *frames;  // [n_frames][lay.words], in layout lay
    Layout lay;
    int32_t n_frames;
    const uint8_t *mask;
    const uint32_t *rcoord;
    int64_t n_pix;
    int32_t height, width;
    int32_t n_bins;
    int32_t tiles;
    int32_t counted;  // the pixel pass has counted the tiles (else k_tile_counts)
    double n_pick, snr, noise2;
    int32_t half, min_count;
    uint32_t *kept_index;
    float *kept_value;
    int64_t capacity;
    int64_t *n_kept;
    ss_peak *peaks;
    int64_t peak_capacity;
    int64_t *n_peaks;
    Workspace ws;
};

// Word of raster pixel p in a frame of layout L (no division for row-major
// frames).
__device__ inline int64_t frame_word(const Layout &L, int64_t p) {
    if (!L.tiled()) return p;
    const uint32_t y = uint32_t(p) / uint32_t(L.width);
    return L.offset(int(y), int(uint32_t(p) - y * uint32_t(L.width)));
}

// Background (mu, sigma_eff) at fraction frac of centre interval t1.
__device__ inline void background_at(int t1, double frac, const Seg *__restrict__ tab, double noise2, double &mu,
                                     double &se) {
    const Seg s = tab[t1];
    const double u = (double(t1 - 1 - s.lo) + frac) * s.inv_span;
    mu = s.m_lo + s.dm * u;
    const double sd = s.s_lo + s.ds * u;
    se = sqrt(sd * sd + noise2);
}

__device__ inline void background(uint32_t rc, const Seg *__restrict__ tab, int n_bins, double noise2,
                                  double &mu, double &se) {
    const int t1 = min(int(rc >> SS_RC_FRAC_BITS), n_bins);
    const double frac = double(rc & ((1u << SS_RC_FRAC_BITS) - 1u)) * (1.0 / double(1u << SS_RC_FRAC_BITS));
    background_at(t1, frac, tab, noise2, mu, se);
}


// ---- per-pixel state and peak test ---------------------------------------------------

// State bits of an unmasked pixel of value x at fraction frac of centre
// interval t1, in float64.
__device__ inline uint8_t pixel_bits(float x, int t1, double frac, const Seg *__restrict__ tab, double noise2,
                                     double n_pick, double snr) {
    if (!isfinite(x)) return 0;
    double mu, se;
    background_at(t1, frac, tab, noise2, mu, se);
    const double d = double(x) - mu;
    return kValid | (d > n_pick * se ? kKeep : 0) | (d >= snr * se ? kCand : 0);
}

// Float32 version of pixel_bits.  Its rounding errors are below 1e-6 of the
// scale |v| + |a| + |b| + |c| + |d| + sigma (a + b frac and c + d frac are
// the interval's lines, |frac| < 1), so when v - mu is further than 1e-5 of
// that scale from both thresholds its decisions are those of the float64
// computation; otherwise it returns kUndecided and the pixel is decided
// again in float64 (pixel_bits).
constexpr uint8_t kUndecided = 0xFF;

// frac: the pixel's position in its interval, NaN for a masked pixel.
// Branch free: every slot's arithmetic runs, the result is selected.
__device__ inline uint8_t pixel_bits_fast(float x, float frac, const SegF &sg, float noise2f, float n_pick_f,
                                          float snr_f) {
    const bool valid = frac == frac && __builtin_isfinite(x);
    const float mu = fmaf(sg.b, frac, sg.a);
    const float sd = fmaf(sg.d, frac, sg.c);
    // the hardware square root (within 1 ulp) is far inside the tolerance
    const float se = noise2f == 0.0f ? fabsf(sd) : __builtin_amdgcn_sqrtf(fmaf(sd, sd, noise2f));
    const float d = x - mu;
    const float tk = n_pick_f * se, tc = snr_f * se;
    const float tol = 1e-5f * (fabsf(x) + fabsf(sg.a) + fabsf(sg.b) + fabsf(sg.c) + fabsf(sg.d) + se) + 1e-30f;
    const bool near = fabsf(d - tk) <= tol || fabsf(d - tc) <= tol;
    const uint32_t bits = kValid | (d > tk ? kKeep : 0u) | (d >= tc ? kCand : 0u);
    return uint8_t(valid ? (near ? uint32_t(kUndecided) : bits) : 0u);
}

// The same decisions from the threshold lines of a noise-free background:
// float32 compares against thresholds whose float32 evaluation lies within
// tol of the exact ones (see k_profile_table); a value within tol of either
// threshold is kUndecided.
__device__ inline uint8_t pixel_bits_lines(float x, float frac, const SegF &tl, float tol) {
    const bool valid = frac == frac && __builtin_isfinite(x);
    const float tk = fmaf(tl.b, frac, tl.a);
    const float tc = fmaf(tl.d, frac, tl.c);
    const bool near = fabsf(x - tk) <= tol || fabsf(x - tc) <= tol;
    const uint32_t bits = kValid | (x > tk ? kKeep : 0u) | (x >= tc ? kCand : 0u);
    return uint8_t(valid ? (near ? uint32_t(kUndecided) : bits) : 0u);
}

// pixel_bits_lines when n_pick == snr: the two lines are the same (same
// float64 expression), and a value further than tol from it is either above
// both thresholds or at most both, so one fma and one compare decide keep
// and candidate together.
__device__ inline uint8_t pixel_bits_line(float x, float frac, float ta, float tb, float tol) {
    const bool valid = frac == frac && __builtin_isfinite(x);
    const float t = fmaf(tb, frac, ta);
    const bool near = fabsf(x - t) <= tol;
    const uint32_t bits = x > t ? uint32_t(kValid | kKeep | kCand) : uint32_t(kValid);
    return uint8_t(valid ? (near ? uint32_t(kUndecided) : bits) : 0u);
}

// How k_pixel_state decides keep and candidate: from the background lines
// (with a noise level), from the two threshold lines, or from one line
// when n_pick == snr.
enum StateMode { kModeBackground = 0, kModeLines = 1, kModeLine = 2 };

// 2-D stencil tile (core pixels), work-group size and frames per
// work-group; compile-time tunables.
#ifndef SS_STENCIL_TILE_H
#define SS_STENCIL_TILE_H 16
#endif
#ifndef SS_STENCIL_TILE_W
#define SS_STENCIL_TILE_W 64
#endif
#ifndef SS_STENCIL_FRAMES
#define SS_STENCIL_FRAMES 16
#endif
constexpr int kTileH = SS_STENCIL_TILE_H;
constexpr int kTileW = SS_STENCIL_TILE_W;
#ifndef SS_STENCIL_BLOCK
#define SS_STENCIL_BLOCK 256
#endif
constexpr int kStencilBlock = SS_STENCIL_BLOCK;
constexpr int kFramesPerBlock = SS_STENCIL_FRAMES;
// staged pixels per thread for a halo of h pixels
constexpr int stage_slots(int h) { return ((kTileH + 2 * h) * (kTileW + 2 * h) + kStencilBlock - 1) / kStencilBlock; }
// staging slots of the kernel that runs half width h (patches 1, 3 and 5
// have their own, 7 and 9 share one, wider ones another)
constexpr int state_slots(int h) {
    return h <= 2 ? stage_slots(h) : h <= 4 ? stage_slots(4) : stage_slots(SS_MAX_PATCH / 2);
}
// LDS of k_pixel_state for a staged region of rn pixels: the region's radial
// codes during set-up, whose bytes then hold two buffers of per-wave
// candidate lists (a wave lists at most all of its staged slots), then two
// buffers of staged values and two of pixel-state bytes, each with room for
// every slot (padding slots store past the region, where nothing reads).
constexpr int kStateWaves = kStencilBlock / kWave;
constexpr size_t state_list_cap(int slots) { return size_t(slots) * kWave; }
constexpr size_t state_head_bytes(int rn, int slots) {
    const size_t rc = size_t(rn) * 4, lists = 2 * kStateWaves * state_list_cap(slots) * sizeof(uint16_t);
    return ((rc > lists ? rc : lists) + 15) & ~size_t(15);
}
// compaction tiles one work-group of the pixel pass can count in LDS: its
// kTileH rows of kTileW pixels span at most ((kTileH - 1) width + kTileW)
// / tile + 2 of them
constexpr int kTileCounters = 64;
constexpr size_t state_lds_bytes(int rn, int slots) {
    return state_head_bytes(rn, slots) + size_t(slots) * kStencilBlock * 10;
}

struct StateArgs {
    const float *frames;  // [n_frames][lay.words], in layout lay
    Layout lay;
    const uint32_t *rcoord;
    const uint8_t *mask;
    int32_t n_frames;
    int32_t height, width;
    int64_t n_pix;
    int32_t n_bins;
    int32_t half, min_count;
    double noise2, n_pick, snr;
    float noise2f, n_pick_f, snr_f;
    int32_t tiles_x, tiles_y, frame_groups;
    int32_t count_shift, count_tiles;  // compaction tiles: 2^count_shift pixels, count_tiles per frame
    int32_t counting;                  // the pass adds the tiles' counts (else k_tile_counts does)
    Workspace ws;
};

// One work-group owns a kTileH x kTileW tile of pixels for kFramesPerBlock
// frames.  The tile and its halo of `half` pixels are staged in LDS: radial
// codes once, then per frame the values and the pixel bits (valid, kept,
// candidate), computed once per staged pixel.  Candidates of the tile then
// take the patch test of Sec. 4 from LDS (maximum of v over the valid
// pixels of the patch, ties to the lower index; at least min_count
// candidates) and the bits, with kPeak, go to the workspace; the kept
// pixels and peaks of every compaction tile are counted on the way.
// Patch test of Sec. 4 from LDS for candidate e: v must be the maximum over
// the valid pixels of the patch (ties to the lower row-major index, i.e. a
// neighbour above, or on the same row to the left, wins a tie) with at least
// min_count candidates in the patch.  For a compile-time half width KH >= 0
// every neighbour is read before any is tested; KH < 0 walks a runtime half
// width h.
template <int KH>
__device__ inline bool patch_is_peak(const float *v_s, const uint8_t *b_s, int e, int RW, int h, int min_count) {
    const float vi = v_s[e];
    if (KH >= 0) {
        constexpr int P = 2 * (KH < 0 ? 0 : KH) + 1;
        uint8_t nb[P * P];
        float nv[P * P];
#pragma unroll
        for (int dy = 0; dy < P; ++dy)
#pragma unroll
            for (int dx = 0; dx < P; ++dx) {
                const int q = e + (dy - KH) * RW + (dx - KH);
                nb[dy * P + dx] = b_s[q];
                nv[dy * P + dx] = v_s[q];
            }
        // Branch free: a neighbour that comes before the centre wins a tie,
        // so it beats the centre when vq >= vi, any other when vq > vi (a
        // valid pixel's value is finite); bitwise operators keep the
        // compiler from turning the tests into short-circuit branches.
        bool best = true;
        int count = 0;
#pragma unroll
        for (int dy = 0; dy < P; ++dy)
#pragma unroll
            for (int dx = 0; dx < P; ++dx) {
                const uint32_t bq = nb[dy * P + dx];
                const float vq = nv[dy * P + dx];
                const bool centre = dy == KH && dx == KH;
                const bool before = dy < KH || (dy == KH && dx < KH);
                const bool valid = (bq & kValid) != 0;
                if (!centre) best = best & !(valid & (before ? vq >= vi : vq > vi));
                count += int((bq >> 2) & 1u);  // kCand (a candidate is valid)
            }
        return best & (count >= min_count);
    }
    bool best = true;
    int count = 0;
    for (int dy = -h; dy <= h && best; ++dy) {
        for (int dx = -h; dx <= h; ++dx) {
            const int q = e + dy * RW + dx;
            const uint8_t bq = b_s[q];
            if (!(bq & kValid)) continue;
            const float vq = v_s[q];
            const bool before = dy < 0 || (dy == 0 && dx < 0);
            if ((dy || dx) && (vq > vi || (vq == vi && before))) {
                best = false;
                break;
            }
            count += (bq & kCand) ? 1 : 0;
        }
    }
    return best && count >= min_count;
}

// Region pixel (row-major index in the RH x RW staged region whose top left
// pixel is (Y0, X0)) of staged slot s, the region's pixels taken tile by
// tile of a tiled frame layout (tiles of 2^sw x 2^sh, aligned to the
// frame): the 64 lanes of a wave then load whole tiles, two 128-byte lines
// for 8 x 4 tiles, instead of one region row that crosses nine.  Tiles cut
// the region into row groups of whole rows (the first and last may be
// partial) and each row group into blocks of whole columns; a row group is
// stored block after block, each block row-major.
// floor(n / d) for 0 <= n < 2^13 and 1 <= d <= 64: (n + 1/2) / d lies at
// least 1/(2d) >= 2^-7 from an integer, and the float32 product with the
// hardware reciprocal (within 1 ulp) is within 2^13 * 2^-22 = 2^-9 of it.
__device__ inline int small_div(int n, int d) {
    return int((float(n) + 0.5f) * __builtin_amdgcn_rcpf(float(d)));
}

// (Row groups and blocks are at most 64 pixels on a side, the region at
// most 78 wide, so the positions divided below stay under 2^13.)
__device__ inline int tile_order_slot(int s, int RW, int RH, int Y0, int X0, int sw, int sh, uint32_t magic) {
    const int oy = Y0 & ((1 << sh) - 1), ox = X0 & ((1 << sw) - 1);
    const int r = int((uint32_t(s) * magic) >> 20);       // region row of s in row-major order
    const int gi = (r + oy) >> sh;                          // its row group (groups hold whole rows)
    const int r0 = max(0, (gi << sh) - oy), r1 = min(RH, ((gi + 1) << sh) - oy);
    const int gh = r1 - r0;
    const int w = s - r0 * RW;                              // position in the row group
    const int gj = (small_div(w, gh) + ox) >> sw;           // block of the row group
    const int c0 = max(0, (gj << sw) - ox), c1 = min(RW, ((gj + 1) << sw) - ox);
    const int u = w - c0 * gh;
    const int gw = c1 - c0;
    const int q = small_div(u, gw);
    return (r0 + q) * RW + c0 + (u - q * gw);
}

template <int kStageSlots, int kH, int MODE, bool TILED>
__global__ __launch_bounds__(kStencilBlock) __attribute__((amdgpu_waves_per_eu(kH == 0 || kH == 1 ? 8 : kStageSlots <= 7 ? 5 : 4)))
void k_pixel_state(StateArgs a) {
    extern __shared__ unsigned char lds[];
    // region sizes are compile-time for the unrolled patches, so that the
    // LDS buffers of a frame sit at constant offsets
    const int h = kH >= 0 ? kH : a.half;
    const int RW = kTileW + 2 * h, RH = kTileH + 2 * h, RN = RW * RH;
    constexpr int SN = kStageSlots * kStencilBlock;  // buffer length: every slot
    const size_t head = state_head_bytes(RN, kStageSlots);
    uint32_t *rc_s = reinterpret_cast<uint32_t *>(lds);    // set-up only
    uint16_t *lists = reinterpret_cast<uint16_t *>(lds);   // same bytes, afterwards
    float *v_base = reinterpret_cast<float *>(lds + head);
    uint8_t *b_base = lds + head + size_t(SN) * 8;
    constexpr int kCap = int(state_list_cap(kStageSlots));
    __shared__ uint32_t cnt_s[2][kStateWaves];
    // kept pixels | peaks << 16 per compaction tile, from the work-group's
    // first tile on, by frame parity (the host counts in a kernel of its own
    // when a tile's rows span more compaction tiles)
    __shared__ uint32_t tc_s[2][kTileCounters];

    // Work-groups go to the 8 XCDs round robin; work-group g takes item
    // (g % 8) * per + g / 8 of the row-major list (frame group, tile row,
    // tile column), so each XCD walks a contiguous run of tiles and the
    // halo cache lines that neighbouring tiles share are fetched into one L2.
    int tx0, ty0, f0;
    {
        const uint32_t total = uint32_t(a.tiles_x) * uint32_t(a.tiles_y) * uint32_t(a.frame_groups);
        const uint32_t per = (total + 7u) / 8u;
        const uint32_t g = blockIdx.x;
        const uint32_t item = (g % 8u) * per + g / 8u;
        if (g / 8u >= per || item >= total) return;
        const uint32_t row = item / uint32_t(a.tiles_x);
        tx0 = int(item - row * uint32_t(a.tiles_x)) * kTileW;
        ty0 = int(row % uint32_t(a.tiles_y)) * kTileH;
        f0 = int(row / uint32_t(a.tiles_y)) * kFramesPerBlock;
    }
    const int f1 = min(a.n_frames, f0 + kFramesPerBlock);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid) / kWave;
    constexpr int kCore = kTileH * kTileW / kStencilBlock;
    // e / RW as (e * magic) >> 20, exact for e < 2^20 / RW (RN is far smaller)
    const uint32_t magic = ((1u << 20) + uint32_t(RW) - 1u) / uint32_t(RW);
    const int first_tile = int((int64_t(ty0) * a.width + tx0) >> a.count_shift);
    if (tid < 2 * kTileCounters) tc_s[tid / kTileCounters][tid % kTileCounters] = 0;

    for (int e = tid; e < RN; e += kStencilBlock) {
        const int r = int((uint32_t(e) * magic) >> 20);
        const int y = ty0 - h + r, x = tx0 - h + (e - r * RW);
        uint32_t rc = SS_RC_MASKED;
        if (y >= 0 && y < a.height && x >= 0 && x < a.width) {
            const int64_t i = int64_t(y) * a.width + x;
            rc = a.rcoord[i];
            if (a.mask && a.mask[i]) rc = SS_RC_MASKED;
        }
        rc_s[e] = rc;
    }
    __syncthreads();
    // Per staged slot, fixed over the frames: the pixel's byte offset in a
    // frame (beyond the frame for masked, out-of-frame and padding slots,
    // whose loads then read 0), its interval's byte offset in a frame's
    // float32 table, and its fraction of the interval (NaN when masked).
    // Frames hold fewer than 2^29 words, so byte offsets fit 32 bits.
    // With a tiled frame layout, slot k of a thread is region pixel e_k
    // (tile by tile), kept in the high half of toff[k] (table offsets are
    // below 2^16 bytes, region indices too); otherwise region pixel
    // tid + k * kStencilBlock.  Table offsets are multiples of 16: bit 2
    // (kCand) of toff[k] marks the tile's own (core) pixels, not halo, so
    // that bv & toff is kCand exactly for the core candidates.
    static_assert(sizeof(SegF) == 16 && kCand == 4, "a flag bit below the table offsets");
    const uint32_t frame_bytes = uint32_t(a.lay.words) * 4u;
    uint32_t voff[kStageSlots], toff[kStageSlots];
    float frac[kStageSlots];
#pragma unroll
    for (int k = 0; k < kStageSlots; ++k) {
        const int sk = tid + k * kStencilBlock;
        int e = sk;
        if constexpr (TILED)
            e = sk < RN ? tile_order_slot(sk, RW, RH, ty0 - h, tx0 - h, a.lay.sw, a.lay.sh, magic) : RN;
        const int ec = min(e, RN - 1);
        const int r = int((uint32_t(ec) * magic) >> 20), c = ec - r * RW;
        const int y = min(max(ty0 - h + r, 0), a.height - 1);
        const int x = min(max(tx0 - h + c, 0), a.width - 1);
        const uint32_t rc = e < RN ? rc_s[e] : SS_RC_MASKED;
        voff[k] = rc == SS_RC_MASKED ? frame_bytes : uint32_t(a.lay.offset(y, x)) * 4u;
        toff[k] = uint32_t(min(int(rc >> SS_RC_FRAC_BITS), a.n_bins)) * uint32_t(sizeof(SegF));
        if constexpr (TILED) toff[k] |= uint32_t(e) << 16;
        frac[k] = rc == SS_RC_MASKED ? __builtin_nanf("")
                                     : float(rc & ((1u << SS_RC_FRAC_BITS) - 1u)) * (1.0f / float(1u << SS_RC_FRAC_BITS));
        const bool core = e < RN && r >= h && r < h + kTileH && c >= h && c < h + kTileW;
        if (core) toff[k] |= kCand;
    }
    // The tile's core pixels this thread stores: pixel j is core pixel
    // tid + j * kStencilBlock, kCoreRows rows below pixel j - 1 in the same
    // column, so its LDS index and its offset in a frame follow from those
    // of pixel 0 (its row is the same for the whole wave).
    static_assert(kTileH * kTileW % kStencilBlock == 0 && kStencilBlock % kTileW == 0, "whole core rows per slot");
    constexpr int kCoreRows = kStencilBlock / kTileW;
    __syncthreads();  // the radial codes are dead; their bytes hold the lists
    // Only the last slot can lie wholly past the region for a wave (every
    // earlier slot index is below RN); such a wave skips it (its loads would
    // read 0, its pixels are masked).
    const bool last_live = wave * kWave + (kStageSlots - 1) * kStencilBlock < RN;
#define SS_SLOT_LIVE(k) ((k) < kStageSlots - 1 || last_live)

    const uint32_t table_bytes = uint32_t(a.n_bins + 1) * uint32_t(sizeof(SegF));
    float xv[kStageSlots];
    if (f0 < f1) {
        const __amdgpu_buffer_rsrc_t rf = buffer_rsrc(a.frames + int64_t(f0) * a.lay.words, frame_bytes);
#pragma unroll
        for (int k = 0; k < kStageSlots; ++k) xv[k] = SS_SLOT_LIVE(k) ? buffer_load_f32(rf, voff[k], 0u) : 0.0f;
    }
    // Frame f's values are loaded while frame f - 1 is classified (one frame
    // ahead) and the LDS buffers alternate by frame, so one barrier per frame
    // separates staging from the patch tests: buffer P is staged again two
    // frames later, after a barrier that every wave reaches only once it is
    // done with the frame before.  Each wave lists the candidates among its
    // staged core pixels before the barrier; after it, the work-group's
    // candidates take the patch test 64 per wave (batches rotated over the
    // waves by frame, so one wave tests a tile's usual few dozen), each
    // tester stores its candidate's state byte, and the owners of the other
    // core pixels store theirs: every byte is written once.  Owners count
    // kept pixels and testers peaks into LDS counters of the frame's
    // parity, which go to memory after the next frame's barrier.
    for (int f = f0; f < f1; ++f) {
        const int P = (f - f0) & 1;
        float *v_s = v_base + P * SN;
        uint8_t *b_s = b_base + P * SN;
        // redefined per frame, so the slot words below are masked and
        // shifted here, not held masked and shifted across frames
        uint32_t tmask = 0xFFF0u, hi = 16u;
        asm volatile("" : "+s"(tmask), "+s"(hi));
        uint8_t bv[kStageSlots];
        {
            const SegF *tbl = MODE == kModeBackground ? a.ws.tablef : a.ws.tablet;
            const __amdgpu_buffer_rsrc_t rt = buffer_rsrc(tbl + int64_t(f) * (a.n_bins + 1), table_bytes);
            SegF sg[kStageSlots];
#pragma unroll
            for (int k = 0; k < kStageSlots; ++k) {
                // (element access on the builtin's vector result is not used:
                // copying the whole vector out keeps the load intact); one
                // line is the entry's first 8 bytes
                sg[k] = SegF{0.0f, 0.0f, 0.0f, 0.0f};
                if (!SS_SLOT_LIVE(k)) continue;
                const uint32_t to = toff[k] & tmask;
                if constexpr (MODE == kModeLine) {
                    const auto q = __builtin_amdgcn_raw_buffer_load_b64(rt, int(to), 0, 0);
                    __builtin_memcpy(&sg[k], &q, 8);
                } else {
                    const auto q = __builtin_amdgcn_raw_buffer_load_b128(rt, int(to), 0, 0);
                    __builtin_memcpy(&sg[k], &q, sizeof(SegF));
                }
            }
            if constexpr (MODE == kModeLine) {
                const float tol = a.ws.tolf[f];
#pragma unroll
                for (int k = 0; k < kStageSlots; ++k)
                    bv[k] = SS_SLOT_LIVE(k) ? pixel_bits_line(xv[k], frac[k], sg[k].a, sg[k].b, tol) : 0;
            } else if constexpr (MODE == kModeLines) {
                const float tol = a.ws.tolf[f];
#pragma unroll
                for (int k = 0; k < kStageSlots; ++k)
                    bv[k] = SS_SLOT_LIVE(k) ? pixel_bits_lines(xv[k], frac[k], sg[k], tol) : 0;
            } else {
#pragma unroll
                for (int k = 0; k < kStageSlots; ++k)
                    bv[k] = SS_SLOT_LIVE(k) ? pixel_bits_fast(xv[k], frac[k], sg[k], a.noise2f, a.n_pick_f, a.snr_f) : 0;
            }
        }
        // pixels within rounding of a threshold, in float64 (rare; the
        // float32 table entries are no longer live here; the fraction is
        // exact in float32, the interval is the table offset's)
        bool undecided = false;
#pragma unroll
        for (int k = 0; k < kStageSlots; ++k) undecided = undecided || bv[k] == kUndecided;
        if (__builtin_amdgcn_ballot_w64(undecided) != 0) {
            const Seg *__restrict__ tab = a.ws.table + int64_t(f) * (a.n_bins + 1);
#pragma unroll
            for (int k = 0; k < kStageSlots; ++k)
                if (bv[k] == kUndecided)
                    bv[k] = pixel_bits(xv[k], int((toff[k] & 0xFFF0u) / uint32_t(sizeof(SegF))), double(frac[k]),
                                       tab, a.noise2, a.n_pick, a.snr);
        }
        uint16_t *own = lists + (P * kStateWaves + wave) * kCap;
        uint32_t n = 0;
#pragma unroll
        for (int k = 0; k < kStageSlots; ++k) {
            if (!SS_SLOT_LIVE(k)) continue;
            const int e = TILED ? int(toff[k] >> hi) : tid + k * kStencilBlock;
            v_s[e] = xv[k];
            b_s[e] = bv[k];
            const bool cand = (uint32_t(bv[k]) & toff[k]) != 0;
            const uint64_t m = __builtin_amdgcn_ballot_w64(cand);
            if (cand)
                own[__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), n))] =
                    uint16_t(e);
            n += uint32_t(__popcll(m));
        }
        if (lane == 0) cnt_s[P][wave] = uint32_t(n);
        if (f + 1 < f1) {
            const __amdgpu_buffer_rsrc_t rf = buffer_rsrc(a.frames + int64_t(f + 1) * a.lay.words, frame_bytes);
#pragma unroll
            for (int k = 0; k < kStageSlots; ++k)
                if (SS_SLOT_LIVE(k)) xv[k] = buffer_load_f32(rf, voff[k], 0u);
        }
        __syncthreads();
        // the previous frame's tile counts are complete (added before this
        // barrier): add them to the frame's, and clear them for frame f + 1
        if (a.counting && f > f0 && tid < kTileCounters) {
            const uint32_t v = tc_s[P ^ 1][tid];
            int t0 = first_tile;
            asm volatile("" : "+s"(t0));  // the address formed here, not held across frames
            if (v) atomicAdd(&a.ws.counts[int64_t(f - 1) * a.count_tiles + t0 + tid], v);
            tc_s[P ^ 1][tid] = 0;
        }
        auto count = [&](uint32_t p, uint32_t v) {
            if (a.counting) atomicAdd(&tc_s[P][int(p >> a.count_shift) - first_tile], v);
        };
        const __amdgpu_buffer_rsrc_t rb = buffer_rsrc(a.ws.bits + int64_t(f) * a.n_pix, uint32_t(a.n_pix));
        // (formed here from the thread index: the width redefined per frame
        // keeps them out of registers held across frames)
        uint32_t width = uint32_t(a.width);
        asm volatile("" : "+s"(width));
        const int core_y0 = ty0 + tid / kTileW, core_x = tx0 + tid % kTileW;
        const uint32_t soff0 = uint32_t(core_y0) * width + uint32_t(core_x);
        const int cidx0 = (tid / kTileW + h) * RW + (tid % kTileW + h);
#pragma unroll
        for (int j = 0; j < kCore; ++j) {
            const uint8_t b = b_s[cidx0 + j * kCoreRows * RW];
            if (core_y0 + j * kCoreRows < a.height && uint32_t(core_x) < width) {
                const uint32_t off = soff0 + uint32_t(j * kCoreRows) * width;
                if ((b & kCand) == 0) __builtin_amdgcn_raw_buffer_store_b8(b, rb, int(off), 0, 0);
                if (b & kKeep) count(off, 1u);
            }
        }
        // candidate i of the work-group is entry i - p_w of wave w's list,
        // p_w the candidates of the waves before w: list slot
        // i + sum over w' < w of (kCap - c_w')
        static_assert((kStateWaves & (kStateWaves - 1)) == 0, "waves per work-group a power of two");
        int cw[kStateWaves], total = 0;
#pragma unroll
        for (int w = 0; w < kStateWaves; ++w) {
            cw[w] = __builtin_amdgcn_readfirstlane(int(cnt_s[P][w]));
            total += cw[w];
        }
        const uint16_t *lists_p = lists + P * kStateWaves * kCap;
        for (int b = (wave - (f - f0)) & (kStateWaves - 1); b * kWave < total; b += kStateWaves) {
            const int i = b * kWave + lane;
            if (i < total) {
                int slot = i, before = 0;
#pragma unroll
                for (int w = 0; w + 1 < kStateWaves; ++w) {
                    before += cw[w];
                    slot += i >= before ? kCap - cw[w] : 0;
                }
                const int e = lists_p[slot];
                const bool peak = patch_is_peak<kH>(v_s, b_s, e, RW, h, a.min_count);
                const int r = int((uint32_t(e) * magic) >> 20);
                const uint32_t y = uint32_t(ty0 - h + r), x = uint32_t(tx0 - h + (e - r * RW));
                const uint32_t p = y * uint32_t(a.width) + x;
                __builtin_amdgcn_raw_buffer_store_b8(uint8_t(b_s[e] | (peak ? kPeak : 0)), rb, int(p), 0, 0);
                if (peak) count(p, 1u << 16);
            }
        }
    }
    // the last frame's tile counts
    __syncthreads();
    if (a.counting && f0 < f1 && tid < kTileCounters) {
        const uint32_t v = tc_s[(f1 - 1 - f0) & 1][tid];
        if (v) atomicAdd(&a.ws.counts[int64_t(f1 - 1) * a.count_tiles + first_tile + tid], v);
    }
#undef SS_SLOT_LIVE
}

// ---- peak test and record ------------------------------------------------------------

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ inline uint32_t wave_inclusive_scan(uint32_t x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(x, off, kWave);
        if (lane >= off) x += t;
    }
    return x;
}

// Kept / peak bits of the PPT consecutive pixels of thread tid in a tile:
// 8-byte loads when every frame's bits start 8-byte aligned (n_pix % 8 ==
// 0), byte loads otherwise.
template <bool KEEP, bool PEAKS, int PPT>
__device__ inline void tile_masks(const uint8_t *__restrict__ bits, int64_t n_pix, int64_t p0, uint32_t &kmask,
                                  uint32_t &pmask) {
    static_assert(PPT % 8 == 0 && PPT <= 32, "whole 8-byte words, one 32-bit mask");
    kmask = 0;
    pmask = 0;
    if (p0 + PPT <= n_pix && (n_pix % 8) == 0) {
#pragma unroll
        for (int q = 0; q < PPT / 8; ++q) {
            const uint2 w = *reinterpret_cast<const uint2 *>(bits + p0 + 8 * q);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint8_t b = uint8_t((k < 4 ? w.x : w.y) >> (8 * (k % 4)));
                if (KEEP && (b & kKeep)) kmask |= 1u << (8 * q + k);
                if (PEAKS && (b & kPeak)) pmask |= 1u << (8 * q + k);
            }
        }
    } else {
        for (int k = 0; k < PPT; ++k) {
            const uint8_t b = p0 + k < n_pix ? bits[p0 + k] : 0;
            if (KEEP && (b & kKeep)) kmask |= 1u << k;
            if (PEAKS && (b & kPeak)) pmask |= 1u << k;
        }
    }
}

// Exclusive block-wide scan of one packed u32 per thread; returns this
// thread's exclusive prefix, and the block total through `total`.
__device__ inline uint32_t block_exclusive_scan(uint32_t mine, uint32_t *wave_tot, uint32_t &total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const uint32_t incl = wave_inclusive_scan(mine);
    if (lane == kWave - 1) wave_tot[wid] = incl;
    __syncthreads();
    uint32_t before = incl - mine;
    total = 0;
#pragma unroll
    for (int w = 0; w < kNW; ++w) {
        if (w < wid) before += wave_tot[w];
        total += wave_tot[w];
    }
    return before;
}

// Per tile: packed count of kept pixels and peaks (each at most kBlock * PPT),
// for frames too wide for the pixel pass to count them.
template <bool KEEP, bool PEAKS, int PPT>
__global__ __launch_bounds__(kBlock) void k_tile_counts(ClassArgs a) {
    __shared__ uint32_t wave_tot[kNW];
    const int tile = blockIdx.x, f = blockIdx.y;
    const int64_t p0 = (int64_t(tile) * kBlock + threadIdx.x) * PPT;
    uint32_t kmask, pmask;
    tile_masks<KEEP, PEAKS, PPT>(a.ws.bits + int64_t(f) * a.n_pix, a.n_pix, p0, kmask, pmask);
    const uint32_t mine = uint32_t(__popc(kmask)) | (uint32_t(__popc(pmask)) << 16);
    const uint32_t x = uint32_t(wave_sum(int(mine)));
    if ((threadIdx.x & (kWave - 1)) == 0) wave_tot[threadIdx.x / kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kNW; ++w) t += wave_tot[w];
        a.ws.counts[int64_t(f) * a.tiles + tile] = t;
    }
}

// Per frame: exclusive offsets of every tile, and the frame totals.
template <bool KEEP, bool PEAKS>
__global__ __launch_bounds__(kScanBlock) void k_tile_scan(ClassArgs a) {
    __shared__ uint64_t part[kScanBlock / kWave];
    __shared__ uint64_t carry_s;
    const int f = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const uint32_t *cnt = a.ws.counts + int64_t(f) * a.tiles;
    uint64_t *off = a.ws.offsets + int64_t(f) * a.tiles;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < a.tiles; base += kScanBlock) {
        const int t = base + int(threadIdx.x);
        const uint32_t c = t < a.tiles ? cnt[t] : 0u;
        // widen to kept | peaks << 32 so sums over a frame cannot overflow
        uint64_t x = uint64_t(c & 0xFFFFu) | (uint64_t(c >> 16) << 32);
        uint64_t incl = x;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t lo = __shfl_up(uint32_t(incl), o, kWave);
            const uint32_t hi = __shfl_up(uint32_t(incl >> 32), o, kWave);
            if (lane >= o) incl += (uint64_t(hi) << 32) | lo;
        }
        if (lane == kWave - 1) part[wid] = incl;
        __syncthreads();
        uint64_t before = carry_s + incl - x, total = 0;
        for (int w = 0; w < kScanBlock / kWave; ++w) {
            if (w < wid) before += part[w];
            total += part[w];
        }
        if (t < a.tiles) off[t] = before;
        __syncthreads();
        if (threadIdx.x == 0) carry_s += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (KEEP) a.n_kept[f] = int64_t(carry_s & 0xFFFFFFFFu);
        if (PEAKS) a.n_peaks[f] = int64_t(carry_s >> 32);
    }
}

// Per tile: kept pixels and peak records in pixel order at the tile's
// offsets; entries beyond the capacities are dropped.
template <bool KEEP, bool PEAKS, int PPT>
__global__ __launch_bounds__(kBlock) void k_tile_write(ClassArgs a) {
    __shared__ uint32_t wave_tot[kNW];
    const int tile = blockIdx.x, f = blockIdx.y;
    const int64_t p0 = (int64_t(tile) * kBlock + threadIdx.x) * PPT;
    const float *__restrict__ fr = a.frames + int64_t(f) * a.lay.words;
    const uint8_t *__restrict__ bits = a.ws.bits + int64_t(f) * a.n_pix;
    // the tile's offsets do not depend on the scan below: load them first
    const uint64_t toff = a.ws.offsets[int64_t(f) * a.tiles + tile];
    uint32_t kmask, pmask;
    tile_masks<KEEP, PEAKS, PPT>(bits, a.n_pix, p0, kmask, pmask);
    const uint32_t mine = uint32_t(__popc(kmask)) | (uint32_t(__popc(pmask)) << 16);
    uint32_t total;
    const uint32_t before = block_exclusive_scan(mine, wave_tot, total);
    if (total == 0) return;
    int64_t pos_k = int64_t(toff & 0xFFFFFFFFu) + (before & 0xFFFFu);
    int64_t pos_p = int64_t(toff >> 32) + (before >> 16);
    if (KEEP) {
        // kept pixels four at a time: their values are loaded together, then stored
        constexpr int kBatch = 4;
        uint32_t m = kmask;
        while (m) {
            int ks[kBatch];
            float vs[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                ks[u] = m ? __builtin_ctz(m) : -1;
                m &= m ? m - 1 : 0u;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) vs[u] = ks[u] >= 0 ? fr[frame_word(a.lay, p0 + ks[u])] : 0.0f;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (ks[u] < 0) break;
                if (pos_k < a.capacity) {
                    a.kept_index[int64_t(f) * a.capacity + pos_k] = uint32_t(p0 + ks[u]);
                    a.kept_value[int64_t(f) * a.capacity + pos_k] = vs[u];
                }
                ++pos_k;
            }
        }
    }
    if (PEAKS) {
        // The wave's peaks one at a time, every lane taking one pixel of the
        // patch (patches of more than 64 pixels in rounds): a record costs
        // two rounds of dependent loads instead of three per neighbour, and
        // the lanes without peaks no longer wait for the one that has them.
        // The sums over the patch are the wave's reductions, in a fixed order.
        const Seg *__restrict__ tab = a.ws.table + int64_t(f) * (a.n_bins + 1);
        const int lane = threadIdx.x & (kWave - 1);
        const int P = 2 * a.half + 1;
        uint64_t owners = __builtin_amdgcn_ballot_w64(pmask != 0);
        while (owners) {
            const int src = __builtin_ctzll(owners);
            owners &= owners - 1;
            uint32_t m = uint32_t(__builtin_amdgcn_readlane(int(pmask), src));
            int64_t pos = (int64_t(__builtin_amdgcn_readlane(int(uint64_t(pos_p) >> 32), src)) << 32) |
                          int64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(pos_p)), src)));
            const int64_t p_src = (int64_t(tile) * kBlock + (threadIdx.x - lane) + src) * PPT;
            while (m) {
                const int k = __builtin_ctz(m);
                m &= m - 1;
                if (pos < a.peak_capacity) {
                    const int64_t i = p_src + k;
                    const int y = int(i / a.width), x = int(i - int64_t(i / a.width) * a.width);
                    double sums[4] = {0.0, 0.0, 0.0, 0.0};  // I, s2, sy, sx
                    for (int base = 0; base < P * P; base += kWave) {
                        const int q = base + lane;
                        const int yy = y + q / P - a.half, xx = x + q % P - a.half;
                        if (q < P * P && yy >= 0 && yy < a.height && xx >= 0 && xx < a.width) {
                            const int64_t j = int64_t(yy) * a.width + xx;
                            if (bits[j] & kCand) {
                                double mu, se;
                                background(a.rcoord[j], tab, a.n_bins, a.noise2, mu, se);
                                const double d = double(fr[a.lay.offset(yy, xx)]) - mu;
                                sums[0] += d;
                                sums[1] += se * se;
                                sums[2] += d * (double(yy) + 0.5);
                                sums[3] += d * (double(xx) + 0.5);
                            }
                        }
                    }
                    wave_sum_last_n(sums);
                    if (lane == kWave - 1) {
                        ss_peak rec;
                        rec.index = uint32_t(i);
                        rec.y = float(sums[2] / sums[0]);
                        rec.x = float(sums[3] / sums[0]);
                        rec.intensity = float(sums[0]);
                        rec.sigma = float(sqrt(sums[1]));
                        a.peaks[int64_t(f) * a.peak_capacity + pos] = rec;
                    }
                }
                ++pos;
            }
        }
    }
}

template <bool KEEP, bool PEAKS, int PPT>
void launch_compaction(const ClassArgs &a, hipStream_t stream) {
    const dim3 grid(uint32_t(a.tiles), uint32_t(a.n_frames));
    if (!a.counted) k_tile_counts<KEEP, PEAKS, PPT><<<grid, kBlock, 0, stream>>>(a);
    k_tile_scan<KEEP, PEAKS><<<dim3(uint32_t(a.n_frames)), kScanBlock, 0, stream>>>(a);
    k_tile_write<KEEP, PEAKS, PPT><<<grid, kBlock, 0, stream>>>(a);
}

template <bool KEEP, bool PEAKS>
void launch_compaction(const ClassArgs &a, bool few, hipStream_t stream) {
    if (few) launch_compaction<KEEP, PEAKS, kPPTFew>(a, stream);
    else launch_compaction<KEEP, PEAKS, kPPT>(a, stream);
}


// ---- densification (Sec. 3.2) -----------------------------------------------------------

constexpr int kDenseBlock = 256;
constexpr int kDensePPT = 4;     // consecutive pixels per thread (two generator blocks, one 16-byte store)
constexpr int kDenseFrames = 8;  // frames per work-group: radial codes read once per 8 frames
constexpr int kScatterBlock = 256;
constexpr int kVetoBlock = 256;

struct DenseArgs {
    const uint32_t *rcoord;
    const uint8_t *mask;
    int64_t n_pix;
    int32_t n_frames;
    int32_t n_bins;
    const Seg *table;
    float *dense;
    int32_t noisy;
    uint32_t key0, key1;
    int64_t frame0;
    float trunc;
    int32_t vec_ok;  // n_pix % 4 == 0 and dense 16-byte aligned: 16-byte stores
};

// Philox4x32-10 (Salmon et al., SC 2011) on the counter c under key (k0, k1):
// ten rounds of two 32 x 32 -> 64-bit products whose high halves are mixed
// into the other two words with the round key; the key advances by the two
// Weyl constants after every round.
__device__ inline void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// A pixel's standard normal from two generator words: Box-Muller on the
// 24-bit uniforms u1 in (0, 1] and u2 in [0, 1) (exact in float32), the
// first of the pair's two normals not above trunc, else trunc.
__device__ inline float noise_draw(uint32_t w1, uint32_t w2, float trunc) {
    const float u1 = float((w1 >> 8) + 1u) * 0x1p-24f;
    const float u2 = float(w2 >> 8) * 0x1p-24f;
    const float r = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    const float za = r * cs, zb = r * sn;
    return za <= trunc ? za : (zb <= trunc ? zb : trunc);
}

// One thread owns kDensePPT consecutive pixels for up to kDenseFrames
// frames: background mu (and sigma) from the frame's table in float64,
// plus sigma z for the noisy variant, 0 for masked pixels.  Pixel i draws
// from generator block i / 2 of counter (i / 2, absolute frame, 0, 0); the
// even pixel of a block takes words 0 and 1, the odd one words 2 and 3.
__global__ __launch_bounds__(kDenseBlock) void k_densify(DenseArgs a) {
    const int64_t p0 = (int64_t(blockIdx.x) * kDenseBlock + threadIdx.x) * kDensePPT;
    if (p0 >= a.n_pix) return;
    const int np = int(min(int64_t(kDensePPT), a.n_pix - p0));
    const int f0 = int(blockIdx.y) * kDenseFrames;
    const int f1 = min(a.n_frames, f0 + kDenseFrames);
    uint32_t rc[kDensePPT];
#pragma unroll
    for (int k = 0; k < kDensePPT; ++k) {
        rc[k] = SS_RC_MASKED;
        if (k < np) {
            rc[k] = a.rcoord[p0 + k];
            if (a.mask && a.mask[p0 + k]) rc[k] = SS_RC_MASKED;
        }
    }
    const bool vec = np == kDensePPT && a.vec_ok;
    for (int f = f0; f < f1; ++f) {
        const Seg *__restrict__ tab = a.table + int64_t(f) * (a.n_bins + 1);
        uint32_t w[2 * kDensePPT];
        if (a.noisy) {
            const uint32_t fr = uint32_t(a.frame0 + f);
#pragma unroll
            for (int b = 0; b < kDensePPT / 2; ++b) {
                uint32_t c[4] = {uint32_t(p0 >> 1) + uint32_t(b), fr, 0u, 0u};
                philox4x32_10(c, a.key0, a.key1);
#pragma unroll
                for (int j = 0; j < 4; ++j) w[4 * b + j] = c[j];
            }
        }
        float out[kDensePPT];
#pragma unroll
        for (int k = 0; k < kDensePPT; ++k) {
            out[k] = 0.0f;
            if (rc[k] != SS_RC_MASKED) {
                double mu, sd;
                background(rc[k], tab, a.n_bins, 0.0, mu, sd);
                out[k] = a.noisy ? float(mu + sd * double(noise_draw(w[2 * k], w[2 * k + 1], a.trunc))) : float(mu);
            }
        }
        float *dst = a.dense + int64_t(f) * a.n_pix + p0;
        if (vec) {
            *reinterpret_cast<float4 *>(dst) = make_float4(out[0], out[1], out[2], out[3]);
        } else {
#pragma unroll
            for (int k = 0; k < kDensePPT; ++k)
                if (k < np) dst[k] = out[k];
        }
    }
}

// Kept pixels back into their frames: entry k < min(n_kept, capacity) of
// frame f writes its value at its index; indices past the frame are skipped.
__global__ __launch_bounds__(kScatterBlock) void k_densify_scatter(const uint32_t *__restrict__ idx,
                                                                   const float *__restrict__ val, int64_t capacity,
                                                                   const int64_t *__restrict__ n_kept, int64_t n_pix,
                                                                   float *__restrict__ dense) {
    const int f = blockIdx.y;
    const int64_t n = min(max(n_kept[f], int64_t(0)), capacity);
    const int64_t o = int64_t(f) * capacity;
    for (int64_t k = int64_t(blockIdx.x) * kScatterBlock + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * kScatterBlock) {
        const uint32_t i = idx[o + k];
        if (int64_t(i) < n_pix) dense[int64_t(f) * n_pix + i] = val[o + k];
    }
}

// ---- peak-count veto (Sec. 4) -----------------------------------------------------------

// Frame f is a hit when n_peaks[f] >= threshold.  Counters (int64, added to,
// so they accumulate over calls): [0] hits, [1] non-hits, [2] kept entries of
// hits, [3] kept entries of non-hits, [4 + p] frames with p peaks and
// [4 + SS_VETO_BINS + p] their kept entries, p clamped to [0, SS_VETO_BINS - 1].
// Integer sums: the totals do not depend on the order of the additions.
__global__ __launch_bounds__(kVetoBlock) void k_veto(const int64_t *__restrict__ n_peaks,
                                                     const int64_t *__restrict__ n_kept, int32_t n_frames,
                                                     int64_t threshold, uint8_t *__restrict__ hit,
                                                     unsigned long long *__restrict__ counters) {
    const int f = int(blockIdx.x) * kVetoBlock + int(threadIdx.x);
    if (f >= n_frames) return;
    const int64_t p = n_peaks[f];
    const unsigned long long k = n_kept ? (unsigned long long)max(n_kept[f], int64_t(0)) : 0ull;
    const bool h = p >= threshold;
    if (hit) hit[f] = h ? 1 : 0;
    const int b = int(min(max(p, int64_t(0)), int64_t(SS_VETO_BINS - 1)));
    atomicAdd(counters + (h ? 0 : 1), 1ull);
    atomicAdd(counters + (h ? 2 : 3), k);
    atomicAdd(counters + 4 + b, 1ull);
    atomicAdd(counters + 4 + SS_VETO_BINS + b, k);
}


// ---- packed results ------------------------------------------------------------------------

constexpr int kPackBlock = 256;

// Exclusive offsets of the kept entries and peaks each frame returns
// (counts clamped to the capacities): offsets[0..F] for kept entries,
// offsets[F+1..2F+1] for peaks.  One work-group walks the frames in order.
__global__ __launch_bounds__(kPackBlock) void k_pack_offsets(const int64_t *__restrict__ n_kept, int64_t capacity,
                                                             const int64_t *__restrict__ n_peaks,
                                                             int64_t peak_capacity, int32_t n_frames,
                                                             int64_t *__restrict__ offsets) {
    __shared__ int64_t carry[2];
    __shared__ int64_t part[2][kPackBlock / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    if (tid == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    for (int base = 0; base < n_frames; base += kPackBlock) {
        const int f = base + tid;
        int64_t v[2] = {0, 0};
        if (f < n_frames) {
            v[0] = n_kept ? min(max(n_kept[f], int64_t(0)), capacity) : 0;
            v[1] = n_peaks ? min(max(n_peaks[f], int64_t(0)), peak_capacity) : 0;
        }
        int64_t incl[2] = {v[0], v[1]};
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int64_t t = __shfl_up(incl[q], off, kWave);
                if (lane >= off) incl[q] += t;
            }
        if (lane == kWave - 1) {
            part[0][wid] = incl[0];
            part[1][wid] = incl[1];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int64_t before = carry[q];
            for (int w = 0; w < wid; ++w) before += part[q][w];
            if (f < n_frames) offsets[int64_t(q) * (n_frames + 1) + f] = before + incl[q] - v[q];
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 0; w < kPackBlock / kWave; ++w) {
                carry[0] += part[0][w];
                carry[1] += part[1][w];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        offsets[n_frames] = carry[0];
        offsets[2 * int64_t(n_frames) + 1] = carry[1];
    }
}

// Frame f's first min(n, capacity) kept entries and peaks to their packed
// positions.
__global__ __launch_bounds__(kPackBlock) void k_pack_copy(const uint32_t *__restrict__ kept_index,
                                                          const float *__restrict__ kept_value, int64_t capacity,
                                                          const ss_peak *__restrict__ peaks, int64_t peak_capacity,
                                                          int32_t n_frames, const int64_t *__restrict__ offsets,
                                                          uint32_t *__restrict__ packed_index,
                                                          float *__restrict__ packed_value,
                                                          ss_peak *__restrict__ packed_peaks) {
    const int f = blockIdx.y;
    const int64_t stride = int64_t(gridDim.x) * kPackBlock;
    const int64_t t0 = int64_t(blockIdx.x) * kPackBlock + threadIdx.x;
    if (packed_index) {
        const int64_t o = offsets[f], n = offsets[f + 1] - o;
        for (int64_t k = t0; k < n; k += stride) {
            packed_index[o + k] = kept_index[int64_t(f) * capacity + k];
            packed_value[o + k] = kept_value[int64_t(f) * capacity + k];
        }
    }
    if (packed_peaks) {
        const int64_t o = offsets[n_frames + 1 + f], n = offsets[n_frames + 2 + f] - o;
        for (int64_t k = t0; k < n; k += stride) packed_peaks[o + k] = peaks[int64_t(f) * peak_capacity + k];
    }
}

}  // namespace
}  // namespace ss

extern "C" size_t ss_classify_workspace(int32_t n_frames, int64_t n_pix, int32_t n_bins) {
    if (n_frames < 0 || n_pix < 0 || n_bins < 0) return 0;
    return ss::workspace_bytes(n_frames, n_pix, n_bins);
}

namespace ss {
namespace {
template <int MODE, bool TILED>
void launch_pixel_state(const StateArgs &sa, int h, dim3 grid, size_t lds, hipStream_t stream) {
    if (h == 0) k_pixel_state<state_slots(0), 0, MODE, TILED><<<grid, kStencilBlock, lds, stream>>>(sa);
    else if (h == 1) k_pixel_state<state_slots(1), 1, MODE, TILED><<<grid, kStencilBlock, lds, stream>>>(sa);
    else if (h == 2) k_pixel_state<state_slots(2), 2, MODE, TILED><<<grid, kStencilBlock, lds, stream>>>(sa);
    else if (h <= 4) k_pixel_state<state_slots(4), -1, MODE, TILED><<<grid, kStencilBlock, lds, stream>>>(sa);
    else k_pixel_state<state_slots(SS_MAX_PATCH / 2), -1, MODE, TILED><<<grid, kStencilBlock, lds, stream>>>(sa);
}
}  // namespace
}  // namespace ss

extern "C" int ss_classify(const float *frames, const uint8_t *mask, int32_t n_frames, int32_t height,
                           int32_t width, const ss_radial *radial, const ss_profile *profile,
                           const ss_params *p, uint32_t *kept_index, float *kept_value, int64_t capacity,
                           int64_t *n_kept, ss_peak *peaks, int64_t peak_capacity, int64_t *n_peaks,
                           void *workspace, size_t ws_bytes, hipStream_t stream) {
    using namespace ss;
    if (!radial || !profile || !p) return SS_EINVAL;
    if (n_frames < 0 || height < 0 || width < 0 || capacity < 0 || peak_capacity < 0) return SS_ESIZE;
    const int64_t n_pix = int64_t(height) * width;
    if (n_pix >= (int64_t(1) << 29) || n_frames > 65535) return SS_ESIZE;
    if (radial->n_bins <= 0 || radial->n_bins > SS_MAX_BINS) return SS_ESIZE;
    if (p->patch < 1 || p->patch > SS_MAX_PATCH || (p->patch % 2) == 0) return SS_EINVAL;
    Layout lay{};
    if (n_pix > 0 && (!make_layout(height, width, radial->tile_w, radial->tile_h, lay) || lay.words >= (int64_t(1) << 29)))
        return SS_ESIZE;
    const bool keep = kept_index || kept_value || n_kept;
    const bool pk = peaks || n_peaks;
    if (keep && (!kept_index || !kept_value || !n_kept)) return SS_EINVAL;
    if (pk && (!peaks || !n_peaks)) return SS_EINVAL;
    if (n_frames == 0 || (!keep && !pk)) return SS_OK;
    if (!frames || !radial->rcoord || !profile->mean || !profile->std || !profile->n_members || !workspace)
        return SS_EINVAL;
    if (ws_bytes < workspace_bytes(n_frames, n_pix, radial->n_bins)) return SS_ESIZE;

    const bool few = n_frames <= kFewFrames;
    const int32_t tiles = int32_t(tiles_of(n_pix, few ? kPPTFew : kPPT));
    Workspace ws = carve(workspace, n_frames, n_pix, radial->n_bins);
    k_profile_table<<<dim3(uint32_t(n_frames)), kTableBlock, 0, stream>>>(
        profile->mean, profile->std, profile->n_members, radial->n_bins, ws, tiles, keep ? n_kept : nullptr,
        pk ? n_peaks : nullptr, double(p->n_pick), double(p->snr));
    SS_RETURN_IF_LAUNCH_FAILED();
    if (tiles == 0) return SS_OK;
    bool counted = false;
    {
        StateArgs sa;
        sa.frames = frames;
        sa.lay = lay;
        sa.rcoord = radial->rcoord;
        sa.mask = mask;
        sa.n_frames = n_frames;
        sa.height = height;
        sa.width = width;
        sa.n_pix = n_pix;
        sa.n_bins = radial->n_bins;
        sa.half = p->patch / 2;
        sa.min_count = p->min_count;
        sa.noise2 = double(p->noise) * double(p->noise);
        sa.n_pick = double(p->n_pick);
        sa.snr = double(p->snr);
        sa.noise2f = float(sa.noise2);
        sa.n_pick_f = p->n_pick;
        sa.snr_f = p->snr;
        sa.ws = ws;
        const int64_t tile_px = int64_t(kBlock) * (few ? kPPTFew : kPPT);
        sa.count_shift = __builtin_ctz(uint32_t(tile_px));
        sa.count_tiles = tiles;
        sa.counting = (int64_t(kTileH - 1) * width + kTileW) / tile_px + 2 <= kTileCounters;
        counted = sa.counting != 0;
        const int h = sa.half;
        const size_t lds = state_lds_bytes((kTileW + 2 * h) * (kTileH + 2 * h), state_slots(h));
        sa.tiles_x = (width + kTileW - 1) / kTileW;
        sa.tiles_y = (height + kTileH - 1) / kTileH;
        sa.frame_groups = (n_frames + kFramesPerBlock - 1) / kFramesPerBlock;
        const int64_t items = int64_t(sa.tiles_x) * sa.tiles_y * sa.frame_groups;
        if (items == 0) return SS_OK;
        if (items > (int64_t(1) << 31)) return SS_ESIZE;
        const dim3 grid(uint32_t(8 * ((items + 7) / 8)));
        // staging registers sized to the halo; patches 1, 3 and 5 unrolled;
        // threshold lines when there is no noise level (one line when
        // n_pick == snr); tile-ordered staging for tiled frame layouts
        const int mode = p->noise != 0.0f ? kModeBackground : p->n_pick == p->snr ? kModeLine : kModeLines;
        if (mode == kModeLine && lay.tiled()) launch_pixel_state<kModeLine, true>(sa, h, grid, lds, stream);
        else if (mode == kModeLine) launch_pixel_state<kModeLine, false>(sa, h, grid, lds, stream);
        else if (mode == kModeLines && lay.tiled()) launch_pixel_state<kModeLines, true>(sa, h, grid, lds, stream);
        else if (mode == kModeLines) launch_pixel_state<kModeLines, false>(sa, h, grid, lds, stream);
        else if (lay.tiled()) launch_pixel_state<kModeBackground, true>(sa, h, grid, lds, stream);
        else launch_pixel_state<kModeBackground, false>(sa, h, grid, lds, stream);
        SS_RETURN_IF_LAUNCH_FAILED();
    }

    ClassArgs a;
    a.frames = frames;
    a.lay = lay;
    a.n_frames = n_frames;
    a.mask = mask;
    a.rcoord = radial->rcoord;
    a.n_pix = n_pix;
    a.height = height;
    a.width = width;
    a.n_bins = radial->n_bins;
    a.tiles = tiles;
    a.counted = counted ? 1 : 0;
    a.n_pick = double(p->n_pick);
    a.snr = double(p->snr);
    a.noise2 = double(p->noise) * double(p->noise);
    a.half = p->patch / 2;
    a.min_count = p->min_count;
    a.kept_index = kept_index;
    a.kept_value = kept_value;
    a.capacity = capacity;
    a.n_kept = n_kept;
    a.peaks = peaks;
    a.peak_capacity = peak_capacity;
    a.n_peaks = n_peaks;
    a.ws = ws;
    if (keep && pk) launch_compaction<true, true>(a, few, stream);
    else if (keep) launch_compaction<true, false>(a, few, stream);
    else launch_compaction<false, true>(a, few, stream);
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}

// ---- classification without allocation ------------------------------------

namespace {

// The workspace of ss_classify_noalloc: one array per device, held from the
// library's load until the process ends.  In host code `scratch` is only a
// host-side stand-in for the symbol; the device address comes from
// hipGetSymbolAddress (once per device, with that device current) and is the
// only handle ever passed to kernels or copies.
static __device__ __align__(256) uint8_t scratch[SS_CLASSIFY_SCRATCH_BYTES];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kScratchDevices] = {};

int scratch_of_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) {
        (void)hipGetLastError();
        return SS_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return SS_EHIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return SS_OK;
}

}  // namespace

extern "C" int ss_classify_noalloc(const float *frames, const uint8_t *mask, int32_t n_frames, int32_t height,
                                   int32_t width, const ss_radial *radial, const ss_profile *profile,
                                   const ss_params *p, uint32_t *kept_index, float *kept_value, int64_t capacity,
                                   int64_t *n_kept, ss_peak *peaks, int64_t peak_capacity, int64_t *n_peaks,
                                   hipStream_t stream) {
    // sizes first, so that a call too large for the array touches no device state
    if (!radial || !profile || !p) return SS_EINVAL;
    if (n_frames < 0 || height < 0 || width < 0) return SS_ESIZE;
    const int64_t n_pix = int64_t(height) * width;
    if (n_pix >= (int64_t(1) << 29) || radial->n_bins <= 0 || radial->n_bins > SS_MAX_BINS) return SS_ESIZE;
    if (ss::workspace_bytes(n_frames, n_pix, radial->n_bins) > size_t(SS_CLASSIFY_SCRATCH_BYTES)) return SS_ESIZE;
    if (n_frames == 0)  // nothing is enqueued: the argument checks of ss_classify only
        return ss_classify(frames, mask, n_frames, height, width, radial, profile, p, kept_index, kept_value,
                           capacity, n_kept, peaks, peak_capacity, n_peaks, nullptr, 0, stream);
    void *ws = nullptr;
    const int rc = scratch_of_current_device(&ws);
    if (rc != SS_OK) return rc;
    return ss_classify(frames, mask, n_frames, height, width, radial, profile, p, kept_index, kept_value, capacity,
                       n_kept, peaks, peak_capacity, n_peaks, ws, size_t(SS_CLASSIFY_SCRATCH_BYTES), stream);
}

extern "C" int ss_compress(const float *frames, const uint8_t *mask, int32_t n_frames, int32_t height,
                           int32_t width, const ss_radial *radial, const ss_profile *profile,
                           const ss_params *params, uint32_t *kept_index, float *kept_value, int64_t capacity,
                           int64_t *n_kept, void *workspace, size_t ws_bytes, hipStream_t stream) {
    if (!kept_index || !kept_value || !n_kept) return SS_EINVAL;
    return ss_classify(frames, mask, n_frames, height, width, radial, profile, params, kept_index, kept_value,
                       capacity, n_kept, nullptr, 0, nullptr, workspace, ws_bytes, stream);
}

extern "C" int ss_peakfind(const float *frames, const uint8_t *mask, int32_t n_frames, int32_t height,
                           int32_t width, const ss_radial *radial, const ss_profile *profile,
                           const ss_params *params, ss_peak *peaks, int64_t peak_capacity, int64_t *n_peaks,
                           void *workspace, size_t ws_bytes, hipStream_t stream) {
    if (!peaks || !n_peaks) return SS_EINVAL;
    return ss_classify(frames, mask, n_frames, height, width, radial, profile, params, nullptr, nullptr, 0,
                       nullptr, peaks, peak_capacity, n_peaks, workspace, ws_bytes, stream);
}

extern "C" size_t ss_densify_workspace(int32_t n_frames, int32_t n_bins) {
    if (n_frames < 0 || n_bins < 0) return 0;
    using namespace ss;
    return 256 + align256(size_t(n_frames) * size_t(n_bins + 1) * sizeof(SegF)) +
           align256(size_t(n_frames) * size_t(n_bins + 1) * sizeof(Seg));
}

extern "C" int ss_densify(const uint32_t *kept_index, const float *kept_value, int64_t capacity,
                          const int64_t *n_kept, const uint8_t *mask, int32_t n_frames, int64_t n_pix,
                          const ss_radial *radial, const ss_profile *profile, const ss_noise *noise, float *dense,
                          void *workspace, size_t ws_bytes, hipStream_t stream) {
    using namespace ss;
    if (!radial || !profile) return SS_EINVAL;
    if (n_frames < 0 || n_pix < 0 || capacity < 0) return SS_ESIZE;
    if (n_pix >= (int64_t(1) << 31) || n_frames > 65535) return SS_ESIZE;
    if (radial->n_bins <= 0 || radial->n_bins > SS_MAX_BINS) return SS_ESIZE;
    if (noise && !(noise->trunc == noise->trunc)) return SS_EINVAL;  // NaN truncation
    if (n_frames == 0 || n_pix == 0) return SS_OK;
    if (!dense || !radial->rcoord || !profile->mean || !profile->std || !profile->n_members || !workspace)
        return SS_EINVAL;
    if (capacity > 0 && (!kept_index || !kept_value || !n_kept)) return SS_EINVAL;
    if (ws_bytes < ss_densify_workspace(n_frames, radial->n_bins)) return SS_ESIZE;

    Workspace ws{};
    uintptr_t q = (reinterpret_cast<uintptr_t>(workspace) + 255) & ~uintptr_t(255);
    ws.tablef = reinterpret_cast<SegF *>(q);
    q += align256(size_t(n_frames) * size_t(radial->n_bins + 1) * sizeof(SegF));
    ws.table = reinterpret_cast<Seg *>(q);
    k_profile_table<<<dim3(uint32_t(n_frames)), kTableBlock, 0, stream>>>(
        profile->mean, profile->std, profile->n_members, radial->n_bins, ws, 0, nullptr, nullptr, 0.0, 0.0);
    SS_RETURN_IF_LAUNCH_FAILED();

    DenseArgs a;
    a.rcoord = radial->rcoord;
    a.mask = mask;
    a.n_pix = n_pix;
    a.n_frames = n_frames;
    a.n_bins = radial->n_bins;
    a.table = ws.table;
    a.dense = dense;
    a.noisy = noise ? 1 : 0;
    a.key0 = noise ? uint32_t(noise->seed & 0xFFFFFFFFu) : 0u;
    a.key1 = noise ? uint32_t(noise->seed >> 32) : 0u;
    a.frame0 = noise ? noise->frame0 : 0;
    a.trunc = noise ? noise->trunc : 0.0f;
    a.vec_ok = (n_pix % kDensePPT) == 0 && (reinterpret_cast<uintptr_t>(dense) % 16) == 0;
    const int64_t threads = (n_pix + kDensePPT - 1) / kDensePPT;
    const dim3 grid(uint32_t((threads + kDenseBlock - 1) / kDenseBlock),
                    uint32_t((n_frames + kDenseFrames - 1) / kDenseFrames));
    k_densify<<<grid, kDenseBlock, 0, stream>>>(a);
    SS_RETURN_IF_LAUNCH_FAILED();
    if (capacity > 0) {
        const int64_t blocks = min(int64_t(256), (capacity + kScatterBlock - 1) / kScatterBlock);
        k_densify_scatter<<<dim3(uint32_t(blocks), uint32_t(n_frames)), kScatterBlock, 0, stream>>>(
            kept_index, kept_value, capacity, n_kept, n_pix, dense);
        SS_RETURN_IF_LAUNCH_FAILED();
    }
    return SS_OK;
}

extern "C" int ss_veto(const int64_t *n_peaks, const int64_t *n_kept, int32_t n_frames, int64_t threshold,
                       uint8_t *hit, int64_t *counters, hipStream_t stream) {
    using namespace ss;
    if (n_frames < 0) return SS_ESIZE;
    if (n_frames == 0) return SS_OK;
    if (!n_peaks || !counters) return SS_EINVAL;
    k_veto<<<dim3(uint32_t((n_frames + kVetoBlock - 1) / kVetoBlock)), kVetoBlock, 0, stream>>>(
        n_peaks, n_kept, n_frames, threshold, hit, reinterpret_cast<unsigned long long *>(counters));
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}

extern "C" int ss_pack_results(const uint32_t *kept_index, const float *kept_value, int64_t capacity,
                               const int64_t *n_kept, const ss_peak *peaks, int64_t peak_capacity,
                               const int64_t *n_peaks, int32_t n_frames, int64_t *offsets, uint32_t *packed_index,
                               float *packed_value, ss_peak *packed_peaks, hipStream_t stream) {
    using namespace ss;
    if (n_frames < 0 || n_frames > 65535 || capacity < 0 || peak_capacity < 0) return SS_ESIZE;
    if (!offsets) return SS_EINVAL;
    const bool keep = kept_index || kept_value || n_kept || packed_index || packed_value;
    const bool pk = peaks || n_peaks || packed_peaks;
    if (keep && (!kept_index || !kept_value || !n_kept || !packed_index || !packed_value)) return SS_EINVAL;
    if (pk && (!peaks || !n_peaks || !packed_peaks)) return SS_EINVAL;
    k_pack_offsets<<<dim3(1), kPackBlock, 0, stream>>>(keep ? n_kept : nullptr, capacity, pk ? n_peaks : nullptr,
                                                       peak_capacity, n_frames, offsets);
    SS_RETURN_IF_LAUNCH_FAILED();
    if (n_frames == 0 || (!keep && !pk)) return SS_OK;
    const int64_t longest = max(keep ? capacity : int64_t(0), pk ? peak_capacity : int64_t(0));
    const int64_t blocks = max(int64_t(1), min(int64_t(64), (longest + kPackBlock - 1) / kPackBlock));
    k_pack_copy<<<dim3(uint32_t(blocks), uint32_t(n_frames)), kPackBlock, 0, stream>>>(
        kept_index, kept_value, capacity, peaks, peak_capacity, n_frames, offsets, keep ? packed_index : nullptr,
        keep ? packed_value : nullptr, pk ? packed_peaks : nullptr);
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}
