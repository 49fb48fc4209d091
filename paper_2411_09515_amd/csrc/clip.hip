// Per-bin weighted statistics and iterative sigma-clipping (Sec. 2.2-2.5).
//
// One work-group owns one (bin, frame) pair.  Moments are float64 sums of
// shifted deviations d = v - K of the members (value v, weight omega):
//   S_w = sum omega, S_wd = sum omega d, S_w2 = sum omega^2,
//   S_w2d = sum omega^2 d, S_w2d2 = sum omega^2 d^2, S_pv = sum omega^2 var_v,
// so that mean = K + S_wd / S_w and, with delta = S_wd / S_w,
//   VV = S_w2d2 - 2 delta S_w2d + delta^2 S_w2     (= sum omega^2 (v - mean)^2).
// The first evaluation is a true two-pass: one sweep gives the mean, a second
// sweep accumulates around K = that mean, so VV is well conditioned (the
// register kernel does this per wave and merges the waves' sums exactly).  Every
// rejection pass then accumulates only the members it removes and subtracts
// them from the sums, so a pass costs one compare per member plus one
// work-group reduction.
//
// Two kernels share that arithmetic and the clip decision:
// * k_clip_regs keeps each member's value in registers (EPT per thread) and
//   re-reads a weight only when its member is removed.  Azimuthal model, no
//   extra mask, rows up to BLOCK * EPT entries: the hot path.
// * k_clip_stream keeps nothing on chip: every pass re-gathers the row and
//   replays the earlier passes' decisions from a (mean, threshold) history.
//   It serves the Poisson and hybrid models, an extra mask and rows of any
//   length.

#include <hip/hip_fp16.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

namespace ss {
namespace {

enum { S_W = 0, S_WD, S_W2, S_W2D, S_W2D2, S_PV, S_N, NSUM };

struct ClipArgs {
    const float *frames;
    int64_t n_pix;
    const float *norm;
    const uint8_t *mask;
    int32_t n_frames;
    int32_t n_bins;
    const int64_t *indptr;
    const int32_t *indices;
    const float *weight;
    int64_t nnz;
    const int32_t *bin_order;  // bins of this launch: bin_order[order_base + i], or i when null
    int32_t order_base;
    int32_t launch_bins;       // bins covered by this launch
    double cutoff;
    int32_t max_iter;
    int32_t model;
    double dark_var;
    double *mean;
    double *std;
    double *sem;
    double *sum_w;
    int32_t *n_members;
    int32_t *n_iter;
    int32_t *converged;
    // surrogate (register kernel only)
    float *features;        // [F][nb][SS_MLP_IN], features mode
    double *stats0;         // [F][nb][3], features mode
    const uint16_t *w16;    // [SS_MLP_PARAMS] float16 bits, surrogate mode
    double widen;           // widening of the predicted bounds, surrogate mode
    int32_t *accepted;      // [F][nb] states, surrogate mode (1 accepted, 0 none, -1 refused)
    const int32_t *redo;    // plain launch after the surrogate: process groups with state -1 only
    const double *pred_mean;  // [F][nb] given predictions, warm mode
    const double *pred_std;
};

// What k_clip_regs computes: the clipped profile, the surrogate's features
// only, the clipped profile with the verified surrogate first, or the
// clipped profile warm-started from given predictions (same verification).
enum { MODE_CLIP = 0, MODE_FEATURES = 1, MODE_SURROGATE = 2, MODE_WARM = 3 };

struct Stats {
    double mean, std, sem, pstd, psem;
};

__device__ inline Stats stats_from(const double (&s)[NSUM], double K) {
    Stats st{0.0, 0.0, 0.0, 0.0, 0.0};
    if (s[S_N] < 0.5 || !(s[S_W] > 0.0)) return st;
    const double delta = s[S_WD] / s[S_W];
    double vv = s[S_W2D2] - 2.0 * delta * s[S_W2D] + delta * delta * s[S_W2];
    vv = vv > 0.0 ? vv : 0.0;
    const double pv = s[S_PV] > 0.0 ? s[S_PV] : 0.0;
    st.mean = K + delta;
    st.std = sqrt(vv / s[S_W2]);
    st.sem = sqrt(vv) / s[S_W];
    st.pstd = sqrt(pv / s[S_W2]);
    st.psem = sqrt(pv) / s[S_W];
    return st;
}

// Pixel variance in units of v for the Poisson model (eq. poisson):
// (max(signal, 0) + sigma_dark^2) / norm^2 with signal = v * norm.
__device__ inline double poisson_var(float v, float nrm, double dark_var) {
    const double s = double(v) * double(nrm);
    return ((s > 0.0 ? s : 0.0) + dark_var) / (double(nrm) * double(nrm));
}

// Value of pixel idx, or NaN (not a member) when idx is outside the frame.
__device__ inline float gather(const float *__restrict__ fr, int32_t idx, int64_t n_pix) {
    return uint64_t(uint32_t(idx)) < uint64_t(n_pix) ? fr[idx] : __builtin_nanf("");
}

__device__ inline bool member_ok(float x, float w, const uint8_t *mask, int32_t idx) {
    return isfinite(x) && w > 0.0f && !(mask && mask[idx]);
}

// The clip decision of eq. clip (strict, two-sided), |v - mean| > thr, taken
// as v > hi or v < lo with hi = mean + thr and lo = mean - thr in float64.
// For a float32 v, v > hi exactly when v > RD32(hi) (no float32 lies
// strictly between RD32(hi) and hi), and v < lo exactly when v < RU32(lo),
// so the per-member test is two float32 compares against bounds rounded
// once per pass.
struct ClipBounds {
    float lo, hi;
};

__device__ inline ClipBounds clip_bounds(double mean, double thr) {
    return ClipBounds{__double2float_ru(mean - thr), __double2float_rd(mean + thr)};
}

__device__ inline bool clipped(float x, ClipBounds b) { return x > b.hi || x < b.lo; }

// Cut-off of pass k: the fixed value, or Chauvenet's value for the current
// size (eq. chauvenet); <= 0 means nothing can be removed.
// (Out of line: the logarithm's constants would otherwise hold registers
// across the whole pass loop of the kernels that inline the planner.)
__device__ __attribute__((noinline)) double chauvenet_cutoff(double size) {
    constexpr double kSqrt2Pi = 2.5066282746310002;
    return size > kSqrt2Pi ? sqrt(2.0 * log(size / kSqrt2Pi)) : -1.0;
}

__device__ inline double cutoff_for(double cutoff, double size) {
    return cutoff > 0.0 ? cutoff : chauvenet_cutoff(size);
}

// The running sums are decremented as members leave.  When the variance they
// imply has lost more than about six of float64's sixteen digits to
// cancellation (aggressive cut-offs shrink the spread by orders of magnitude
// over many passes), they are re-accumulated around the current mean.
__device__ inline bool needs_refresh(const double (&s)[NSUM]) {
    if (s[S_N] < 0.5 || !(s[S_W] > 0.0)) return false;
    const double delta = s[S_WD] / s[S_W];
    const double mag = s[S_W2D2] + delta * delta * s[S_W2];
    const double vv = s[S_W2D2] - 2.0 * delta * s[S_W2D] + delta * delta * s[S_W2];
    return mag > 0.0 && !(vv > 1e-6 * mag);
}

__device__ inline void add_member(double (&s)[NSUM], double w, double d, double pv) {
    const double w2 = w * w;
    s[S_W] += w;
    s[S_WD] += w * d;
    s[S_W2] += w2;
    s[S_W2D] += w2 * d;
    s[S_W2D2] += w2 * d * d;
    s[S_PV] += w2 * pv;
    s[S_N] += 1.0;
}

// Work-group -> (frame, bin), or (group of fpi frames, bin).  Work-groups are
// dispatched to the 8 XCDs round robin (work-group g runs on XCD g % 8), so
// work-group g is given item x * per + g / 8 of an ordered item list,
// x = g % 8: each XCD walks a contiguous run of that list.  The list is
// tiled: kTileFrames frame groups by kTileBins bins at a time, frame-major
// inside a tile, tiles bin-major inside a run of kTileFrames frame groups.
// The work-groups an XCD holds at once then cover a few neighbouring bins of
// a few frames: neighbouring bins share the cache lines of their rings
// (gathers), and the frames of one bin share its CSR row, so both are read
// from HBM about once per tile instead of once per work-group.  Returns
// false for the padding work-groups beyond the list.
#ifndef SS_CLIP_TILE_FRAMES
#define SS_CLIP_TILE_FRAMES 1
#endif
#ifndef SS_CLIP_TILE_BINS
#define SS_CLIP_TILE_BINS 8
#endif
constexpr uint32_t kTileFrames = SS_CLIP_TILE_FRAMES;
constexpr uint32_t kTileBins = SS_CLIP_TILE_BINS;

__device__ inline void tile_item(uint32_t item, uint32_t nfg, uint32_t nb, uint32_t &fg, uint32_t &local) {
    const uint32_t ft = item / (kTileFrames * nb);
    const uint32_t gt = min(kTileFrames, nfg - ft * kTileFrames);
    const uint32_t rem = item - ft * kTileFrames * nb;
    const uint32_t bt = rem / (gt * kTileBins);
    const uint32_t btn = min(kTileBins, nb - bt * kTileBins);
    const uint32_t r2 = rem - bt * gt * kTileBins;
    fg = ft * kTileFrames + r2 / btn;
    local = bt * kTileBins + r2 % btn;
}

__device__ inline bool block_item(const ClipArgs &a, int fpi, int &f, int &bin) {
    const uint32_t nb = uint32_t(a.launch_bins);
    const uint32_t nfg = uint32_t((a.n_frames + fpi - 1) / fpi);
    const uint32_t total = nfg * nb;
    const uint32_t per = (total + 7u) / 8u;
    const uint32_t g = blockIdx.x;
    const uint32_t item = (g % 8u) * per + g / 8u;
    if (g / 8u >= per || item >= total) return false;
    uint32_t fg, local;
    tile_item(item, nfg, nb, fg, local);
    f = int(fg);
    bin = a.bin_order ? a.bin_order[a.order_base + int(local)] : int(local);
    return uint32_t(bin) < uint32_t(a.n_bins);
}

// Grid size for block_item: 8 runs of ceil(total / 8) work-groups.
inline uint32_t item_grid(int64_t total) { return uint32_t(8 * ((total + 7) / 8)); }

__device__ inline void row_bounds(const ClipArgs &a, int bin, int64_t &start, int64_t &end) {
    // clamped to [0, nnz] so a malformed indptr cannot read past the arrays
    end = min(max(a.indptr[bin + 1], int64_t(0)), a.nnz);
    start = min(max(a.indptr[bin], int64_t(0)), end);
}

__device__ inline void write_profile(const ClipArgs &a, int f, int bin, const double (&s)[NSUM], const Stats &st,
                                     int n_iter, int converged) {
    const int64_t o = int64_t(f) * a.n_bins + bin;
    const bool report_poisson = a.model != SS_AZIMUTHAL;
    const bool empty = s[S_N] < 0.5;
    a.mean[o] = empty ? 0.0 : st.mean;
    a.std[o] = empty ? 0.0 : (report_poisson ? st.pstd : st.std);
    a.sem[o] = empty ? 0.0 : (report_poisson ? st.psem : st.sem);
    a.sum_w[o] = empty ? 0.0 : s[S_W];
    a.n_members[o] = int32_t(s[S_N]);
    a.n_iter[o] = n_iter;
    a.converged[o] = converged;
}

// Shift for the first sweep: the row's first value (any value near the data
// keeps the sums well scaled).
__device__ inline double first_shift(const ClipArgs &a, const float *fr, int64_t start, int64_t end) {
    if (end <= start) return 0.0;
    const float x0 = gather(fr, a.indices[start], a.n_pix);
    return isfinite(x0) ? double(x0) : 0.0;
}

// ---------------------------------------------------------------------------

// Pass control, computed by one thread and published to the work-group.
struct PassCtl {
    double mean, thr, K;
    ClipBounds bounds;
    int go, n_iter, converged, refresh;
};

// Bookkeeping after rejection pass: stop when it removed nothing.
__device__ inline void after_pass(PassCtl &c, bool removed_any) {
    if (!removed_any) {
        c.converged = 1;
        c.go = 0;
    } else {
        c.n_iter += 1;
    }
}

// Plan pass k_next from the running sums: a refresh of the sums when they
// have lost precision, otherwise the next (mean, threshold), or stop.
__device__ inline void plan(const ClipArgs &a, const double (&s)[NSUM], PassCtl &c, int k_next, bool allow_refresh) {
    // only the mean and the spread that clips are needed here (the other
    // statistics are formed once, for the output)
    double spread = 0.0;
    c.mean = 0.0;
    if (s[S_N] >= 0.5 && s[S_W] > 0.0) {
        const double delta = s[S_WD] / s[S_W];
        c.mean = c.K + delta;
        double var = (a.model == SS_POISSON) ? s[S_PV]
                                             : s[S_W2D2] - 2.0 * delta * s[S_W2D] + delta * delta * s[S_W2];
        var = var > 0.0 ? var : 0.0;
        spread = sqrt(var / s[S_W2]);
    }
    c.refresh = 0;
    if (allow_refresh && needs_refresh(s)) {
        c.refresh = 1;
        c.go = 1;
        return;
    }
    if (k_next >= a.max_iter) {
        c.go = 0;
        return;
    }
    const double ncut = cutoff_for(a.cutoff, s[S_N]);
    if (!(ncut > 0.0)) {
        c.converged = 1;
        c.go = 0;
        return;
    }
    c.thr = ncut * spread;
    c.bounds = clip_bounds(c.mean, c.thr);
    c.go = 1;
}

__device__ inline void load_state(const double *state, double (&s)[NSUM]) {
#pragma unroll
    for (int q = 0; q < NSUM; ++q) s[q] = state[q];
}

// Capacity (entries) of one wave's list of removed members, per frame and
// round, in k_clip_regs.  It holds a full slot's worth (one entry per lane),
// so every round makes progress.
constexpr int kRemCap = kWave;

// Removal lists the planning wave reads together per LDS round trip.
#ifndef SS_CLIP_LIST_GROUP
#define SS_CLIP_LIST_GROUP 4
#endif
constexpr int kListGroup = SS_CLIP_LIST_GROUP;

enum { R_W = 0, R_WD, R_W2, R_W2D, R_W2D2, NREM };

// Per-wave sums of the first evaluation (around the wave's own mean).
enum { W_W = 0, W_WD, W_W2, W_W2D, W_W2D2, W_N, W_MEAN, NWSTAT };

typedef float float2v __attribute__((ext_vector_type(2)));

__device__ inline void add_removed(double (&r)[NREM], double w, double d) {
    const double w2 = w * w;
    r[R_W] += w;
    r[R_WD] += w * d;
    r[R_W2] += w2;
    r[R_W2D] += w2 * d;
    r[R_W2D2] += w2 * d * d;
}

// Register-resident clip of one bin for FB frames at once.
//
// The work-group holds the row's weights in LDS (loaded once for all FB
// frames) and each member's value in registers, slot e of thread t holding
// entry e * BLOCK + t; a value is NaN when the entry is not, or no longer, a
// member, so a clip compare leaves it alone.  The frames' reductions are
// independent, so their latency chains overlap.
//
// A rejection pass: every wave compares its values against the frame's
// bounds and packs the (weight, value) pairs of the members it removes into
// its LDS list for that frame (ballot + prefix count); after a barrier,
// wave f % NW sums the lists of frame f in a fixed order (deterministic),
// takes the sums off the running state and plans the frame's next pass.  A wave
// whose list fills up stops and asks for another round of the same pass.
// Smallest bin the warm start is tried on.
constexpr int kWarmMinMembers = 64;

// Per-frame surrogate state, in LDS.
struct Surrogate {
    double n0, m0, s0;          // unclipped statistics
    double mean_hat, std_hat;   // the network's prediction
    double half;                // predicted keep half-width cutoff (1 + widen) std_hat
    ClipBounds fin;             // bounds of the final statistics
    int on;                     // a real frame with members
    int warm;                   // pass 0 uses the prediction
    int back;                   // a removed member lies within the final bounds
};

__device__ inline float half_to_float(uint16_t h) { return __half2float(__ushort_as_half(h)); }

__device__ inline float gelu(float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define SS_V(f, e) vp[f][(e) >> 1][(e) & 1]

__device__ inline double u_mean(const Surrogate &u, double y0) { return u.m0 + y0 * u.s0; }
__device__ inline double u_std(const Surrogate &u, double y1) { return u.s0 * exp(y1); }

// The warm start of a frame's clip from a predicted converged (mean, std):
// pass 0 also removes the members outside mean_hat +- cutoff (1 + widen)
// std_hat.  No warm start in small bins or where the predicted interval
// reaches zero (low counts): their clip can have several fixed points (for
// low counts one per photon-number cluster), and a warm start could settle
// on another one than the plain clip.
__device__ inline void warm_start(const ClipArgs &a, Surrogate &u, PassCtl &ctl, double mean_hat, double std_hat) {
    u.mean_hat = mean_hat;
    u.std_hat = std_hat;
    u.half = a.cutoff * (1.0 + a.widen) * u.std_hat;
    u.warm = u.on && u.n0 >= double(kWarmMinMembers) && u.s0 > 0.0 && ctl.go && u.half > 0.0 &&
             u.mean_hat - u.half > 0.0;
    if (u.warm) {
        // pass 0 keeps the members within both its own bounds and
        // |v - mean_hat| <= half, i.e. RU32(mean_hat - half) <= v <= RD32(mean_hat + half)
        ctl.bounds.lo = fmaxf(ctl.bounds.lo, __double2float_ru(u.mean_hat - u.half));
        ctl.bounds.hi = fminf(ctl.bounds.hi, __double2float_rd(u.mean_hat + u.half));
    }
}

// The surrogate stage of k_clip_regs, after the first evaluation: the
// 16-point sketch and the features; in surrogate mode also the network's
// prediction (wave 0, one hidden unit per lane), which narrows the bounds of
// the first clipping pass (a warm start of the plain passes that follow).
// Returns true when the work-group is done (features mode).
template <int BLOCK, int EPT, int FB, int MODE>
__device__ inline bool surrogate_stage(const ClipArgs &a, float2v (&vp)[FB][EPT / 2], uint32_t *hist,
                                       float (*sk_s)[16], float (*feat_s)[SS_MLP_IN], Surrogate *sur_s,
                                       const uint16_t *wts_s, float *h1_s, PassCtl *ctl, int f0, int nf, int bin) {
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;

    // sketch: member v goes to bucket j = #{k : v > b_k}; then #{v <= b_k} is
    // the sum of buckets 0..k (the bounds do not decrease)
#pragma unroll
    for (int f = 0; f < FB; ++f)
        if (lane < 17) hist[(f * NW + wid) * 17 + lane] = 0u;
    wave_sync();
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        if (!sur_s[f].on) continue;
        float b[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) b[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sk_s[f][k])));
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const float x = SS_V(f, e);
            if (x == x) {
                uint32_t j = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) j += x > b[k] ? 1u : 0u;
                atomicAdd(&hist[(f * NW + wid) * 17 + j], 1u);
            }
        }
    }
    __syncthreads();
    if (tid < FB) {
        const int f = tid;
        const Surrogate u = sur_s[f];
        float x[SS_MLP_IN];
#pragma unroll
        for (int q = 0; q < SS_MLP_IN; ++q) x[q] = 0.0f;
        if (u.on) {
            x[0] = float(log1p(u.n0));
            x[1] = float(asinh(u.m0));
            x[2] = float(asinh(u.s0));
            uint32_t cum = 0;
            for (int k = 0; k < 16; ++k) {
                for (int w = 0; w < NW; ++w) cum += hist[(f * NW + w) * 17 + k];
                x[3 + k] = float(double(cum) / u.n0);
            }
        }
#pragma unroll
        for (int q = 0; q < SS_MLP_IN; ++q) feat_s[f][q] = x[q];
        if (MODE == MODE_FEATURES && f < nf) {
            const int64_t o = int64_t(f0 + f) * a.n_bins + bin;
#pragma unroll
            for (int q = 0; q < SS_MLP_IN; ++q) a.features[o * SS_MLP_IN + q] = x[q];
            a.stats0[o * 3] = u.n0;
            a.stats0[o * 3 + 1] = u.on ? u.m0 : 0.0;
            a.stats0[o * 3 + 2] = u.on ? u.s0 : 0.0;
        }
    }
    if constexpr (MODE == MODE_FEATURES) return true;
    __syncthreads();

    // the network, on wave 0: lane j is hidden unit j of both layers
    if (wid == 0) {
        float z[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) z[f] = half_to_float(wts_s[SS_MLP_OFF_B1 + lane]);
#pragma unroll 1
        for (int i = 0; i < SS_MLP_IN; ++i) {
            const float w = half_to_float(wts_s[SS_MLP_OFF_W1 + i * SS_MLP_HID + lane]);
#pragma unroll
            for (int f = 0; f < FB; ++f) z[f] = fmaf(feat_s[f][i], w, z[f]);
        }
#pragma unroll
        for (int f = 0; f < FB; ++f) h1_s[f * SS_MLP_HID + lane] = gelu(z[f]);
        wave_sync();
#pragma unroll
        for (int f = 0; f < FB; ++f) z[f] = half_to_float(wts_s[SS_MLP_OFF_B2 + lane]);
#pragma unroll 2
        for (int i = 0; i < SS_MLP_HID; ++i) {
            const float w = half_to_float(wts_s[SS_MLP_OFF_W2 + i * SS_MLP_HID + lane]);
#pragma unroll
            for (int f = 0; f < FB; ++f) z[f] = fmaf(h1_s[f * SS_MLP_HID + i], w, z[f]);
        }
        const float w30 = half_to_float(wts_s[SS_MLP_OFF_W3 + lane * SS_MLP_OUT_PAD]);
        const float w31 = half_to_float(wts_s[SS_MLP_OFF_W3 + lane * SS_MLP_OUT_PAD + 1]);
        const float b30 = half_to_float(wts_s[SS_MLP_OFF_B3]);
        const float b31 = half_to_float(wts_s[SS_MLP_OFF_B3 + 1]);
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            const float h2 = gelu(z[f]);
            const double y0 = wave_sum(double(h2 * w30)) + double(b30);
            const double y1 = wave_sum(double(h2 * w31)) + double(b31);
            if (lane == 0) warm_start(a, sur_s[f], ctl[f], u_mean(sur_s[f], y0), u_std(sur_s[f], y1));
        }
    }
    __syncthreads();
    return false;
}

// The register clip of one (frame group, bin).  WLDS: the row's weights are
// staged in LDS (rows up to 24 576 entries); otherwise they are read again
// from memory (L2) where needed, for the longest rows.
template <int BLOCK, int EPT, int FB, int MODE, bool WLDS>
__device__ __forceinline__ void clip_body(const ClipArgs &a, int g, int bin) {
    constexpr int NW = BLOCK / kWave;
    constexpr int FPW = (FB + NW - 1) / NW;  // frames finished per wave
    static_assert(FB >= 1 && BLOCK % kWave == 0, "whole waves, at least one frame");
    constexpr bool SKETCH = MODE == MODE_FEATURES || MODE == MODE_SURROGATE;
    constexpr bool SUR = MODE == MODE_SURROGATE || MODE == MODE_WARM;
    __shared__ uint32_t hist[SKETCH ? FB : 1][SKETCH ? NW : 1][17];
    __shared__ float sk_s[FB][16];          // sketch bounds
    __shared__ float feat_s[FB][SS_MLP_IN];
    __shared__ Surrogate sur_s[FB];
    __shared__ uint16_t wts_s[MODE == MODE_SURROGATE ? SS_MLP_PARAMS : 2];
    __shared__ float h1_s[MODE == MODE_SURROGATE ? FB : 1][SS_MLP_HID];
    __shared__ float w_s[WLDS ? EPT * BLOCK : 1];
    __shared__ float2 rem_s[NW][FB][kRemCap];
    __shared__ int cnt_s[NW][FB];
    __shared__ int more_s[NW];
    __shared__ double part[NSUM * NW];
    __shared__ double tot[NSUM];
    __shared__ double state[FB][NSUM];
    __shared__ double wstat[FB][NW][NWSTAT];
    __shared__ PassCtl ctl[FB];

    const int f0 = g * FB;
    const int nf = min(FB, a.n_frames - f0);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    if (a.redo) {
        // a second, plain launch after the surrogate: only groups holding a refused frame
        bool any = false;
        for (int f = 0; f < nf; ++f) any = any || a.redo[int64_t(f0 + f) * a.n_bins + bin] == -1;
        if (!any) return;
    }
    int64_t start, end;
    row_bounds(a, bin, start, end);
    const int len = int(end - start);

    if (len == 0) {
        if (tid < nf) {
            const int64_t o = int64_t(f0 + tid) * a.n_bins + bin;
            if constexpr (MODE == MODE_FEATURES) {
                for (int q = 0; q < SS_MLP_IN; ++q) a.features[o * SS_MLP_IN + q] = 0.0f;
                for (int q = 0; q < 3; ++q) a.stats0[o * 3 + q] = 0.0;
            } else if (a.redo == nullptr || a.redo[o] == -1) {
                const double z[NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                write_profile(a, f0 + tid, bin, z, Stats{0.0, 0.0, 0.0, 0.0, 0.0}, 0, a.max_iter > 0 ? 1 : 0);
                if (SUR) a.accepted[o] = 0;
            }
        }
        return;
    }
    const uint32_t last = uint32_t(a.n_pix - 1);

    // Buffer views of the row and of the frames: every load below is issued
    // unconditionally with its whole offset in the range-checked vector
    // offset, so slots past the row end read index 0 and weight 0 (not an
    // entry), and frames past the batch read 0 and are masked after.  A
    // work-group waits for two memory round trips: the row's indices and
    // weights, then the gathers.
    const __amdgpu_buffer_rsrc_t ri = buffer_rsrc(a.indices + start, uint32_t(len) * 4u);
    const __amdgpu_buffer_rsrc_t rw = buffer_rsrc(a.weight + start, uint32_t(len) * 4u);
    __amdgpu_buffer_rsrc_t rf[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        const bool real = f < nf;
        const float *fr = a.frames + (real ? int64_t(f0 + f) * a.n_pix : 0);
        rf[f] = buffer_rsrc(fr, real ? uint32_t(a.n_pix) * 4u : 0u);
    }
    const uint32_t tofs = uint32_t(tid) * 4u;
    // weight of slot e: from LDS, or again from memory for the longest rows
#define SS_W(e) (WLDS ? w_s[(e) * BLOCK + tid] : buffer_load_f32(rw, tofs + uint32_t((e) * BLOCK) * 4u, 0u))

    // Values are held in pairs: float64 operands need even-aligned register
    // pairs, and single floats scattered over odd registers would leave the
    // even ones unusable for them.
    static_assert(EPT % 2 == 0, "values are held in pairs");
    float2v vp[FB][EPT / 2];
    double K[FB];
    // sweep 1: gather, Omega, the wave's mean.  Register use peaks here, so the
    // weights go to LDS as soon as they arrive (0 for a slot that is not an
    // entry: past the row, weight <= 0 or index outside the frame; without
    // LDS, a bit mask holds that instead), and each index register is free
    // once its gathers are issued.
    {
        uint64_t ok_entry = 0;
        {
            int32_t ix[EPT];
            float wt[EPT];
#pragma unroll
            for (int e = 0; e < EPT; ++e) wt[e] = buffer_load_f32(rw, tofs + uint32_t(e * BLOCK) * 4u, 0u);
#pragma unroll
            for (int e = 0; e < EPT; ++e) ix[e] = buffer_load_i32(ri, tofs + uint32_t(e * BLOCK) * 4u, 0u);
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const bool ok = wt[e] > 0.0f && uint32_t(ix[e]) <= last;
                if constexpr (WLDS)
                    w_s[e * BLOCK + tid] = ok ? wt[e] : 0.0f;
                else
                    ok_entry |= uint64_t(ok) << e;
            }
#pragma unroll
            for (int f = 0; f < FB; ++f)
#pragma unroll
                for (int e = 0; e < EPT; ++e) SS_V(f, e) = buffer_load_f32(rf[f], uint32_t(ix[e]) * 4u, 0u);
        }
        if constexpr (MODE == MODE_SURROGATE) {
            // the network's parameters, while the gathers are in flight
            const uint4 *src = reinterpret_cast<const uint4 *>(a.w16);
            uint4 *dst = reinterpret_cast<uint4 *>(wts_s);
            for (int i = tid; i < SS_MLP_PARAMS / 8; i += BLOCK) dst[i] = src[i];
        }
        // (the weights are read back from LDS below, not kept in registers)
        asm volatile("" ::: "memory");
        // branch-free: a non-member enters the sums with weight and value 0
        double t[3 * FB];
        int n_ok[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            n_ok[f] = 0;
            t[3 * f] = t[3 * f + 1] = 0.0;
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const float w = SS_W(e);
            const bool entry_ok = WLDS ? w > 0.0f : (uint32_t(ok_entry >> e) & 1u) != 0;
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const float x = SS_V(f, e);
                const bool ok = entry_ok && (f < nf) && __builtin_isfinite(x);
                float wz = ok ? w : 0.0f;
                float xz = ok ? x : 0.0f;
                // select in float32, then widen (one select per operand
                // instead of one per half of its float64 widening)
                asm("" : "+v"(wz), "+v"(xz));
                // one frame per group: the LDS weight becomes the member's
                // weight (0 for a non-member), so sweep 2 needs no select
                if constexpr (WLDS && FB == 1) w_s[e * BLOCK + tid] = wz;
                t[3 * f + 0] += double(wz);
                t[3 * f + 1] = fma(double(wz), double(xz), t[3 * f + 1]);
                n_ok[f] += ok ? 1 : 0;
                SS_V(f, e) = ok ? x : __builtin_nanf("");
            }
        }
        // this wave's mean of each frame, known to all its lanes (the
        // member counts summed as float64, exact)
#pragma unroll
        for (int f = 0; f < FB; ++f) t[3 * f + 2] = double(n_ok[f]);
        wave_sum_last_n(t);
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            t[3 * f + 0] = readlane(t[3 * f + 0], kWave - 1);
            t[3 * f + 1] = readlane(t[3 * f + 1], kWave - 1);
            t[3 * f + 2] = readlane(t[3 * f + 2], kWave - 1);
            K[f] = t[3 * f] > 0.0 ? t[3 * f + 1] / t[3 * f] : 0.0;
            if (lane == kWave - 1) {
                wstat[f][wid][W_W] = t[3 * f];
                wstat[f][wid][W_N] = t[3 * f + 2];
                wstat[f][wid][W_MEAN] = K[f];
            }
        }
    }
    // The float64 conversions of sweep 1 are not kept for sweep 2 (that
    // would hold two more registers per member): the values pass through an
    // empty asm statement, which the compiler cannot see through, and no
    // instruction is scheduled across this point (sweep 2's weight reads
    // would otherwise be hoisted above the reductions, with their registers).
#pragma unroll
    for (int f = 0; f < FB; ++f)
#pragma unroll
        for (int e = 0; e < EPT / 2; ++e) asm volatile("" : "+v"(vp[f][e]));
    __builtin_amdgcn_sched_barrier(0);
    // sweep 2: deviations around the wave's mean (two-pass VV per wave)
    {
        double t[4 * FB];
#pragma unroll
        for (int q = 0; q < 4 * FB; ++q) t[q] = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const float w = SS_W(e);
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const float x = SS_V(f, e);
                const bool ok = x == x;
                const double wz = double((WLDS && FB == 1) || ok ? w : 0.0f);
                const double d = double(ok ? x : 0.0f) - K[f];
                const double wd = wz * d;
                t[4 * f + 0] += wd;
                t[4 * f + 1] = fma(wz, wz, t[4 * f + 1]);
                t[4 * f + 2] = fma(wz, wd, t[4 * f + 2]);
                t[4 * f + 3] = fma(wd, wd, t[4 * f + 3]);
            }
        }
        wave_sum_last_n(t);
        if (lane == kWave - 1) {
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                wstat[f][wid][W_WD] = t[4 * f];
                wstat[f][wid][W_W2] = t[4 * f + 1];
                wstat[f][wid][W_W2D] = t[4 * f + 2];
                wstat[f][wid][W_W2D2] = t[4 * f + 3];
            }
        }
    }
    __syncthreads();
    // Merge the waves' sums, each taken around its own mean m_w, at the
    // frame's mean K: with D = m_w - K a deviation around K is d + D, so
    // S_wd gains D S_w, S_w2d gains D S_w2 and S_w2d2 gains
    // 2 D S_w2d + D^2 S_w2 (exact algebra; every wave's own VV is two-pass).
    if (tid < FB) {
        const int f = tid;
        double sw = 0.0, sv = 0.0;
        // four waves' sums per LDS round trip (not fully unrolled: one
        // thread, and the whole table would fill its registers)
#pragma unroll 4
        for (int w = 0; w < NW; ++w) {
            sw += wstat[f][w][W_W];
            sv += wstat[f][w][W_W] * wstat[f][w][W_MEAN] + wstat[f][w][W_WD];
        }
        const double Kf = sw > 0.0 ? sv / sw : 0.0;
        double st[NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int w = 0; w < NW; ++w) {
            const double *x = wstat[f][w];
            const double D = x[W_MEAN] - Kf;
            st[S_W] += x[W_W];
            st[S_WD] += x[W_WD] + D * x[W_W];
            st[S_W2] += x[W_W2];
            st[S_W2D] += x[W_W2D] + D * x[W_W2];
            st[S_W2D2] += x[W_W2D2] + D * (2.0 * x[W_W2D] + D * x[W_W2]);
            st[S_N] += x[W_N];
        }
#pragma unroll
        for (int q = 0; q < NSUM; ++q) state[f][q] = st[q];
        PassCtl c{0.0, 0.0, Kf, ClipBounds{0.0f, 0.0f}, 0, 0, 0, 0};
        plan(a, st, c, 0, false);
        if (f >= nf) c.go = 0;
        ctl[f] = c;
        if constexpr (SKETCH || SUR) {
            const Stats s0 = stats_from(st, Kf);
            Surrogate u{};
            u.n0 = st[S_N];
            u.m0 = s0.mean;
            u.s0 = s0.std;
            u.on = f < nf && st[S_N] >= 0.5;
            if constexpr (MODE == MODE_WARM) {
                // the given prediction of this (frame, bin)
                const int64_t o = int64_t(f0 + f) * a.n_bins + bin;
                if (u.on) warm_start(a, u, c, a.pred_mean[o], a.pred_std[o]);
                ctl[f] = c;
            }
            sur_s[f] = u;
            // v <= m0 + t s0 exactly when v <= RD32(m0 + t s0)
            if constexpr (SKETCH) {
#pragma unroll
                for (int k = 0; k < 16; ++k) sk_s[f][k] = __double2float_rd(s0.mean + (-3.75 + 0.5 * k) * s0.std);
            }
        }
    }
    __syncthreads();
    if constexpr (SKETCH) {
        if (surrogate_stage<BLOCK, EPT, FB, MODE>(a, vp, &hist[0][0][0], sk_s, feat_s, sur_s, wts_s, &h1_s[0][0], ctl, f0,
                                                  nf, bin))
            return;
    }

    // members removed by a pass (surrogate mode keeps their values; the
    // other modes overwrite a removed value with NaN instead)
    uint64_t gone[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) gone[f] = 0;
    static_assert(!SUR || EPT <= 64, "removal flags live in one 64-bit word");

    // rejection passes
    for (int k = 0;; ++k) {
        // One frame per group (the plain clip): this pass's bounds and flags
        // are read together once, one LDS round trip at the head of the
        // pass instead of a read of the flag, a branch, then a read of the
        // bounds (with more frames the held copies would cost registers).
        constexpr bool HOLD = FB == 1 && !SUR && !SKETCH;
        ClipBounds bnd_f[FB];
        int go_f[FB], refresh_f[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            bnd_f[f] = ctl[f].bounds;
            go_f[f] = ctl[f].go;
            refresh_f[f] = ctl[f].refresh;
        }
        auto go_of = [&](int f) { return HOLD ? go_f[f] : ctl[f].go; };
        auto bnd_of = [&](int f) { return HOLD ? bnd_f[f] : ctl[f].bounds; };
        bool any = false;
#pragma unroll
        for (int f = 0; f < FB; ++f) any = any || go_of(f) != 0;
        if (!any) break;
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            if (!(go_of(f) && (HOLD ? refresh_f[f] : ctl[f].refresh))) continue;
            // re-accumulate the surviving members around the current mean
            const double Kn = ctl[f].mean;
            double t[NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                if (SS_V(f, e) == SS_V(f, e) && !(SUR && ((gone[f] >> e) & 1u)))
                    add_member(t, double(SS_W(e)), double(SS_V(f, e)) - Kn, 0.0);
            block_sum<NSUM, BLOCK>(t, part, tot);
            if (tid == 0) {
                t[S_N] = rint(t[S_N]);
#pragma unroll
                for (int q = 0; q < NSUM; ++q) state[f][q] = t[q];
                PassCtl c = ctl[f];
                c.K = Kn;
                plan(a, t, c, k, false);
                ctl[f] = c;
            }
            __syncthreads();
            bnd_f[f] = ctl[f].bounds;
            go_f[f] = ctl[f].go;
        }
        // running sums of the removed members of the frames this wave
        // finishes (frames wid, wid + NW, ...), over the rounds of the pass
        double r[FPW][NREM];
        int n_removed[FPW];
#pragma unroll
        for (int j = 0; j < FPW; ++j) {
            n_removed[j] = 0;
#pragma unroll
            for (int q = 0; q < NREM; ++q) r[j][q] = 0.0;
        }
        for (;;) {
            int more = 0;
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                int used = 0;
                if (go_of(f)) {
                    const ClipBounds bnd = bnd_of(f);
#pragma unroll
                    for (int e = 0; e < EPT; ++e) {
                        const bool out = !(SUR && ((gone[f] >> e) & 1u)) && clipped(SS_V(f, e), bnd);
                        // the wave's mask straight from the two compares
                        // (2 = ordered greater, 4 = ordered less; NaN never
                        // compares), not a ballot of a materialised flag
                        const uint64_t m = SUR ? __builtin_amdgcn_ballot_w64(out)
                                               : (__builtin_amdgcn_fcmpf(SS_V(f, e), bnd.hi, 2) |
                                                  __builtin_amdgcn_fcmpf(SS_V(f, e), bnd.lo, 4));
                        if (m == 0) continue;
                        const int cnt = __popcll(m);
                        if (used + cnt > kRemCap) {
                            more = 1;  // this slot waits for the next round
                            continue;
                        }
                        if (out) {
                            rem_s[wid][f][used + lanes_below(m)] = make_float2(SS_W(e), SS_V(f, e));
                            if constexpr (SUR)
                                gone[f] |= uint64_t(1) << e;  // the value stays for the final check
                            else
                                SS_V(f, e) = __builtin_nanf("");
                        }
                        used = __builtin_amdgcn_readfirstlane(used + cnt);
                    }
                }
                if (lane == 0) cnt_s[wid][f] = used;
            }
            if (lane == 0) more_s[wid] = more;
            __syncthreads();
            int again = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) again |= more_s[w];
#pragma unroll
            for (int j = 0; j < FPW; ++j) {
                const int f = wid + j * NW;
                if (f >= FB || !go_of(f)) continue;
                const double Kc = ctl[f].K;
                // kListGroup lists at a time: their counts and this lane's
                // entries are read together (one LDS round trip), then added
                // in list order; a lane past a list's end adds zeros, which
                // leaves the sums exactly as they were
                constexpr int LG = NW < kListGroup ? NW : kListGroup;
                static_assert(NW % LG == 0, "whole groups of lists");
#pragma unroll 1
                for (int w0 = 0; w0 < NW; w0 += LG) {
                    int cnt[LG];
                    float2 x[LG];
#pragma unroll
                    for (int u = 0; u < LG; ++u) {
                        cnt[u] = cnt_s[w0 + u][f];
                        x[u] = rem_s[w0 + u][f][lane];
                    }
#pragma unroll
                    for (int u = 0; u < LG; ++u) {
                        n_removed[j] += cnt[u];
                        const bool in = lane < cnt[u];
                        add_removed(r[j], in ? double(x[u].x) : 0.0, in ? double(x[u].y) - Kc : 0.0);
                    }
                }
                if (again) continue;
                wave_sum_last_n(r[j]);
                if (lane == kWave - 1) {
                    double sv[NSUM];
                    load_state(state[f], sv);
                    sv[S_W] -= r[j][R_W];
                    sv[S_WD] -= r[j][R_WD];
                    sv[S_W2] -= r[j][R_W2];
                    sv[S_W2D] -= r[j][R_W2D];
                    sv[S_W2D2] -= r[j][R_W2D2];
                    sv[S_N] -= double(n_removed[j]);
#pragma unroll
                    for (int q = 0; q < NSUM; ++q) state[f][q] = sv[q];
                    PassCtl c = ctl[f];
                    after_pass(c, n_removed[j] > 0);
                    if (c.go) plan(a, sv, c, k + 1, true);
                    ctl[f] = c;
                }
            }
            __syncthreads();
            if (!again) break;
        }
    }
    if constexpr (SUR) {
        // a warm start is accepted only if no removed member lies within the
        // final bounds (the final set is exactly the members the final bounds keep)
        if (tid < FB) {
            double sv[NSUM];
            load_state(state[tid], sv);
            const Stats st = stats_from(sv, ctl[tid].K);
            sur_s[tid].fin = clip_bounds(st.mean, a.cutoff * st.std);
            sur_s[tid].back = 0;
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            if (!sur_s[f].warm) continue;
            const ClipBounds fin = sur_s[f].fin;
            bool back = false;
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                back = back || (((gone[f] >> e) & 1u) && !clipped(SS_V(f, e), fin));
            if (__ballot(back) != 0 && lane == 0) atomicOr(&sur_s[f].back, 1);
        }
        __syncthreads();
    }
    if (tid < nf) {
        const int64_t o = int64_t(f0 + tid) * a.n_bins + bin;
        if (a.redo == nullptr || a.redo[o] == -1) {
            double sv[NSUM];
            load_state(state[tid], sv);
            const Stats st = stats_from(sv, ctl[tid].K);
            write_profile(a, f0 + tid, bin, sv, st, ctl[tid].n_iter, ctl[tid].converged);
            if constexpr (SUR) {
                // accepted when the clip converged inside the predicted bounds, so pass 0
                // removed nothing the final bounds keep; else clipped again from scratch
                const Surrogate u = sur_s[tid];
                int state_out = 0;
                if (u.warm) {
                    const bool inside = st.mean - a.cutoff * st.std >= u.mean_hat - u.half &&
                                        st.mean + a.cutoff * st.std <= u.mean_hat + u.half;
                    state_out = (ctl[tid].converged && inside && !u.back) ? 1 : -1;
                }
                a.accepted[o] = state_out;
            }
        }
    }
#undef SS_W
}

template <int BLOCK, int EPT, int FB, int WPE, int MODE, bool WLDS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_clip_regs(ClipArgs a) {
    int g, bin;
    if (!block_item(a, FB, g, bin)) return;
    clip_body<BLOCK, EPT, FB, MODE, WLDS>(a, g, bin);
}

// Several batches, each with its own geometry, in one launch per row-length
// class: the items (frame group, bin) of every batch's bins of the class,
// batch after batch, mapped to work-groups as block_item does.
constexpr int kMaxJobs = 8;

struct MultiArgs {
    int32_t n_jobs;
    uint32_t base[kMaxJobs + 1];  // first item of each batch; base[n_jobs] = all items
    ClipArgs job[kMaxJobs];
};

template <int BLOCK, int EPT, int FB, int WPE, bool WLDS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_clip_regs_multi(MultiArgs m) {
    const uint32_t total = m.base[m.n_jobs];
    const uint32_t per = (total + 7u) / 8u;
    const uint32_t gb = blockIdx.x;
    const uint32_t item = (gb % 8u) * per + gb / 8u;
    if (gb / 8u >= per || item >= total) return;
    int j = 0;
    while (j + 1 < m.n_jobs && item >= m.base[j + 1]) ++j;
    const ClipArgs &a = m.job[j];
    const uint32_t local = item - m.base[j];
    const uint32_t nb = uint32_t(a.launch_bins);
    const int bin = a.bin_order ? a.bin_order[a.order_base + int(local % nb)] : int(local % nb);
    if (uint32_t(bin) >= uint32_t(a.n_bins)) return;
    clip_body<BLOCK, EPT, FB, MODE_CLIP, WLDS>(a, int(local / nb), bin);
}
#undef SS_V

// ---------------------------------------------------------------------------

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_clip_stream(ClipArgs a) {
    constexpr int NW = BLOCK / kWave;
    __shared__ double part[NSUM * NW];
    __shared__ double tot[NSUM];
    __shared__ ClipBounds hist[SS_MAX_ITER];

    int f, bin;
    if (!block_item(a, 1, f, bin)) return;
    const int tid = threadIdx.x;
    int64_t start, end;
    row_bounds(a, bin, start, end);
    const float *__restrict__ fr = a.frames + int64_t(f) * a.n_pix;
    const bool need_pv = a.model != SS_AZIMUTHAL;

    double K = first_shift(a, fr, start, end);
    double s1[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t j = start + tid; j < end; j += BLOCK) {
        const int32_t idx = a.indices[j];
        const float wt = a.weight[j];
        const float x = gather(fr, idx, a.n_pix);
        if (member_ok(x, wt, a.mask, idx)) {
            const double wd = double(wt);
            s1[0] += wd;
            s1[1] += wd * (double(x) - K);
            s1[2] += wd * wd;
            s1[3] += 1.0;
        }
    }
    block_sum<4, BLOCK>(s1, part, tot);
    double s[NSUM] = {s1[0], 0.0, s1[2], 0.0, 0.0, 0.0, s1[3]};
    K = (s[S_N] > 0.5 && s[S_W] > 0.0) ? K + s1[1] / s[S_W] : 0.0;
    {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t j = start + tid; j < end; j += BLOCK) {
            const int32_t idx = a.indices[j];
            const float wt = a.weight[j];
            const float x = gather(fr, idx, a.n_pix);
            if (member_ok(x, wt, a.mask, idx)) {
                const double wd = double(wt);
                const double d = double(x) - K;
                const double w2 = wd * wd;
                t[0] += wd * d;
                t[1] += w2 * d;
                t[2] += w2 * d * d;
                if (need_pv) t[3] += w2 * poisson_var(x, a.norm ? a.norm[idx] : 1.0f, a.dark_var);
            }
        }
        block_sum<4, BLOCK>(t, part, tot);
        s[S_WD] = t[0];
        s[S_W2D] = t[1];
        s[S_W2D2] = t[2];
        s[S_PV] = t[3];
    }
    // every thread holds the same block-reduced sums and runs the same plan
    PassCtl c{0.0, 0.0, K, ClipBounds{0.0f, 0.0f}, 0, 0, 0, 0};
    plan(a, s, c, 0, false);
    for (int k = 0; c.go; ++k) {
        if (c.refresh) {
            // re-accumulate the surviving members around the current mean
            const double Kn = c.mean;
            double t[NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int64_t j = start + tid; j < end; j += BLOCK) {
                const int32_t idx = a.indices[j];
                const float wt = a.weight[j];
                const float x = gather(fr, idx, a.n_pix);
                if (!member_ok(x, wt, a.mask, idx)) continue;
                bool alive = true;
                for (int q = 0; q < k && alive; ++q) alive = !clipped(x, hist[q]);
                if (alive) {
                    const double pv = need_pv ? poisson_var(x, a.norm ? a.norm[idx] : 1.0f, a.dark_var) : 0.0;
                    add_member(t, double(wt), double(x) - Kn, pv);
                }
            }
            block_sum<NSUM, BLOCK>(t, part, tot);
#pragma unroll
            for (int q = 0; q < NSUM; ++q) s[q] = t[q];
            s[S_N] = rint(s[S_N]);
            c.K = Kn;
            plan(a, s, c, k, false);
            if (!c.go) break;
        }
        if (tid == 0) hist[k] = c.bounds;
        __syncthreads();
        double r[NSUM] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t j = start + tid; j < end; j += BLOCK) {
            const int32_t idx = a.indices[j];
            const float wt = a.weight[j];
            const float x = gather(fr, idx, a.n_pix);
            if (!member_ok(x, wt, a.mask, idx)) continue;
            bool alive = true;
            for (int q = 0; q < k && alive; ++q) alive = !clipped(x, hist[q]);
            if (alive && clipped(x, c.bounds)) {
                const double pv = need_pv ? poisson_var(x, a.norm ? a.norm[idx] : 1.0f, a.dark_var) : 0.0;
                add_member(r, double(wt), double(x) - c.K, pv);
            }
        }
        block_sum<NSUM, BLOCK>(r, part, tot);
#pragma unroll
        for (int q = 0; q < NSUM; ++q) s[q] -= r[q];
        s[S_N] = rint(s[S_N]);
        after_pass(c, r[S_N] >= 0.5);
        if (c.go) plan(a, s, c, k + 1, true);
    }
    if (tid == 0) write_profile(a, f, bin, s, stats_from(s, c.K), c.n_iter, c.converged);
}

// ---------------------------------------------------------------------------

template <int BLOCK, int EPT, int FB, int WPE, int MODE, bool WLDS>
void launch_regs(const ClipArgs &a, hipStream_t stream) {
    const int64_t groups = (int64_t(a.n_frames) + FB - 1) / FB;
    k_clip_regs<BLOCK, EPT, FB, WPE, MODE, WLDS><<<dim3(item_grid(groups * a.launch_bins)), BLOCK, 0, stream>>>(a);
}

template <int BLOCK>
void launch_stream(const ClipArgs &a, hipStream_t stream) {
    k_clip_stream<BLOCK><<<dim3(item_grid(int64_t(a.n_frames) * a.launch_bins)), BLOCK, 0, stream>>>(a);
}

// Shapes of the register kernel: threads, values per thread, frames per
// work-group, waves per SIMD the register budget is set for, and whether the
// weights sit in LDS.  Per row-length class (rows up to ss_class_rows(c)):
// variant 0 is the default for batches, 1 and 2 the alternatives the
// autotuner may pick (plain clip of batches only); single frames use the
// SINGLE shape.  Measured on gfx950: more independent work-groups per CU
// hide the gather latency better than more frames per work-group.
//   class  rows     variant 0        variant 1        variant 2
//   0      1024     128 x 8,  2 fr   256 x 4,  4 fr   256 x 4,  2 fr
//   1      2048     128 x 16, 2 fr   256 x 8,  4 fr   256 x 8,  2 fr
//   2      4096     256 x 16, 2 fr   128 x 32, 1 fr   256 x 16, 1 fr
//   3      8192     256 x 32, 1 fr   512 x 16, 2 fr   1024 x 8, 4 fr
//   4      16384    512 x 32, 1 fr   1024 x 16, 2 fr  512 x 32, 2 fr
//   5      24576    1024 x 24, 2 fr  1024 x 24, 1 fr  512 x 48, 1 fr
//   6      51200    1024 x 50, 1 fr, weights read again from memory
//   7      longer   the streaming kernel

template <int ROWS, int BLOCK, int EPT, int FB, int WPE, bool WLDS = true>
void launch_shape(const ClipArgs &a, int mode, hipStream_t stream) {
    static_assert(BLOCK * EPT >= ROWS, "a work-group holds the longest row of its class");
    switch (mode) {
        case MODE_FEATURES: launch_regs<BLOCK, EPT, FB, WPE, MODE_FEATURES, WLDS>(a, stream); break;
        case MODE_SURROGATE: launch_regs<BLOCK, EPT, FB, WPE, MODE_SURROGATE, WLDS>(a, stream); break;
        case MODE_WARM: launch_regs<BLOCK, EPT, FB, WPE, MODE_WARM, WLDS>(a, stream); break;
        default: launch_regs<BLOCK, EPT, FB, WPE, MODE_CLIP, WLDS>(a, stream); break;
    }
}

template <int ROWS, int BLOCK, int EPT, int FB, int WPE, bool WLDS = true>
void launch_plain(const ClipArgs &a, hipStream_t stream) {
    static_assert(BLOCK * EPT >= ROWS, "a work-group holds the longest row of its class");
    launch_regs<BLOCK, EPT, FB, WPE, MODE_CLIP, WLDS>(a, stream);
}

// (the surrogate modes use variant 0 of classes 0-5 only; the surrogate
// entry points refuse longer rows before launching)
void launch_class(const ClipArgs &a, int c, int variant, int mode, hipStream_t stream) {
    const bool batch = a.n_frames > 1;
    if (c == 6) {
        launch_plain<51200, 1024, 50, 1, 4, false>(a, stream);
        return;
    }
    if (c > 6) {
        launch_stream<1024>(a, stream);
        return;
    }
    if (!batch) {
        switch (c) {
            case 0: launch_shape<1024, 256, 4, 1, 5>(a, mode, stream); break;
            case 1: launch_shape<2048, 256, 8, 1, 5>(a, mode, stream); break;
            case 2: launch_shape<4096, 128, 32, 1, 4>(a, mode, stream); break;
            case 3: launch_shape<8192, 256, 32, 1, 4>(a, mode, stream); break;
            case 4: launch_shape<16384, 512, 32, 1, 4>(a, mode, stream); break;
            default: launch_shape<24576, 1024, 24, 1, 4>(a, mode, stream); break;
        }
        return;
    }
    if (mode != MODE_CLIP || variant < 0 || variant > 2) variant = 0;
    switch (c * 3 + variant) {
        case 0: launch_shape<1024, 128, 8, 2, 4>(a, mode, stream); break;
        case 1: launch_plain<1024, 256, 4, 4, 4>(a, stream); break;
        case 2: launch_plain<1024, 256, 4, 2, 4>(a, stream); break;
        case 3: launch_shape<2048, 128, 16, 2, 4>(a, mode, stream); break;
        case 4: launch_plain<2048, 256, 8, 4, 4>(a, stream); break;
        case 5: launch_plain<2048, 256, 8, 2, 4>(a, stream); break;
        case 6: launch_shape<4096, 256, 16, 2, 4>(a, mode, stream); break;
        case 7: launch_plain<4096, 128, 32, 1, 4>(a, stream); break;
        case 8: launch_plain<4096, 256, 16, 1, 5>(a, stream); break;
        case 9: launch_shape<8192, 256, 32, 1, 4>(a, mode, stream); break;
        case 10: launch_plain<8192, 512, 16, 2, 4>(a, stream); break;
        case 11: launch_plain<8192, 1024, 8, 4, 4>(a, stream); break;
        case 12: launch_shape<16384, 512, 32, 1, 4>(a, mode, stream); break;
        case 13: launch_plain<16384, 1024, 16, 2, 4>(a, stream); break;
        case 14: launch_plain<16384, 512, 32, 2, 2>(a, stream); break;
        case 15: launch_shape<24576, 1024, 24, 2, 4>(a, mode, stream); break;
        case 16: launch_plain<24576, 1024, 24, 1, 4>(a, stream); break;
        default: launch_plain<24576, 512, 48, 1, 2>(a, stream); break;
    }
}

// One launch per class over several batches (plain clip, batches of > 1 frame).
template <int ROWS, int BLOCK, int EPT, int FB, int WPE, bool WLDS = true>
void launch_multi(MultiArgs &m, hipStream_t stream) {
    static_assert(BLOCK * EPT >= ROWS, "a work-group holds the longest row of its class");
    m.base[0] = 0;
    for (int j = 0; j < m.n_jobs; ++j) {
        const int64_t groups = (int64_t(m.job[j].n_frames) + FB - 1) / FB;
        m.base[j + 1] = m.base[j] + uint32_t(groups * m.job[j].launch_bins);
    }
    if (m.base[m.n_jobs] == 0) return;
    k_clip_regs_multi<BLOCK, EPT, FB, WPE, WLDS><<<dim3(item_grid(m.base[m.n_jobs])), BLOCK, 0, stream>>>(m);
}

void launch_class_multi(MultiArgs &m, int c, int variant, hipStream_t stream) {
    if (variant < 0 || variant > 2) variant = 0;
    if (c == 6) {
        launch_multi<51200, 1024, 50, 1, 4, false>(m, stream);
        return;
    }
    switch (c * 3 + variant) {
        case 0: launch_multi<1024, 128, 8, 2, 4>(m, stream); break;
        case 1: launch_multi<1024, 256, 4, 4, 4>(m, stream); break;
        case 2: launch_multi<1024, 256, 4, 2, 4>(m, stream); break;
        case 3: launch_multi<2048, 128, 16, 2, 4>(m, stream); break;
        case 4: launch_multi<2048, 256, 8, 4, 4>(m, stream); break;
        case 5: launch_multi<2048, 256, 8, 2, 4>(m, stream); break;
        case 6: launch_multi<4096, 256, 16, 2, 4>(m, stream); break;
        case 7: launch_multi<4096, 128, 32, 1, 4>(m, stream); break;
        case 8: launch_multi<4096, 256, 16, 1, 5>(m, stream); break;
        case 9: launch_multi<8192, 256, 32, 1, 4>(m, stream); break;
        case 10: launch_multi<8192, 512, 16, 2, 4>(m, stream); break;
        case 11: launch_multi<8192, 1024, 8, 4, 4>(m, stream); break;
        case 12: launch_multi<16384, 512, 32, 1, 4>(m, stream); break;
        case 13: launch_multi<16384, 1024, 16, 2, 4>(m, stream); break;
        case 14: launch_multi<16384, 512, 32, 2, 2>(m, stream); break;
        case 15: launch_multi<24576, 1024, 24, 2, 4>(m, stream); break;
        case 16: launch_multi<24576, 1024, 24, 1, 4>(m, stream); break;
        default: launch_multi<24576, 512, 48, 1, 2>(m, stream); break;
    }
}

int class_of(int32_t rows) {
    int c = 0;
    while (c < SS_N_CLASSES - 1 && rows > ss_class_rows(c)) ++c;
    return c;
}

// One launch per row-length class when the CSR carries a schedule (register
// kernels sized to the class); otherwise one launch sized to the longest
// row.  The Poisson and hybrid models and an extra mask take the streaming
// kernel.
// Side streams for small batches.  The row-length classes of one call are
// independent, and with one or two frames each class launch holds too few
// work-groups to fill the device, so their launches run side by side: the
// caller's stream forks to up to kSide side streams through an event and
// joins them through one event each (default priority; capturable in a
// graph).  Created once per device; the enqueue sequence is serialised by a
// mutex, and each wait takes the event's state at the time it is enqueued,
// so the events are reused.
constexpr int kSide = 3;
constexpr int kSideMaxFrames = 2;
constexpr int kMaxDevices = 64;

struct SideStreams {
    bool ok = false, failed = false;
    hipStream_t s[kSide];
    hipEvent_t fork, join[kSide];
};

std::mutex g_side_mu;
SideStreams g_side[kMaxDevices];

SideStreams *side_streams_locked() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    SideStreams &ss = g_side[dev];
    if (ss.ok) return &ss;
    if (ss.failed) return nullptr;
    bool good = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kSide && good; ++i)
        good = hipStreamCreateWithFlags(&ss.s[i], hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&ss.join[i], hipEventDisableTiming) == hipSuccess;
    ss.ok = good;
    ss.failed = !good;
    if (!good) (void)hipGetLastError();  // fall back to one stream; clear the error
    return good ? &ss : nullptr;
}

void dispatch(ClipArgs a, const ss_csr *csr, int n_frames, int mode, hipStream_t stream) {
    const bool regs = a.model == SS_AZIMUTHAL && a.mask == nullptr && a.n_pix < (int64_t(1) << 30);
    if (!regs) {
        a.bin_order = nullptr;
        a.order_base = 0;
        a.launch_bins = a.n_bins;
        if (csr->max_row <= 4096) launch_stream<256>(a, stream);
        else launch_stream<1024>(a, stream);
        return;
    }
    if (csr->bin_order == nullptr) {
        a.bin_order = nullptr;
        a.order_base = 0;
        a.launch_bins = a.n_bins;
        const int c = class_of(csr->max_row);
        launch_class(a, c, csr->shape[c], mode, stream);
        return;
    }
    int classes = 0;
    for (int c = 0; c < SS_N_CLASSES; ++c) classes += csr->class_count[c] > 0 ? 1 : 0;
    std::unique_lock<std::mutex> lock(g_side_mu, std::defer_lock);
    SideStreams *side = nullptr;
    if (n_frames <= kSideMaxFrames && classes > 1) {
        lock.lock();
        side = side_streams_locked();
        if (side) {
            (void)hipEventRecord(side->fork, stream);
            for (int i = 0; i < kSide; ++i) (void)hipStreamWaitEvent(side->s[i], side->fork, 0);
        } else {
            lock.unlock();
        }
    }
    int32_t base = 0;
    int q = 0;
    for (int c = SS_N_CLASSES - 1; c >= 0; --c) {
        const int32_t cnt = csr->class_count[c];
        if (cnt <= 0) continue;
        a.bin_order = csr->bin_order;
        a.order_base = base;
        a.launch_bins = cnt;
        // longest class on the caller's stream, the others spread over the side streams
        const hipStream_t target = (side && q > 0) ? side->s[(q - 1) % kSide] : stream;
        launch_class(a, c, csr->shape[c], mode, target);
        base += cnt;
        ++q;
    }
    if (side) {
        for (int i = 0; i < kSide; ++i) {
            (void)hipEventRecord(side->join[i], side->s[i]);
            (void)hipStreamWaitEvent(stream, side->join[i], 0);
        }
    }
}

}  // namespace
}  // namespace ss

namespace {

struct SurrogateIo {
    int mode = ss::MODE_CLIP;
    float *features = nullptr;
    double *stats0 = nullptr;
    const uint16_t *w16 = nullptr;
    float widen = 0.0f;
    int32_t *accepted = nullptr;
    const double *pred_mean = nullptr;
    const double *pred_std = nullptr;
};

// Checks one call's arguments and fills the kernel arguments; returns an
// error code, or SS_OK with `empty` set when there is nothing to launch.
int clip_args(const float *frames, const float *norm, const uint8_t *mask, int32_t n_frames, const ss_csr *csr,
              const ss_params *p, const ss_profile *out, bool integrate_only, const SurrogateIo &io, ss::ClipArgs &a,
              bool &empty) {
    empty = true;
    const bool features = io.mode == ss::MODE_FEATURES;
    if (!csr || !p || (!features && !out)) return SS_EINVAL;
    if (n_frames < 0) return SS_ESIZE;
    if (csr->n_bins <= 0 || csr->n_bins > SS_MAX_BINS || csr->n_pix < 0 ||
        csr->n_pix >= (int64_t(1) << 31) || csr->nnz < 0 || csr->nnz >= (int64_t(1) << 31) ||
        csr->max_row < 0)
        return SS_ESIZE;
    if (!integrate_only && (p->max_iter < 0 || p->max_iter > SS_MAX_ITER)) return SS_ESIZE;
    if (p->error_model != SS_AZIMUTHAL && p->error_model != SS_POISSON && p->error_model != SS_HYBRID)
        return SS_EINVAL;
    if (io.mode != ss::MODE_CLIP) {
        // the surrogate runs in the register kernel only
        if (mask || csr->max_row > ss_class_rows(SS_SURROGATE_MAX_CLASS) || csr->n_pix >= (int64_t(1) << 30))
            return SS_EINVAL;
        if (features && (!io.features || !io.stats0)) return SS_EINVAL;
        if (io.mode == ss::MODE_SURROGATE &&
            (p->error_model != SS_AZIMUTHAL || !(p->cutoff > 0.0f) || !io.w16 ||
             (reinterpret_cast<uintptr_t>(io.w16) & 15u) != 0 || !(io.widen >= 0.0f) || !io.accepted))
            return SS_EINVAL;
        if (io.mode == ss::MODE_WARM &&
            (p->error_model != SS_AZIMUTHAL || !(p->cutoff > 0.0f) || !io.pred_mean || !io.pred_std ||
             !(io.widen >= 0.0f) || !io.accepted))
            return SS_EINVAL;
    }
    if (n_frames == 0) return SS_OK;
    empty = false;
    if (csr->n_pix == 0 && csr->nnz > 0) return SS_ESIZE;
    if (!frames || !csr->indptr || (csr->nnz > 0 && (!csr->indices || !csr->weight)))
        return SS_EINVAL;
    if (!features && (!out->mean || !out->std || !out->sem || !out->sum_w || !out->n_members || !out->n_iter ||
                      !out->converged))
        return SS_EINVAL;
    const int64_t items = int64_t(csr->n_bins) * n_frames;
    if (items >= (int64_t(1) << 31) - 8) return SS_ESIZE;
    a = ss::ClipArgs{};
    a.frames = frames;
    a.n_pix = csr->n_pix;
    a.norm = norm;
    a.mask = mask;
    a.n_frames = n_frames;
    a.n_bins = csr->n_bins;
    a.indptr = csr->indptr;
    a.indices = csr->indices;
    a.weight = csr->weight;
    a.nnz = csr->nnz;
    a.bin_order = nullptr;
    a.order_base = 0;
    a.launch_bins = csr->n_bins;
    a.cutoff = double(p->cutoff);
    a.max_iter = integrate_only ? 0 : p->max_iter;
    a.model = p->error_model;
    a.dark_var = double(p->dark_var);
    if (!features) {
        a.mean = out->mean;
        a.std = out->std;
        a.sem = out->sem;
        a.sum_w = out->sum_w;
        a.n_members = out->n_members;
        a.n_iter = out->n_iter;
        a.converged = out->converged;
    }
    a.features = io.features;
    a.stats0 = io.stats0;
    a.w16 = io.w16;
    a.widen = double(io.widen);
    a.accepted = io.accepted;
    a.pred_mean = io.pred_mean;
    a.pred_std = io.pred_std;
    if (csr->bin_order) {
        int64_t sum = 0;
        for (int c = 0; c < SS_N_CLASSES; ++c) {
            if (csr->class_count[c] < 0) return SS_EINVAL;
            sum += csr->class_count[c];
        }
        if (sum != csr->n_bins) return SS_EINVAL;
        if (io.mode != ss::MODE_CLIP)
            for (int c = SS_SURROGATE_MAX_CLASS + 1; c < SS_N_CLASSES; ++c)
                if (csr->class_count[c] != 0) return SS_EINVAL;
    }
    return SS_OK;
}

int clip_entry(const float *frames, const float *norm, const uint8_t *mask, int32_t n_frames, const ss_csr *csr,
               const ss_params *p, const ss_profile *out, bool integrate_only, const SurrogateIo &io,
               hipStream_t stream) {
    ss::ClipArgs a;
    bool empty = true;
    const int rc = clip_args(frames, norm, mask, n_frames, csr, p, out, integrate_only, io, a, empty);
    if (rc != SS_OK || empty) return rc;
    ss::dispatch(a, csr, n_frames, io.mode, stream);
    if (io.mode == ss::MODE_SURROGATE || io.mode == ss::MODE_WARM) {
        // the groups holding a refused bin, clipped again from scratch
        a.redo = io.accepted;
        ss::dispatch(a, csr, n_frames, ss::MODE_CLIP, stream);
    }
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}

}  // namespace

extern "C" int ss_sigma_clip(const float *frames, const float *norm, const uint8_t *mask,
                             int32_t n_frames, const ss_csr *csr, const ss_params *params,
                             const ss_profile *out, hipStream_t stream) {
    return clip_entry(frames, norm, mask, n_frames, csr, params, out, false, SurrogateIo{}, stream);
}

extern "C" int ss_integrate_csr(const float *frames, const float *norm, const uint8_t *mask,
                                int32_t n_frames, const ss_csr *csr, const ss_params *params,
                                const ss_profile *out, hipStream_t stream) {
    return clip_entry(frames, norm, mask, n_frames, csr, params, out, true, SurrogateIo{}, stream);
}

extern "C" int ss_clip_features(const float *frames, const float *norm, const uint8_t *mask, int32_t n_frames,
                                const ss_csr *csr, float *features, double *stats0, hipStream_t stream) {
    ss_params p{};
    p.cutoff = 3.0f;
    p.max_iter = 0;
    p.error_model = SS_AZIMUTHAL;
    SurrogateIo io;
    io.mode = ss::MODE_FEATURES;
    io.features = features;
    io.stats0 = stats0;
    return clip_entry(frames, norm, mask, n_frames, csr, &p, nullptr, false, io, stream);
}

extern "C" int ss_sigma_clip_surrogate(const float *frames, const float *norm, const uint8_t *mask,
                                       int32_t n_frames, const ss_csr *csr, const ss_params *params,
                                       const uint16_t *w16, float widen, const ss_profile *out,
                                       int32_t *accepted, hipStream_t stream) {
    SurrogateIo io;
    io.mode = ss::MODE_SURROGATE;
    io.w16 = w16;
    io.widen = widen;
    io.accepted = accepted;
    return clip_entry(frames, norm, mask, n_frames, csr, params, out, false, io, stream);
}

extern "C" int ss_sigma_clip_warm(const float *frames, const float *norm, const uint8_t *mask, int32_t n_frames,
                                  const ss_csr *csr, const ss_params *params, const double *pred_mean,
                                  const double *pred_std, float widen, const ss_profile *out, int32_t *accepted,
                                  hipStream_t stream) {
    SurrogateIo io;
    io.mode = ss::MODE_WARM;
    io.pred_mean = pred_mean;
    io.pred_std = pred_std;
    io.widen = widen;
    io.accepted = accepted;
    return clip_entry(frames, norm, mask, n_frames, csr, params, out, false, io, stream);
}

extern "C" int ss_sigma_clip_batches(const ss_clip_batch *batches, int32_t n_batches, const ss_params *params,
                                     hipStream_t stream) {
    if (n_batches < 0) return SS_ESIZE;
    if (n_batches == 0) return SS_OK;
    if (!batches || !params) return SS_EINVAL;
    std::vector<ss::ClipArgs> args(static_cast<size_t>(n_batches));
    std::vector<char> shared(static_cast<size_t>(n_batches), 0);
    for (int32_t b = 0; b < n_batches; ++b) {
        const ss_clip_batch &x = batches[b];
        bool empty = true;
        const int rc = clip_args(x.frames, x.norm, nullptr, x.n_frames, x.csr, params, x.out, false, SurrogateIo{},
                                 args[size_t(b)], empty);
        if (rc != SS_OK) return rc;
        // shared launches: azimuthal model, scheduled CSR, batches of frames
        shared[size_t(b)] = !empty && params->error_model == SS_AZIMUTHAL && x.csr->bin_order != nullptr &&
                            x.n_frames > 1 && x.csr->n_pix < (int64_t(1) << 30);
    }
    const int32_t *shape = batches[0].csr->shape;
    for (int32_t b = 0; b < n_batches; ++b)
        if (!shared[size_t(b)] && batches[b].n_frames > 0)
            ss::dispatch(args[size_t(b)], batches[b].csr, batches[b].n_frames, ss::MODE_CLIP, stream);
    for (int c = SS_N_CLASSES - 1; c >= 0; --c) {
        ss::MultiArgs m{};
        auto flush = [&]() {
            if (m.n_jobs == 0) return;
            if (c == SS_N_CLASSES - 1) {
                for (int j = 0; j < m.n_jobs; ++j) ss::launch_stream<1024>(m.job[j], stream);
            } else {
                ss::launch_class_multi(m, c, shape[c], stream);
            }
            m.n_jobs = 0;
        };
        for (int32_t b = 0; b < n_batches; ++b) {
            if (!shared[size_t(b)]) continue;
            const ss_csr *csr = batches[b].csr;
            const int32_t cnt = csr->class_count[c];
            if (cnt <= 0) continue;
            int32_t base = 0;
            for (int c2 = SS_N_CLASSES - 1; c2 > c; --c2) base += csr->class_count[c2];
            ss::ClipArgs a = args[size_t(b)];
            a.bin_order = csr->bin_order;
            a.order_base = base;
            a.launch_bins = cnt;
            m.job[m.n_jobs++] = a;
            if (m.n_jobs == ss::kMaxJobs) flush();
        }
        flush();
    }
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
}
