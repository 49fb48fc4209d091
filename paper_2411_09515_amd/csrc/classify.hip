// Per-pixel classification against the clipped profile: sparsification
// (Sec. 3) and the peak finder (Sec. 4) in one pass over the pixels.
//
// k_profile_table (one work-group per frame) turns the per-bin profile into a
// lookup table over the n_bins + 1 intervals between bin centres: for each
// interval the bracketing non-empty bins and their mean/std, so that the
// background of a pixel is one table read plus a linear interpolation.  It
// also clears the look-back flags, the tile counter and the output counts.
//
// k_classify works on tiles of TILE consecutive pixels of one frame.  A tile
// classifies its pixels, runs the peak test for the (rare) candidates by
// reading their patch directly, and then appends its kept pixels and peaks
// in index order.  Ordering across tiles is a decoupled look-back: each tile
// publishes its counts, then adds up its predecessors' counts until it meets
// one that published an inclusive prefix.  Tiles take their id from an
// atomic counter, so a tile only ever waits on tiles whose work-groups are
// already running, and every wait ends.

#include <cmath>

#include "common.h"

namespace ss {
namespace {

constexpr int kBlock = 256;
constexpr int kPPT = 16;
constexpr int kTile = kBlock * kPPT;
constexpr int kNW = kBlock / kWave;
constexpr int kTableBlock = 256;

constexpr uint64_t kAggregate = uint64_t(1) << 62;
constexpr uint64_t kPrefix = uint64_t(2) << 62;
constexpr uint64_t kCountMask = kAggregate - 1;
constexpr int kPeakShift = 31;

struct Seg {
    double m_lo, dm, s_lo, ds, inv_span;
    int32_t lo, pad;
};

struct Workspace {
    uint32_t *counter;
    uint64_t *flags;  // [n_frames][tiles]
    Seg *table;       // [n_frames][n_bins + 1]
};

size_t tiles_of(int64_t n_pix) { return size_t((n_pix + kTile - 1) / kTile); }

size_t workspace_bytes(int32_t n_frames, int64_t n_pix, int32_t n_bins) {
    return 256 + size_t(n_frames) * tiles_of(n_pix) * sizeof(uint64_t) +
           size_t(n_frames) * size_t(n_bins + 1) * sizeof(Seg) + 256;
}

Workspace carve(void *base, int32_t n_frames, int64_t n_pix) {
    char *p = static_cast<char *>(base);
    Workspace w;
    w.counter = reinterpret_cast<uint32_t *>(p);
    p += 256;
    w.flags = reinterpret_cast<uint64_t *>(p);
    p += size_t(n_frames) * tiles_of(n_pix) * sizeof(uint64_t);
    uintptr_t q = (reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255);
    w.table = reinterpret_cast<Seg *>(q);
    return w;
}

// ---- table ---------------------------------------------------------------

__global__ __launch_bounds__(kTableBlock) void k_profile_table(
    const double *__restrict__ mean, const double *__restrict__ stdv, const int32_t *__restrict__ members,
    int32_t n_bins, Workspace ws, int32_t tiles, int64_t *n_kept, int64_t *n_peaks) {
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
    __syncthreads();
    if (tid == 0) {
        int best = -1;
        for (int c = 0; c < kTableBlock; ++c) {
            const int here = chunk_lo[c];
            chunk_lo[c] = best;  // exclusive prefix max
            if (here > best) best = here;
        }
        best = n_bins;
        for (int c = kTableBlock - 1; c >= 0; --c) {
            const int here = chunk_hi[c];
            chunk_hi[c] = best;  // exclusive suffix min
            if (here < best) best = here;
        }
    }
    __syncthreads();
    for (int r = a0; r < a1; ++r) {
        if (lo_s[r] < 0) lo_s[r] = chunk_lo[tid];
        if (hi_s[r] >= n_bins) hi_s[r] = chunk_hi[tid];
    }
    __syncthreads();

    // interval t (stored at t + 1) lies between centres t and t + 1
    Seg *tab = ws.table + int64_t(f) * (n_bins + 1);
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
    }
    uint64_t *fl = ws.flags + int64_t(f) * tiles;
    for (int i = tid; i < tiles; i += kTableBlock) fl[i] = 0;
    if (tid == 0) {
        if (n_kept) n_kept[f] = 0;
        if (n_peaks) n_peaks[f] = 0;
        if (f == 0) *ws.counter = 0;
    }
}

// ---- classification ----------------------------------------------------------

struct ClassArgs {
    const float *frames;
    const uint8_t *mask;
    const uint32_t *rcoord;
    int64_t n_pix;
    int32_t height, width;
    int32_t n_bins;
    int32_t tiles;
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

__device__ inline void background(uint32_t rc, const Seg *__restrict__ tab, int n_bins, double noise2,
                                  double &mu, double &se) {
    const int t1 = min(int(rc >> SS_RC_FRAC_BITS), n_bins);
    const double frac = double(rc & ((1u << SS_RC_FRAC_BITS) - 1u)) * (1.0 / double(1u << SS_RC_FRAC_BITS));
    const Seg s = tab[t1];
    const double u = (double(t1 - 1 - s.lo) + frac) * s.inv_span;
    mu = s.m_lo + s.dm * u;
    const double sd = s.s_lo + s.ds * u;
    se = sqrt(sd * sd + noise2);
}

__device__ inline bool pixel_valid(float x, uint32_t rc, const uint8_t *mask, int64_t i) {
    return rc != SS_RC_MASKED && isfinite(x) && !(mask && mask[i]);
}

struct PeakSums {
    int count;
    double I, s2, sy, sx;
};

// Patch test of Sec. 4 for candidate pixel i.  Returns whether i is a peak;
// with `full` the record sums are complete, otherwise the walk may stop as
// soon as i is beaten.
__device__ bool patch_eval(const ClassArgs &a, const float *__restrict__ fr, const Seg *__restrict__ tab,
                           int64_t i, double vi, bool full, PeakSums &ps) {
    const int y = int(i / a.width);
    const int x = int(i - int64_t(y) * a.width);
    const int y0 = max(0, y - a.half), y1 = min(a.height - 1, y + a.half);
    const int x0 = max(0, x - a.half), x1 = min(a.width - 1, x + a.half);
    bool is_max = true;
    ps = PeakSums{0, 0.0, 0.0, 0.0, 0.0};
    for (int yy = y0; yy <= y1; ++yy) {
        for (int xx = x0; xx <= x1; ++xx) {
            const int64_t j = int64_t(yy) * a.width + xx;
            const float xj = fr[j];
            const uint32_t rcj = a.rcoord[j];
            if (!pixel_valid(xj, rcj, a.mask, j)) continue;
            const double vj = double(xj);
            if (j != i && (vj > vi || (vj == vi && j < i))) {
                is_max = false;
                if (!full) return false;
            }
            double mu, se;
            background(rcj, tab, a.n_bins, a.noise2, mu, se);
            const double d = vj - mu;
            if (d >= a.snr * se) {
                ps.count += 1;
                ps.I += d;
                ps.s2 += se * se;
                ps.sy += d * (double(yy) + 0.5);
                ps.sx += d * (double(xx) + 0.5);
            }
        }
    }
    return is_max && ps.count >= a.min_count;
}

__device__ inline uint64_t load_flag(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void store_flag(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish this tile's packed counts and return the exclusive prefix.
__device__ uint64_t look_back(uint64_t *fl, int tile, uint64_t agg) {
    if (tile == 0) {
        store_flag(fl, kPrefix | agg);
        return 0;
    }
    store_flag(fl + tile, kAggregate | agg);
    uint64_t excl = 0;
    for (int p = tile - 1;; --p) {
        uint64_t w = load_flag(fl + p);
        while ((w >> 62) == 0) {
            __builtin_amdgcn_s_sleep(1);
            w = load_flag(fl + p);
        }
        excl += w & kCountMask;
        if ((w >> 62) == 2) break;
    }
    store_flag(fl + tile, kPrefix | (excl + agg));
    return excl;
}

template <bool KEEP, bool PEAKS>
__global__ __launch_bounds__(kBlock) void k_classify(ClassArgs a) {
    __shared__ uint32_t tile_s;
    __shared__ int cnt_k[kPPT * kNW];
    __shared__ int cnt_p[kPPT * kNW];
    __shared__ uint64_t excl_s;

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    if (tid == 0) tile_s = atomicAdd(a.ws.counter, 1u);
    __syncthreads();
    const uint32_t g = tile_s;
    const int f = int(g / uint32_t(a.tiles));
    const int tile = int(g % uint32_t(a.tiles));
    const int64_t base = int64_t(tile) * kTile;
    const float *__restrict__ fr = a.frames + int64_t(f) * a.n_pix;
    const Seg *__restrict__ tab = a.ws.table + int64_t(f) * (a.n_bins + 1);

    float val[kPPT];
    uint32_t kbits = 0, pbits = 0;
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        const int64_t i = base + int64_t(k) * kBlock + tid;
        bool keep = false, peak = false;
        val[k] = 0.0f;
        if (i < a.n_pix) {
            const float x = fr[i];
            const uint32_t rc = a.rcoord[i];
            if (pixel_valid(x, rc, a.mask, i)) {
                double mu, se;
                background(rc, tab, a.n_bins, a.noise2, mu, se);
                const double d = double(x) - mu;
                val[k] = x;
                keep = KEEP && d > a.n_pick * se;
                if (PEAKS && d >= a.snr * se) {
                    PeakSums ps;
                    peak = patch_eval(a, fr, tab, i, double(x), false, ps);
                }
            }
        }
        kbits |= uint32_t(keep) << k;
        pbits |= uint32_t(peak) << k;
        const uint64_t km = __ballot(keep);
        const uint64_t pm = __ballot(peak);
        if (lane == 0) {
            cnt_k[k * kNW + wid] = __popcll(km);
            cnt_p[k * kNW + wid] = __popcll(pm);
        }
    }
    __syncthreads();

    // exclusive scan of the (pass, wave) counts in pixel order: one wave,
    // one slot per lane (kPPT * kNW == 64)
    static_assert(kPPT * kNW == kWave, "one scan slot per lane");
    if (wid == 0) {
        const int ck = cnt_k[lane], cp = cnt_p[lane];
        int sk = ck, sp = cp;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int tk = __shfl_up(sk, off, kWave);
            const int tp = __shfl_up(sp, off, kWave);
            if (lane >= off) {
                sk += tk;
                sp += tp;
            }
        }
        cnt_k[lane] = sk - ck;
        cnt_p[lane] = sp - cp;
        const int tot_k = __shfl(sk, kWave - 1, kWave);
        const int tot_p = __shfl(sp, kWave - 1, kWave);
        if (lane == 0) {
            const uint64_t agg = uint64_t(tot_k) | (uint64_t(tot_p) << kPeakShift);
            const uint64_t excl = look_back(a.ws.flags + int64_t(f) * a.tiles, tile, agg);
            excl_s = excl;
            if (tile == a.tiles - 1) {
                const uint64_t total = excl + agg;
                if (KEEP) a.n_kept[f] = int64_t(total & ((uint64_t(1) << kPeakShift) - 1));
                if (PEAKS) a.n_peaks[f] = int64_t((total & kCountMask) >> kPeakShift);
            }
        }
    }
    __syncthreads();
    const uint64_t excl = excl_s;
    const int64_t excl_k = int64_t(excl & ((uint64_t(1) << kPeakShift) - 1));
    const int64_t excl_p = int64_t((excl & kCountMask) >> kPeakShift);

#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        const bool keep = (kbits >> k) & 1u;
        const bool peak = (pbits >> k) & 1u;
        const uint64_t km = __ballot(keep);
        const uint64_t pm = __ballot(peak);
        const int64_t i = base + int64_t(k) * kBlock + tid;
        if (KEEP && keep) {
            const int64_t pos = excl_k + cnt_k[k * kNW + wid] + lanes_below(km);
            if (pos < a.capacity) {
                a.kept_index[int64_t(f) * a.capacity + pos] = uint32_t(i);
                a.kept_value[int64_t(f) * a.capacity + pos] = val[k];
            }
        }
        if (PEAKS && peak) {
            const int64_t pos = excl_p + cnt_p[k * kNW + wid] + lanes_below(pm);
            if (pos < a.peak_capacity) {
                PeakSums ps;
                patch_eval(a, fr, tab, i, double(val[k]), true, ps);
                ss_peak rec;
                rec.index = uint32_t(i);
                rec.y = float(ps.sy / ps.I);
                rec.x = float(ps.sx / ps.I);
                rec.intensity = float(ps.I);
                rec.sigma = float(sqrt(ps.s2));
                a.peaks[int64_t(f) * a.peak_capacity + pos] = rec;
            }
        }
    }
}

}  // namespace
}  // namespace ss

extern "C" size_t ss_classify_workspace(int32_t n_frames, int64_t n_pix, int32_t n_bins) {
    if (n_frames < 0 || n_pix < 0 || n_bins < 0) return 0;
    return ss::workspace_bytes(n_frames, n_pix, n_bins);
}

extern "C" int ss_classify(const float *frames, const uint8_t *mask, int32_t n_frames, int32_t height,
                           int32_t width, const ss_radial *radial, const ss_profile *profile,
                           const ss_params *p, uint32_t *kept_index, float *kept_value, int64_t capacity,
                           int64_t *n_kept, ss_peak *peaks, int64_t peak_capacity, int64_t *n_peaks,
                           void *workspace, size_t ws_bytes, hipStream_t stream) {
    using namespace ss;
    if (!radial || !profile || !p) return SS_EINVAL;
    if (n_frames < 0 || height < 0 || width < 0 || capacity < 0 || peak_capacity < 0) return SS_ESIZE;
    const int64_t n_pix = int64_t(height) * width;
    if (n_pix >= (int64_t(1) << 31) || int64_t(n_frames) * int64_t(tiles_of(n_pix)) >= (int64_t(1) << 32))
        return SS_ESIZE;
    if (radial->n_bins <= 0 || radial->n_bins > SS_MAX_BINS) return SS_ESIZE;
    if (p->patch < 1 || p->patch > SS_MAX_PATCH || (p->patch % 2) == 0) return SS_EINVAL;
    const bool keep = kept_index || kept_value || n_kept;
    const bool pk = peaks || n_peaks;
    if (keep && (!kept_index || !kept_value || !n_kept)) return SS_EINVAL;
    if (pk && (!peaks || !n_peaks)) return SS_EINVAL;
    if (n_frames == 0 || (!keep && !pk)) return SS_OK;
    if (!frames || !radial->rcoord || !profile->mean || !profile->std || !profile->n_members || !workspace)
        return SS_EINVAL;
    if (ws_bytes < workspace_bytes(n_frames, n_pix, radial->n_bins)) return SS_ESIZE;

    const int32_t tiles = int32_t(tiles_of(n_pix));
    Workspace ws = carve(workspace, n_frames, n_pix);
    k_profile_table<<<dim3(uint32_t(n_frames)), kTableBlock, 0, stream>>>(
        profile->mean, profile->std, profile->n_members, radial->n_bins, ws, tiles, keep ? n_kept : nullptr,
        pk ? n_peaks : nullptr);
    SS_RETURN_IF_LAUNCH_FAILED();
    if (tiles == 0) return SS_OK;

    ClassArgs a;
    a.frames = frames;
    a.mask = mask;
    a.rcoord = radial->rcoord;
    a.n_pix = n_pix;
    a.height = height;
    a.width = width;
    a.n_bins = radial->n_bins;
    a.tiles = tiles;
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
    const dim3 grid(uint32_t(int64_t(tiles) * n_frames));
    if (keep && pk) k_classify<true, true><<<grid, kBlock, 0, stream>>>(a);
    else if (keep) k_classify<true, false><<<grid, kBlock, 0, stream>>>(a);
    else k_classify<false, true><<<grid, kBlock, 0, stream>>>(a);
    SS_RETURN_IF_LAUNCH_FAILED();
    return SS_OK;
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
