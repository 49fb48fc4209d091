"""Per-pixel classification: sparsification, densification, peak finding (FP64).

Background at a pixel (reading of Sec. 3, which stores the background
profile together with "the distance to the centre of every pixel"): the
mean and std of the clipped profile, linearly interpolated in 2theta between
the centres of the non-empty bins at the pixel-centre angle, held constant
beyond the first and last non-empty bins (``numpy.interp``).  The same
mu_i, sigma_i serve sparsification, densification and the peak finder.
sigma_eff = sqrt(sigma^2 + noise^2), with the noise level of Sec. 4.1.

Every decision is taken on the corrected intensity v = signal / norm of
eq. norm, the units of the stored profile, formed in float64: a frame is
either the float32 signal with its ``norm`` (then v = signal / norm), or,
with ``norm=None``, already in those units (norm = 1).  Kept values and peak
intensities are in units of v; the stored sparse format holds a kept value
as float32 (the rounding of v).

Sparsification (Sec. 3): keep pixel i when it is valid (not masked, finite)
and v_i - mu_i > n_pick * sigma_eff_i (strict, one-sided: low outliers are
shadows or dead pixels, not signal).  Output is (pixel index, v) in ascending
index order.  Densification (Sec. 3.2), noise free: kept pixels get their
stored value, other valid pixels mu_i, masked pixels 0.

Peak finder (Sec. 4).  Readings:
* candidate: valid and v - mu >= snr * sigma_eff;
* pixel i is a peak when it is a candidate, it is the maximum of v over the
  valid pixels of the P x P patch centred on it (clipped at the frame
  border; ties go to the lowest row-major index), and at least
  ``min_count`` candidates (the centre included) lie in that patch;
* record (the "centroid, sum of data and propagated deviation"): over the
  candidate pixels j of the patch, w_j = v_j - mu_j; I = sum w_j;
  sigma_I = sqrt(sum sigma_eff_j^2); centroid = sum w_j (y_j + 1/2, x_j + 1/2)
  / sum w_j.  Peaks are listed in ascending index order.
"""

from __future__ import annotations

import numpy as np

PEAK_DTYPE = np.dtype([("index", np.int64), ("y", np.float64), ("x", np.float64),
                       ("intensity", np.float64), ("sigma", np.float64)])


def background_at(position, centres, profile):
    """mu_i, sigma_i at pixel angles ``position`` from the profile's non-empty bins."""
    ne = np.asarray(profile["n_members"]) > 0
    pos = np.asarray(position, dtype=np.float64)
    if not ne.any():
        z = np.zeros(pos.shape)
        return z, z.copy()
    xp = np.asarray(centres, dtype=np.float64)[ne]
    mu = np.interp(pos, xp, np.asarray(profile["mean"], dtype=np.float64)[ne])
    sd = np.interp(pos, xp, np.asarray(profile["std"], dtype=np.float64)[ne])
    return mu, sd


def pixel_state(frame, mask, position, centres, profile, noise=0.0, norm=None):
    """v, mu, sigma_eff and validity for every pixel of one frame (flat arrays)."""
    s = np.asarray(frame, dtype=np.float64).reshape(-1)
    valid = np.isfinite(s)
    if mask is not None:
        valid &= np.asarray(mask).reshape(-1) == 0
    if norm is not None:
        s = s / np.asarray(norm, dtype=np.float64).reshape(-1)
    v = np.where(valid, s, 0.0)
    mu, sd = background_at(position, centres, profile)
    return v, mu, np.sqrt(sd * sd + noise * noise), valid


def compress(frame, mask, position, centres, profile, n_pick=3.0, noise=0.0, norm=None):
    """Sparse frame: (indices int64 ascending, values float64 = v)."""
    v, mu, se, valid = pixel_state(frame, mask, position, centres, profile, noise, norm)
    keep = valid & (v - mu > n_pick * se)
    idx = np.nonzero(keep)[0]
    return idx, v[idx]


def densify(indices, values, n_pix, mask, position, centres, profile, valid=None):
    """Noise-free dense frame from a sparse one (float64 [n_pix])."""
    mu, _ = background_at(position, centres, profile)
    ok = np.ones(n_pix, dtype=bool) if mask is None else np.asarray(mask).reshape(-1) == 0
    if valid is not None:
        ok &= valid
    dense = np.where(ok, mu, 0.0)
    dense[np.asarray(indices)] = values
    return dense


def densify_noisy(indices, values, n_pix, mask, position, centres, profile, seed, frame, trunc=np.inf):
    """Dense frame with regenerated background noise (float64 [n_pix]).

    Sec. 3.2 asks for the background to be rebuilt "with noise" of the
    original's spread for programs that analyse noise.  Reading: a pixel
    that was not kept gets mu_i + sigma_i z_i, z_i a standard normal of the
    counter-based generator of ``oracle.rng`` (seed, absolute frame number,
    pixel), drawn at most ``trunc``: a pixel that was not kept lay at most
    n_pick sigma above the background, so passing trunc = n_pick keeps the
    regenerated noise below the sparsification threshold (the first of the
    pixel's two normals not above trunc, else trunc itself).  Kept pixels get
    their stored value, masked pixels 0.
    """
    from . import rng
    mu, sd = background_at(position, centres, profile)
    za, zb = rng.pixel_normals(seed, frame, n_pix)
    z = rng.truncated(za, zb, trunc)
    ok = np.ones(n_pix, dtype=bool) if mask is None else np.asarray(mask).reshape(-1) == 0
    dense = np.where(ok, mu + sd * z, 0.0)
    dense[np.asarray(indices)] = values
    return dense


def veto(n_peaks, n_kept, threshold, hist_bins=256):
    """Peak-count veto of Sec. 4 ("Peak count as veto algorithm").

    A frame is a hit when its peak count reaches the threshold; the
    acquisition keeps hits and may discard the rest.  Besides the per-frame
    decision the counters needed to choose the threshold live are returned:
    hits, non-hits, kept entries (the sparse payload) of each, and for every
    peak count p < hist_bins - 1 the number of frames and of kept entries
    with exactly p peaks (the last bin collects p >= hist_bins - 1, the first
    any count below 0, which the path never produces).  For any
    threshold T < hist_bins the frames (payload) a veto at T would discard
    are the sums of those histograms below T.
    """
    n_peaks = np.asarray(n_peaks, dtype=np.int64)
    n_kept = np.asarray(n_kept, dtype=np.int64)
    hit = n_peaks >= threshold
    b = np.clip(n_peaks, 0, hist_bins - 1)
    return dict(hit=hit,
                hits=int(hit.sum()), misses=int((~hit).sum()),
                kept_hits=int(n_kept[hit].sum()), kept_misses=int(n_kept[~hit].sum()),
                hist_frames=np.bincount(b, minlength=hist_bins).astype(np.int64),
                hist_kept=np.bincount(b, weights=n_kept, minlength=hist_bins).astype(np.int64))


def _shift(a, dy, dx, fill):
    """out[y, x] = a[y + dy, x + dx] where in bounds, else ``fill``."""
    H, W = a.shape
    out = np.full_like(a, fill)
    ys, yd = (slice(dy, H), slice(0, H - dy)) if dy >= 0 else (slice(0, H + dy), slice(-dy, H))
    xs, xd = (slice(dx, W), slice(0, W - dx)) if dx >= 0 else (slice(0, W + dx), slice(-dx, W))
    out[yd, xd] = a[ys, xs]
    return out


def peakfind(frame, mask, height, width, position, centres, profile,
             snr=3.0, patch=3, min_count=3, noise=0.0, norm=None):
    """Peaks of one frame as a structured array (PEAK_DTYPE), ascending index."""
    v, mu, se, valid = pixel_state(frame, mask, position, centres, profile, noise, norm)
    H, W = height, width
    cand = valid & (v - mu >= snr * se)
    V = v.reshape(H, W)
    VA = valid.reshape(H, W)
    C = cand.reshape(H, W)
    Wt = np.where(cand, v - mu, 0.0).reshape(H, W)
    S2 = np.where(cand, se * se, 0.0).reshape(H, W)
    idx = np.arange(H * W, dtype=np.int64).reshape(H, W)
    yy = np.broadcast_to(np.arange(H, dtype=np.float64)[:, None] + 0.5, (H, W))
    xx = np.broadcast_to(np.arange(W, dtype=np.float64)[None, :] + 0.5, (H, W))
    is_max = C.copy()
    count = np.zeros((H, W), dtype=np.int64)
    I = np.zeros((H, W))
    s2 = np.zeros((H, W))
    cy = np.zeros((H, W))
    cx = np.zeros((H, W))
    h = patch // 2
    for dy in range(-h, h + 1):
        for dx in range(-h, h + 1):
            nv = _shift(V, dy, dx, 0.0)
            nva = _shift(VA, dy, dx, False)
            ni = _shift(idx, dy, dx, -1)
            beats = nva & ((nv > V) | ((nv == V) & (ni < idx)))
            if dy or dx:
                is_max &= ~beats
            count += _shift(C, dy, dx, False)
            w = _shift(Wt, dy, dx, 0.0)
            I += w
            s2 += _shift(S2, dy, dx, 0.0)
            cy += w * _shift(yy, dy, dx, 0.0)
            cx += w * _shift(xx, dy, dx, 0.0)
    peak = is_max & (count >= min_count)
    sel = np.nonzero(peak.reshape(-1))[0]
    out = np.zeros(sel.size, dtype=PEAK_DTYPE)
    out["index"] = sel
    Ii = I.reshape(-1)[sel]
    out["intensity"] = Ii
    out["sigma"] = np.sqrt(s2.reshape(-1)[sel])
    out["y"] = cy.reshape(-1)[sel] / Ii
    out["x"] = cx.reshape(-1)[sel] / Ii
    return out


def peakfind_loops(frame, mask, height, width, position, centres, profile,
                   snr=3.0, patch=3, min_count=3, noise=0.0, norm=None):
    """The same peak rule with explicit Python loops (small frames only)."""
    v, mu, se, valid = pixel_state(frame, mask, position, centres, profile, noise, norm)
    H, W = height, width
    cand = valid & (v - mu >= snr * se)
    h = patch // 2
    rows = []
    for i in np.nonzero(cand)[0]:
        y, x = divmod(int(i), W)
        best = True
        n = 0
        I = s2 = sy = sx = 0.0
        for yy in range(max(0, y - h), min(H, y + h + 1)):
            for xx in range(max(0, x - h), min(W, x + h + 1)):
                j = yy * W + xx
                if valid[j] and j != i and (v[j] > v[i] or (v[j] == v[i] and j < i)):
                    best = False
                if cand[j]:
                    n += 1
                    w = v[j] - mu[j]
                    I += w
                    s2 += se[j] ** 2
                    sy += w * (yy + 0.5)
                    sx += w * (xx + 0.5)
        if best and n >= min_count:
            rows.append((i, sy / I, sx / I, I, np.sqrt(s2)))
    return np.array(rows, dtype=PEAK_DTYPE)


def ideal_ratio(kept_fraction: float, dense_bytes: float = 4.0, sparse_bytes: float = 8.0) -> float:
    """Size ratio of a dense float32 frame to its sparse form (index + value per kept pixel)."""
    return dense_bytes / (sparse_bytes * kept_fraction)
