"""Comparison helpers for the GPU-vs-oracle parity tests.

What is compared
----------------
* Profile statistics (mean, std, sem, Omega): |x - x_ref| <= 1e-5 |x_ref| +
  1e-7 |mean_ref| (the relative tolerance asked of bin means and stds).
* Integer results (members, passes, converged flag) exactly, against the
  oracle's clip *replayed* (R22): at every pass, each decision that the
  rounding of the GPU's inputs could flip (a member inside the band below)
  is taken both ways, and the GPU must reproduce one outcome of that replay
  exactly in its integers and within the tolerance in its statistics.  A bin
  is never dropped from the comparison; a bin whose replay grows beyond a
  few hundred outcomes would be reported as unresolved (tests require none).
* Kept pixels and peaks against the oracle's classification with the
  *resolved* profile (each bin's matched outcome), exactly, except pixels
  whose own keep / candidate decision lies within rounding of its threshold
  (their count is bounded by the tests), and kept values bit for bit as the
  float32 rounding of v.

Why there is a band, and its width
----------------------------------
The oracle forms v = signal / norm and omega = c norm in float64 from the
float32 signal, norm and its own float64 CSR coefficients.  The GPU holds per
member the float32 value v' = RN32(signal / norm) (``ss_correct`` is pinned
bit-exact to that rounding) and the float32 weight w' = RN32(c' norm) with
c' its own builder's coefficient (pinned to |c' - c| <= 1e-12 c by the ABI
tests), and accumulates in float64.  Hence, with u = 2^-24:
  |v' - v| <= eps_v |v|,  eps_v = u (0 when the frame is float32 data with
  norm = 1: then v' = v);
  |w' - omega| <= eps_w omega, eps_w = u (1 + 2^-20) (0 when c = 1, norm = 1).
For one pass over one member set with oracle statistics (m, s), to first
order in eps (A = sum omega |v| / Omega, s1 = sum omega |v - m| / Omega,
R = sqrt(sum omega^2 v^2 / sum omega^2)):
  |m' - m| <= eps_w s1 + eps_v A                     =: dm
  |s' - s| <= 2 eps_w s + eps_v R + dm                (azimuthal; triangle
                                                       inequality in the
                                                       omega^2-weighted norm)
  |s'_p - s_p| <= (2 eps_w + eps_v) s_p               (Poisson)
so the deviation test d = |v - m| - n s of one member moves by at most
eps_v |v| + (1 + n) dm + n ds.  The band is twice that (second-order
terms) plus gamma (|m| + n s) with gamma = 2^-26 for the float64
accumulation of both sides (the GPU subtracts removed members from running
sums and re-accumulates before cancellation exceeds six digits).  With
eps = 0 (float32 frames, unit weights) the band is gamma alone: a relative
~6e-8 of the threshold for Poisson-like bins.  Only the GPU's own clip
decisions are exact functions of its float32 inputs (it compares v' against
bounds rounded once per pass), so that is the whole error budget.

Pixel decisions: v - mu > n sigma_eff (keep) and >= snr sigma_eff
(candidate).  The GPU's mu, sigma come from its own profile, interpolated at
the pixel's position stored to 2^-20 of an interval; its decision is exact
for those (a float32 fast path with a certified bound, float64 otherwise).
The band of a pixel: 2 (eps_v |v| + dmu + n dsigma) + 2^-40 (|v| + |mu| +
n sigma_eff), with dmu, dsigma the largest |GPU - oracle| profile
difference of the pixel's two bracketing bins plus 2^-20 of the profile
step across them.
"""

from __future__ import annotations

import math

import numpy as np

import synth
from oracle import classify as OK
from oracle import correct as OC
from oracle import geometry as OG
from oracle import stats as OS

REL = 1e-5
ABS_OF_MEAN = 1e-7
U32 = 2.0 ** -24
GAMMA = 2.0 ** -26
PIX_GAMMA = 2.0 ** -40
POS_QUANTUM = 2.0 ** -20
MAX_OUTCOMES = 512
MODELS = {"azimuthal": OS.AZIMUTHAL, "poisson": OS.POISSON, "hybrid": OS.HYBRID}


def f32(x):
    """A parameter as the library sees it (float32), back in float64."""
    return float(np.float32(x))


def input_eps(norm, split):
    """(eps_v, eps_w) of a geometry: the relative rounding of the GPU's
    member values and weights against the oracle's float64 ones."""
    eps_v = U32 if norm is not None else 0.0
    eps_w = U32 * (1.0 + 2.0 ** -20) if (norm is not None or split != "none") else 0.0
    return eps_v, eps_w


class OracleScene:
    """Oracle-side geometry of a synth geometry (built by the oracle only)."""

    def __init__(self, geom):
        self.geom = geom
        self.mask = synth.stripe_mask(geom).reshape(-1)
        self.norm = synth.normalisation(geom).reshape(-1).astype(np.float32) if geom.normalised else None
        self.csr = OG.csr_for(geom, self.mask)
        self.position = OG.position_for(geom)
        self.centres = self.csr.centres
        self.eps_v, self.eps_w = input_eps(self.norm, geom.split)

    def signal_from_raw(self, raw):
        """float32 signal frames [F, N] (NaN where the gain code is invalid)."""
        ped, gain = synth.jungfrau_calibration(self.geom)
        sig, bad = OC.correct(raw.reshape(raw.shape[0], -1), ped, gain)
        return sig, bad

    def corrected(self, signal):
        """The float32 corrected frames a correction stage hands out."""
        return np.stack([OC.normalise(s, self.norm) for s in signal])

    def profile(self, signal, p):
        return OS.sigma_clip(signal, self.norm, self.csr, self.mask, cutoff=f32(p.cutoff), max_iter=p.max_iter,
                             error_model=MODELS[p.error_model], dark_var=f32(p.dark_var))

    def check_profile(self, gpu, signal, p, label="", mask=None, csr=None, bins=None):
        """Replay comparison of one frame's GPU profile (see the module
        docstring); returns (resolved profile, counts)."""
        return compare_profile(gpu, signal, self.norm, self.csr if csr is None else csr,
                               self.mask if mask is None else mask, p, self.eps_v, self.eps_w, label, bins)

    def check_classify(self, signal, gpu_prof, resolved, kept_index, kept_value, peaks, p, label="", region=None):
        return compare_classify(signal, self.norm, self.mask, self.geom.height, self.geom.width, self.position,
                                self.centres, gpu_prof, resolved, kept_index, kept_value, peaks, p, self.eps_v,
                                label, region)

    def tile_bins(self, region, margin=2):
        """The bins the pixels of tile ``region`` interpolate between (with a
        margin of bins each side)."""
        y0, y1, x0, x1 = region
        pos = self.position.reshape(self.geom.height, self.geom.width)[y0:y1, x0:x1]
        w = self.csr.width
        lo = int(np.floor(pos.min() / w - 0.5)) - margin
        hi = int(np.ceil(pos.max() / w - 0.5)) + margin
        return np.arange(max(lo, 0), min(hi, self.csr.n_bins - 1) + 1)


# -- the clip replay ------------------------------------------------------------------

def clip_band(mb, keep, m, spread, n, model, eps_v, eps_w):
    """Per-member bound on how far the GPU's deviation test |v - m| - n s
    can sit from the oracle's for this member set (module docstring)."""
    w, x = mb.omega[keep], mb.v[keep]
    om = float(np.sum(w))
    oo = float(np.sum(w * w))
    a = float(np.dot(w, np.abs(x))) / om
    s1 = float(np.dot(w, np.abs(x - m["mean"]))) / om
    r = math.sqrt(float(np.dot(w * w, x * x)) / oo)
    dm = eps_w * s1 + eps_v * a
    if model == OS.POISSON:
        ds = (2.0 * eps_w + eps_v) * spread
    else:
        ds = 2.0 * eps_w * spread + eps_v * r + dm
    slack = GAMMA * (abs(m["mean"]) + n * spread)
    return 2.0 * (eps_v * np.abs(mb.v) + (1.0 + n) * dm + n * ds) + slack


def _groups(vals, idx):
    """Members idx split into runs of equal float32 value, ascending."""
    if idx.size == 0:
        return []
    key = vals[idx].astype(np.float32)
    o = np.argsort(key, kind="stable")
    idx, key = idx[o], key[o]
    cut = np.nonzero(np.diff(key) != 0)[0] + 1
    return np.split(idx, cut)


def clip_outcomes(mb, cutoff, max_iter, model, eps_v, eps_w, cap=MAX_OUTCOMES):
    """Every outcome (keep, n_iter, converged) of the clip of eq. clip on the
    members ``mb`` when each decision inside its band may go either way.

    A GPU pass removes the members whose float32 value lies above one bound
    or below another, so its possible removal sets among the band members
    are a run of the largest values above the mean and a run of the smallest
    below it (equal float32 values decided alike): those are the branches.
    Returns (outcomes, complete); complete is False when more than ``cap``
    states were visited.
    """
    v = mb.v
    out, seen, stack, visited = [], set(), [(np.ones(v.size, dtype=bool), 0, 0)], 0
    while stack:
        keep, k, n_iter = stack.pop()
        key = (keep.tobytes(), k, n_iter)
        if key in seen:
            continue
        seen.add(key)
        visited += 1
        if visited > cap:
            return out, False
        if k >= max_iter:
            out.append((keep, n_iter, 0))
            continue
        m = OS.moments(v[keep], mb.omega[keep], mb.pvar[keep], mb.csig[keep])
        n = cutoff if cutoff > 0 else OS.chauvenet(int(keep.sum()))
        spread = m["std_p"] if model == OS.POISSON else m["std"]
        thr = n * spread
        dev = np.abs(v - m["mean"])
        if keep.any() and math.isfinite(thr):
            tau = clip_band(mb, keep, m, spread, n, model, eps_v, eps_w)
            sure = keep & (dev - thr > tau)
            maybe = keep & ~sure & (dev - thr >= -tau)
        else:
            sure = keep & (dev > thr)
            maybe = np.zeros_like(keep)
        up = _groups(v, np.nonzero(maybe & (v >= m["mean"]))[0])
        lo = _groups(v, np.nonzero(maybe & (v < m["mean"]))[0])
        for i in range(len(up) + 1):          # drop the i largest groups above the mean
            for j in range(len(lo) + 1):      # and the j smallest below it
                drop = sure.copy()
                for g in up[len(up) - i:]:
                    drop[g] = True
                for g in lo[:j]:
                    drop[g] = True
                if not drop.any():
                    out.append((keep, n_iter, 1))
                else:
                    stack.append((keep & ~drop, k + 1, n_iter + 1))
    return out, True


def _reported(m, model):
    poisson = model in (OS.POISSON, OS.HYBRID)
    return dict(mean=m["mean"], std=m["std_p"] if poisson else m["std"], sem=m["sem_p"] if poisson else m["sem"],
                sum_w=m["Omega"], n_members=m["n"])


def _matches(g, rep, n_iter, conv):
    if g["n_members"] != rep["n_members"] or g["n_iter"] != n_iter or g["converged"] != conv:
        return False
    tol_ref = ABS_OF_MEAN * abs(rep["mean"])
    return all(abs(g[k] - rep[k]) <= REL * abs(rep[k]) + tol_ref for k in ("mean", "std", "sem", "sum_w"))


def compare_profile(gpu, signal, norm, csr, mask, p, eps_v, eps_w, label="", bins=None):
    """Compare one frame's GPU profile (dict of host arrays [n_bins]) with the
    oracle's clip of ``signal``, replaying decisions inside the band where
    the plain oracle result is not reproduced.  Returns (resolved, counts):
    resolved is the oracle profile of the matched outcome of every compared
    bin, counts = dict(bins, replayed, unresolved).  ``bins`` restricts the
    comparison to a sample of bins (the others keep the GPU's values in
    ``resolved`` and must not be used)."""
    model = MODELS[p.error_model]
    cutoff, dark = f32(p.cutoff), f32(p.dark_var)
    signal = np.asarray(signal).reshape(-1)
    nb = csr.n_bins
    res = dict(mean=np.zeros(nb), std=np.zeros(nb), sem=np.zeros(nb), sum_w=np.zeros(nb),
               n_members=np.zeros(nb, dtype=np.int64), n_iter=np.zeros(nb, dtype=np.int64),
               converged=np.zeros(nb, dtype=np.int64))
    replayed, unresolved = [], []
    if bins is not None:
        for k in res:
            res[k][:] = np.asarray(gpu[k])
    todo = range(nb) if bins is None else sorted(set(int(b) for b in bins))
    for r in todo:
        mb = OS.bin_members(signal, norm, csr, r, mask, dark)
        g = {k: gpu[k][r].item() for k in res}
        keep, n_iter, conv, _ = OS._clip_bin(mb.v, mb.omega, mb.pvar, cutoff, p.max_iter, model, mb.csig)
        plain = _reported(OS.moments(mb.v[keep], mb.omega[keep], mb.pvar[keep], mb.csig[keep]), model)
        found = (plain, n_iter, conv) if _matches(g, plain, n_iter, conv) else None
        if found is None:
            outcomes, complete = clip_outcomes(mb, cutoff, p.max_iter, model, eps_v, eps_w)
            for kp, ni, cv in outcomes:
                rep = _reported(OS.moments(mb.v[kp], mb.omega[kp], mb.pvar[kp], mb.csig[kp]), model)
                if _matches(g, rep, ni, cv):
                    found = (rep, ni, cv)
                    break
            if found is None:
                assert not complete, (label, "bin", r, "GPU", g, "oracle", plain, n_iter, conv,
                                      f"none of {len(outcomes)} replay outcomes matches")
                unresolved.append(r)
                found = (plain, n_iter, conv)
            else:
                replayed.append(r)
        rep, ni, cv = found
        for k in ("mean", "std", "sem", "sum_w", "n_members"):
            res[k][r] = rep[k]
        res["n_iter"][r], res["converged"][r] = ni, cv
    return res, dict(bins=len(todo), replayed=len(replayed), unresolved=len(unresolved), replayed_bins=replayed,
                     unresolved_bins=unresolved)


# -- classification -----------------------------------------------------------------------

def _bracket_dev(position, centres, gpu, ref, key):
    """Per pixel: the largest |gpu - ref| of ``key`` over the pixel's two
    bracketing non-empty bins, plus 2^-20 of the profile step across them."""
    ne = np.asarray(ref["n_members"]) > 0
    if not ne.any():
        return np.zeros(position.size)
    xp = np.asarray(centres, dtype=np.float64)[ne]
    d = np.abs(np.asarray(gpu[key], dtype=np.float64)[ne] - np.asarray(ref[key], dtype=np.float64)[ne])
    y = np.asarray(ref[key], dtype=np.float64)[ne]
    hi = np.clip(np.searchsorted(xp, position, side="right"), 0, xp.size - 1)
    lo = np.clip(hi - 1, 0, xp.size - 1)
    return np.maximum(d[lo], d[hi]) + POS_QUANTUM * np.abs(y[hi] - y[lo])


def pixel_bands(signal, norm, mask, position, centres, gpu_prof, resolved, p, eps_v):
    """(v, keep band, candidate band, valid) of one frame (module docstring)."""
    v, mu, se, valid = OK.pixel_state(signal, mask, position, centres, resolved, f32(p.noise), norm)
    dmu = _bracket_dev(position, centres, gpu_prof, resolved, "mean")
    dsd = _bracket_dev(position, centres, gpu_prof, resolved, "std")
    bands = []
    for thr in (f32(p.n_pick), f32(p.snr)):
        d = v - mu - thr * se
        tau = 2.0 * (eps_v * np.abs(v) + dmu + abs(thr) * dsd) + PIX_GAMMA * (np.abs(v) + np.abs(mu) + abs(thr) * se)
        bands.append(valid & (np.abs(d) <= tau))
    return v, bands[0], bands[1], valid


def _near_tie(v, valid, i, width, patch, eps_v):
    """Whether pixel i has a valid patch neighbour whose value the GPU's
    float32 rounding could put on the other side of v_i (or level with it)."""
    if eps_v == 0.0:
        return False
    y, x = divmod(int(i), width)
    h = patch // 2
    height = v.size // width
    for yy in range(max(0, y - h), min(height, y + h + 1)):
        for xx in range(max(0, x - h), min(width, x + h + 1)):
            j = yy * width + xx
            if j != i and valid[j] and abs(v[j] - v[i]) <= 2.0 * eps_v * max(abs(v[i]), abs(v[j])):
                return True
    return False


def compare_classify(signal, norm, mask, height, width, position, centres, gpu_prof, resolved, kept_index,
                     kept_value, peaks, p, eps_v, label="", region=None):
    """Kept pixels (index and float32 value arrays of one frame) and peaks (a
    PEAK_DTYPE-like structured array) of the GPU against the oracle's
    classification with the resolved profile.  ``region`` = (y0, y1, x0, x1)
    restricts the comparison to a tile: kept pixels inside it, peaks whose
    whole patch lies inside it (the resolved profile must then hold every
    bin the tile's pixels interpolate between).  Returns counts: kept,
    peaks, excused keep / candidate pixels, valid pixels and the list
    differences found inside the band."""
    signal = np.asarray(signal).reshape(-1)
    v, band_k, band_c, valid = pixel_bands(signal, norm, mask, position, centres, gpu_prof, resolved, p, eps_v)
    ri, rv = OK.compress(signal, mask, position, centres, resolved, f32(p.n_pick), f32(p.noise), norm)
    gi = np.asarray(kept_index).astype(np.int64)
    gv = np.asarray(kept_value, dtype=np.float32)
    assert np.all(np.diff(gi) > 0), label
    h = p.patch // 2
    inside = core = None
    if region is not None:
        y0, y1, x0, x1 = region
        yy, xx = np.divmod(np.arange(height * width), width)
        inside = (yy >= y0) & (yy < y1) & (xx >= x0) & (xx < x1)
        core = (yy >= y0 + h) & (yy < y1 - h) & (xx >= x0 + h) & (xx < x1 - h)
        gsel, rsel = inside[gi], inside[ri]
        gi, gv, ri, rv = gi[gsel], gv[gsel], ri[rsel], rv[rsel]
        band_k, band_c, valid = band_k & inside, band_c & inside, valid & inside
    diff = np.setxor1d(gi, ri)
    assert np.all(band_k[diff]), (label, "kept", diff[~band_k[diff]][:10])
    _, gp, rp = np.intersect1d(gi, ri, return_indices=True)
    assert np.array_equal(gv[gp].view(np.uint32), rv[rp].astype(np.float32).view(np.uint32)), label

    ref = OK.peakfind(signal, mask, height, width, position, centres, resolved, f32(p.snr), p.patch, p.min_count,
                      f32(p.noise), norm)
    gpk = np.asarray(peaks["index"]).astype(np.int64)
    rpk = ref["index"].astype(np.int64)
    assert np.all(np.diff(gpk) > 0), label
    if core is not None:
        peaks, ref = peaks[core[gpk]], ref[core[rpk]]
        gpk, rpk = gpk[core[gpk]], rpk[core[rpk]]
    pdiff = np.setxor1d(gpk, rpk)
    for i in pdiff:
        y, x = divmod(int(i), width)
        ys = np.arange(max(0, y - h), min(height, y + h + 1))
        xs = np.arange(max(0, x - h), min(width, x + h + 1))
        patch_idx = (ys[:, None] * width + xs[None, :]).reshape(-1)
        assert band_c[patch_idx].any() or _near_tie(v, valid, i, width, p.patch, eps_v), (label, "peak", int(i))
    _, gp, rp = np.intersect1d(gpk, rpk, return_indices=True)
    for k in ("y", "x", "intensity", "sigma"):
        a = np.asarray(peaks[k])[gp].astype(np.float64)
        b = ref[k][rp]
        assert np.allclose(a, b, rtol=2e-6, atol=1e-6 * (np.abs(b).max() if b.size else 1)), (label, k)
    return dict(kept=int(ri.size), peaks=int(rpk.size), excused_keep=int(band_k.sum()),
                excused_cand=int(band_c.sum()), valid=int(valid.sum()), kept_diffs=int(diff.size),
                peak_diffs=int(pdiff.size))
