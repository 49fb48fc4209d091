"""Comparison helpers for the GPU-vs-oracle parity tests.

Tolerances (derived from the arithmetic: float32 frames and weights, float64
accumulation on both sides):
* profile statistics: |x - x_ref| <= 1e-5 |x_ref| + 1e-7 |mean_ref|;
* integer decisions (members, passes, kept pixels, peaks) must be identical
  except where the oracle itself puts a decision within a relative 1e-5 of
  its threshold (the margin band), where float rounding may legitimately
  decide either way; such cases are counted and must stay rare.
"""

from __future__ import annotations

import numpy as np

import synth
from oracle import classify as OK
from oracle import correct as OC
from oracle import geometry as OG
from oracle import stats as OS

REL = 1e-5
ABS_OF_MEAN = 1e-7
BAND = 1e-5


def f32(x):
    """A parameter as the library sees it (float32), back in float64."""
    return float(np.float32(x))


class OracleScene:
    """Oracle-side geometry of a synth geometry (built by the oracle only)."""

    def __init__(self, geom):
        self.geom = geom
        self.mask = synth.stripe_mask(geom).reshape(-1)
        self.norm = synth.normalisation(geom).reshape(-1) if geom.normalised else None
        self.csr = OG.csr_for(geom, self.mask)
        self.position = OG.position_for(geom)
        self.centres = self.csr.centres

    def frames_from_raw(self, raw):
        ped, gain = synth.jungfrau_calibration(self.geom)
        sig, bad = OC.correct(raw.reshape(raw.shape[0], -1), ped, gain)
        return np.stack([OC.normalise(s, self.norm) for s in sig]), bad

    def profile(self, frame, p):
        return OS.sigma_clip(frame, self.norm, self.csr, self.mask, cutoff=f32(p.cutoff), max_iter=p.max_iter,
                             error_model={"azimuthal": 0, "poisson": 1, "hybrid": 2}[p.error_model],
                             dark_var=f32(p.dark_var), return_margin=True)

    def compress(self, frame, prof, p):
        return OK.compress(frame, self.mask, self.position, self.centres, prof, f32(p.n_pick), f32(p.noise))

    def peaks(self, frame, prof, p):
        return OK.peakfind(frame, self.mask, self.geom.height, self.geom.width, self.position, self.centres,
                           prof, f32(p.snr), p.patch, p.min_count, f32(p.noise))

    def band_pixels(self, frame, prof, thr, noise):
        """Pixels whose v - mu sits within the band of ``thr`` sigma_eff."""
        v, mu, se, valid = OK.pixel_state(frame, self.mask, self.position, self.centres, prof, f32(noise))
        d = v - mu
        return valid & (np.abs(d - thr * se) <= BAND * thr * se + 1e-12)

    def bins_touching(self, bins):
        """Pixels whose background interpolation reads one of ``bins``."""
        if len(bins) == 0:
            return np.zeros(self.position.size, dtype=bool)
        w = self.csr.width
        t = np.floor((self.position - self.centres[0]) / w).astype(np.int64)
        hit = np.zeros(self.position.size, dtype=bool)
        for b in bins:
            hit |= np.abs(t - b) <= 2
        return hit


def compare_profile(gpu, ref, label=""):
    """Compare one frame's profile; returns the bins excused by the band."""
    margin = ref["margin"]
    band = np.nonzero(margin < BAND)[0]
    ok = np.ones(margin.size, dtype=bool)
    ok[band] = False
    mref = np.abs(ref["mean"])
    for k in ("mean", "std", "sem", "sum_w"):
        g = gpu[k][ok]
        r = ref[k][ok]
        tol = REL * np.abs(r) + ABS_OF_MEAN * mref[ok]
        bad = np.abs(g - r) > tol
        assert not bad.any(), (label, k, np.nonzero(ok)[0][bad][:5], g[bad][:5], r[bad][:5])
    for k in ("n_members", "n_iter", "converged"):
        g = gpu[k][ok]
        r = ref[k][ok]
        assert np.array_equal(g, r), (label, k, np.nonzero(g != r)[0][:5])
    return band


def compare_kept(g_idx, g_val, ref_idx, ref_val, excused, label=""):
    """Kept lists equal outside the excused pixels; values bit-equal."""
    gi = np.asarray(g_idx, dtype=np.int64)
    assert np.all(np.diff(gi) > 0), label
    gs, rs = set(gi.tolist()), set(np.asarray(ref_idx).tolist())
    diff = np.array(sorted(gs ^ rs), dtype=np.int64)
    assert np.all(excused[diff]) if diff.size else True, (label, diff[~excused[diff]][:10])
    common, gpos, rpos = np.intersect1d(gi, ref_idx, return_indices=True)
    assert np.array_equal(np.asarray(g_val)[gpos].astype(np.float64), np.asarray(ref_val)[rpos]), label
    return diff.size


def compare_peaks(g, ref, excused_px, width, patch, label=""):
    """Peak lists equal except peaks whose patch holds an excused pixel."""
    def near_excused(i):
        y, x = divmod(int(i), width)
        h = patch // 2
        ys = np.arange(max(0, y - h), y + h + 1)
        xs = np.arange(max(0, x - h), min(width, x + h + 1))
        idx = (ys[:, None] * width + xs[None, :]).reshape(-1)
        idx = idx[idx < excused_px.size]
        return excused_px[idx].any()

    gi = g["index"].astype(np.int64)
    ri = ref["index"].astype(np.int64)
    assert np.all(np.diff(gi) > 0), label
    diff = sorted(set(gi.tolist()) ^ set(ri.tolist()))
    for i in diff:
        assert near_excused(i), (label, "peak", i)
    common, gp, rp = np.intersect1d(gi, ri, return_indices=True)
    for k in ("y", "x", "intensity", "sigma"):
        a = g[k][gp].astype(np.float64)
        b = ref[k][rp]
        assert np.allclose(a, b, rtol=2e-6, atol=1e-6 * (np.abs(b).max() if b.size else 1)), (label, k)
    return len(diff)
