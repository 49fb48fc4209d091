"""Pins of the oracle's classification, compression and peak finder (CPU only)."""

import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.special import ndtr

import synth
from oracle import classify as K
from oracle import geometry as G
from oracle import stats as S


def _small_frame(k=0):
    g = synth.SMALL
    m = synth.stripe_mask(g)
    csr = G.csr_for(g, m)
    f, truth = synth.float_frame(g, k)
    prof = S.sigma_clip(f.reshape(-1), None, csr, m.reshape(-1))
    return g, m, csr, f, prof, truth


def test_background_interpolation_by_search(rng):
    """numpy.interp over non-empty bins equals a hand search of the bracketing
    non-empty bin centres, constant beyond the ends."""
    nb = 40
    centres = (np.arange(nb) + 0.5) * 0.25
    prof = dict(n_members=rng.integers(0, 3, nb), mean=rng.uniform(1, 9, nb), std=rng.uniform(0.1, 2, nb))
    prof["n_members"][[0, 1, nb - 1]] = 0
    ne = [r for r in range(nb) if prof["n_members"][r] > 0]
    pos = rng.uniform(-1, 11, 500)
    mu, sd = K.background_at(pos, centres, prof)
    for p, a, b in zip(pos, mu, sd):
        below = [r for r in ne if centres[r] <= p]
        above = [r for r in ne if centres[r] >= p]
        if not below:
            want = (prof["mean"][ne[0]], prof["std"][ne[0]])
        elif not above:
            want = (prof["mean"][ne[-1]], prof["std"][ne[-1]])
        else:
            lo, hi = below[-1], above[0]
            t = 0.0 if hi == lo else (p - centres[lo]) / (centres[hi] - centres[lo])
            want = (prof["mean"][lo] + t * (prof["mean"][hi] - prof["mean"][lo]),
                    prof["std"][lo] + t * (prof["std"][hi] - prof["std"][lo]))
        assert a == pytest.approx(want[0], rel=1e-12) and b == pytest.approx(want[1], rel=1e-12)


def test_kept_fraction_follows_normal_tails(golden):
    """Fig. distribution: a normal background keeps 16 / 2.3 / 0.13 percent of
    pixels at n = 1 / 2 / 3 (no clipping, so mu and sigma are the sample's)."""
    gd = golden("compression.txt")
    rng = np.random.default_rng(7)
    n_pix = 2_000_000
    values = rng.normal(500.0, 20.0, n_pix)
    csr = G.build_csr(1, n_pix, 1e-9, 1.0, 0.5, -1e6, 1, "none")
    prof = S.integrate(values, None, csr)
    pos = np.full(n_pix, csr.centres[0])
    for n, key in ((1, "tail_n1_percent"), (2, "tail_n2_percent"), (3, "tail_n3_percent")):
        idx, _ = K.compress(values, None, pos, csr.centres, prof, n_pick=float(n))
        frac = idx.size / n_pix
        p = 1.0 - ndtr(n)
        assert abs(frac - p) <= 5 * math.sqrt(p * (1 - p) / n_pix)
        # the paper prints the tail to 1 / 0.1 / 0.01 percent
        unit = {1: 1.0, 2: 0.1, 3: 0.01}[n]
        assert abs(100 * p - gd[key]) <= unit / 2 + 1e-3


def test_compression_ratio_arithmetic(golden):
    gd = golden("compression.txt")
    assert round(K.ideal_ratio(1.0 - ndtr(2.0))) == gd["ratio_2sigma"]
    need = gd["detector_links_gbit"] / gd["storage_link_gbit"] * gd["expansion"]
    assert need == pytest.approx(gd["minimum_ratio"])
    assert K.ideal_ratio(1.0 - ndtr(gd["sufficient_cutoff_sigma"])) >= need
    assert K.ideal_ratio(1.0 - ndtr(1.4)) < need


def test_round_trip_invariant():
    g, m, csr, f, prof, _ = _small_frame(1)
    pos = G.position_for(g)
    n_pick = 3.0
    idx, val = K.compress(f, m, pos, csr.centres, prof, n_pick=n_pick)
    assert np.all(np.diff(idx) > 0)
    dense = K.densify(idx, val, g.n_pix, m, pos, csr.centres, prof)
    v = f.reshape(-1).astype(np.float64)
    mu, sd = K.background_at(pos, csr.centres, prof)
    kept = np.zeros(g.n_pix, dtype=bool)
    kept[idx] = True
    valid = m.reshape(-1) == 0
    assert np.array_equal(dense[kept], v[kept])
    drop = valid & ~kept
    assert np.all(v[drop] - dense[drop] <= n_pick * sd[drop])
    assert np.all(dense[~valid] == 0.0)
    # raising the threshold never keeps more
    idx2, _ = K.compress(f, m, pos, csr.centres, prof, n_pick=4.0)
    assert set(idx2.tolist()) <= set(idx.tolist())


def _peaks_scipy(v, valid, cand, mu, se, H, W, patch, min_count):
    """A second implementation on scipy.ndimage filters.  Ties in v are broken
    towards the lower index by subtracting index / (2 N), valid for values
    that differ by at least 1 (integer counts)."""
    N = H * W
    key = np.where(valid, v - np.arange(N) / (2.0 * N), -np.inf).reshape(H, W)
    mx = ndimage.maximum_filter(key, size=patch, mode="constant", cval=-np.inf)
    is_max = cand.reshape(H, W) & (key == mx)
    ones = np.ones((patch, patch))
    cnt = ndimage.correlate(cand.reshape(H, W).astype(np.int64), ones.astype(np.int64), mode="constant")
    w = np.where(cand, v - mu, 0.0).reshape(H, W)
    I = ndimage.correlate(w, ones, mode="constant")
    yy, xx = np.mgrid[0:H, 0:W] + 0.5
    sy = ndimage.correlate(w * yy, ones, mode="constant")
    sx = ndimage.correlate(w * xx, ones, mode="constant")
    s2 = ndimage.correlate(np.where(cand, se * se, 0.0).reshape(H, W), ones, mode="constant")
    sel = np.nonzero((is_max & (cnt >= min_count)).reshape(-1))[0]
    I = np.where(I == 0, 1.0, I)
    return sel, (sy.reshape(-1) / I.reshape(-1))[sel], (sx.reshape(-1) / I.reshape(-1))[sel], \
        I.reshape(-1)[sel], np.sqrt(s2.reshape(-1)[sel])


@pytest.mark.parametrize("patch,min_count", [(3, 3), (5, 4), (3, 1)])
def test_peakfind_three_implementations_agree(patch, min_count):
    g, m, csr, f, prof, _ = _small_frame(2)
    pos = G.position_for(g)
    args = (f, m, g.height, g.width, pos, csr.centres, prof)
    a = K.peakfind(*args, snr=3.0, patch=patch, min_count=min_count)
    b = K.peakfind_loops(*args, snr=3.0, patch=patch, min_count=min_count)
    assert a.size > 5
    assert np.array_equal(a["index"], b["index"])
    for k in ("y", "x", "intensity", "sigma"):
        assert np.allclose(a[k], b[k], rtol=1e-12)
    v, mu, se, valid = K.pixel_state(f, m, pos, csr.centres, prof)
    cand = valid & (v - mu >= 3.0 * se)
    sel, y, x, I, s = _peaks_scipy(v, valid, cand, mu, se, g.height, g.width, patch, min_count)
    assert np.array_equal(a["index"], sel)
    assert np.allclose(a["y"], y, rtol=1e-12) and np.allclose(a["x"], x, rtol=1e-12)
    assert np.allclose(a["intensity"], I, rtol=1e-12) and np.allclose(a["sigma"], s, rtol=1e-12)


def test_peakfind_tie_goes_to_lower_index():
    H, W = 5, 5
    v = np.zeros(H * W)
    v[[6, 7, 11]] = 10.0  # three equal pixels: (1, 1), (1, 2), (2, 1)
    prof = dict(n_members=np.array([1]), mean=np.array([0.0]), std=np.array([1.0]))
    pos = np.zeros(H * W)
    out = K.peakfind(v, None, H, W, pos, np.array([0.0]), prof, snr=3.0, patch=3, min_count=3)
    assert out["index"].tolist() == [6]
    assert out["intensity"][0] == 30.0
    assert out["y"][0] == pytest.approx(5.5 / 3) and out["x"][0] == pytest.approx(5.5 / 3)


def test_isolated_spots_are_found_once():
    """Strong isolated spots on a Poisson background: one peak each, centroid
    close to the spot centre."""
    H, W = 200, 200
    rng = np.random.default_rng(3)
    centres = [(40.3, 50.7), (120.5, 30.2), (150.8, 160.1), (60.1, 140.6)]
    lam = np.full((H, W), 50.0)
    for cy, cx in centres:
        ey, ex = np.arange(H + 1.0), np.arange(W + 1.0)
        py = np.diff(ndtr((ey - cy) / 1.2))
        px = np.diff(ndtr((ex - cx) / 1.2))
        lam += 5000.0 * py[:, None] * px[None, :]
    img = rng.poisson(lam).astype(np.float64).reshape(-1)
    csr = G.build_csr(H, W, 75e-6, 0.1, 100.3, 100.7, 40, "none")
    prof = S.sigma_clip(img, None, csr)
    pos = G.centre_angle(H, W, 75e-6, 0.1, 100.3, 100.7)
    # the setting of the paper's comparison (Sec. 4.1): SNR 3, 4 pixels in a 5x5 patch
    pk = K.peakfind(img, None, H, W, pos, csr.centres, prof, snr=3.0, patch=5, min_count=4)
    strong = [p for p in pk if p["intensity"] > 1000]
    assert len(strong) == len(centres)
    for cy, cx in centres:
        d = [math.hypot(p["y"] - cy, p["x"] - cx) for p in strong]
        assert min(d) < 0.15
