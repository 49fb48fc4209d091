"""Pins of the oracle's geometry and CSR builder (CPU only)."""

import math

import numpy as np
import pytest

import synth
from oracle import geometry as G


def _corner_angles_loop(H, W, p, D, cy, cx, y, x):
    out = []
    for yy in (y, y + 1):
        for xx in (x, x + 1):
            out.append(math.degrees(math.atan(p * math.hypot(yy - cy, xx - cx) / D)))
    return out


def test_angle_closed_forms():
    # pixel (0, 0) has its centre at (0.5, 0.5); put the beam one pixel to
    # its left so r = 1 pixel, and pixel size = distance: 2theta = 45 deg
    t = G.centre_angle(1, 1, 1.0, 1.0, 0.5, -0.5)
    assert t[0] == pytest.approx(45.0, abs=1e-12)
    # 3-4-5 triangle: offset (3, 4) pixels, r = 5 pixels, distance = 5 pixels
    t = G.centre_angle(1, 1, 1e-4, 5e-4, 0.5 - 3, 0.5 - 4)
    assert t[0] == pytest.approx(45.0, abs=1e-12)
    # the beam centre on a pixel centre gives 0
    t = G.centre_angle(3, 3, 75e-6, 0.1, 1.5, 1.5)
    assert t[4] == 0.0


def test_tth_max_is_largest_corner():
    H, W, p, D, cy, cx = 7, 9, 75e-6, 0.01, 2.3, 6.1
    csr = G.build_csr(H, W, p, D, cy, cx, 10, "bbox")
    best = max(max(_corner_angles_loop(H, W, p, D, cy, cx, y, x)) for y in range(H) for x in range(W))
    assert csr.tth_max == pytest.approx(best, rel=1e-14)
    assert csr.width == pytest.approx(best / 10, rel=1e-14)


def test_no_split_small_config():
    g = synth.SMALL
    m = synth.stripe_mask(g)
    csr = G.csr_for(g, m)
    assert csr.nnz == int((m == 0).sum()) == 249001
    assert np.all(csr.coef == 1.0)
    tc = G.position_for(g)
    rows = np.repeat(np.arange(csr.n_bins), np.diff(csr.indptr))
    lo = rows * csr.width
    hi = (rows + 1) * csr.width
    t = tc[csr.indices]
    assert np.all((t >= lo) & ((t < hi) | (rows == csr.n_bins - 1)))
    for r in range(csr.n_bins):
        idx, _ = csr.row(r)
        assert np.all(np.diff(idx) > 0)
    assert not np.any(m.reshape(-1)[csr.indices])


def test_bbox_coefficients_sum_to_one():
    g = synth.JUNGFRAU1M
    m = synth.stripe_mask(g)
    csr = G.csr_for(g, m)
    s = np.bincount(csr.indices, weights=csr.coef, minlength=csr.n_pix)
    valid = m.reshape(-1) == 0
    assert np.abs(s[valid] - 1.0).max() <= 1e-12
    assert np.all(s[~valid] == 0.0)
    per_pixel = np.bincount(csr.indices, minlength=csr.n_pix)
    assert per_pixel.max() <= 4
    assert np.all(csr.coef > 0) and np.all(csr.coef <= 1.0 + 1e-15)
    for r in range(0, csr.n_bins, 37):
        idx, _ = csr.row(r)
        assert np.all(np.diff(idx) > 0)


def test_bbox_coefficients_by_sampling(rng):
    """Each coefficient equals the share of its pixel's angle interval that a
    dense uniform sampling puts in the bin."""
    H, W, p, D, cy, cx, nb = 40, 50, 75e-6, 0.002, 17.4, 22.6, 60
    csr = G.build_csr(H, W, p, D, cy, cx, nb, "bbox")
    w = csr.tth_max / nb
    for _ in range(60):
        y, x = int(rng.integers(H)), int(rng.integers(W))
        ang = _corner_angles_loop(H, W, p, D, cy, cx, y, x)
        lo, hi = min(ang), max(ang)
        if y == int(math.floor(cy)) and x == int(math.floor(cx)):
            lo = 0.0
        n = 200000
        s = lo + (np.arange(n) + 0.5) * (hi - lo) / n
        b = np.minimum((s / w).astype(np.int64), nb - 1)
        share = np.bincount(b, minlength=nb) / n
        i = y * W + x
        got = np.zeros(nb)
        for r in range(nb):
            idx, c = csr.row(r)
            hit = np.nonzero(idx == i)[0]
            if hit.size:
                got[r] = c[hit[0]]
        assert np.abs(got - share).max() <= 2.0 / n + 1e-9


def test_centre_pixel_reaches_zero():
    H, W, cy, cx = 9, 9, 4.3, 4.6
    csr = G.build_csr(H, W, 75e-6, 0.01, cy, cx, 50, "bbox")
    idx, c = csr.row(0)
    assert (4 * W + 4) in set(idx.tolist())
