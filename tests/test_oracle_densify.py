"""Pins of the oracle's noisy densification, its generator and the veto
counters (CPU only).

* Philox4x32-10 against the generator's published known-answer vectors;
* the uniforms' ranges and resolution;
* the Box-Muller normals against the normal distribution (Kolmogorov-Smirnov,
  moments, independence of the pair);
* the truncated draw's mean and point mass against their closed forms;
* noisy densification: kept pixels restored, masked pixels zero, the noise-free
  densification as the zero-spread case, the background's mean and spread;
* the veto on a worked example and its counters' invariants.
"""

import os

import numpy as np
import pytest
from scipy import stats as sst

import synth
from oracle import classify as K
from oracle import geometry as G
from oracle import rng as R

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_kat.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                c, k, o = ([int(x, 16) for x in part.split()] for part in line.split("|"))
                rows.append((c, k, o))
    return rows


@pytest.mark.parametrize("case", range(3))
def test_philox_known_answers(case):
    c, k, o = _kat()[case]
    got = R.philox4x32(np.array([c], dtype=np.uint64), k)[0]
    assert [int(x) for x in got] == o


def test_philox_counter_and_key_sensitivity():
    base = R.philox4x32(np.zeros((1, 4), dtype=np.uint64), (7, 9))[0]
    for j in range(4):
        c = np.zeros((1, 4), dtype=np.uint64)
        c[0, j] = 1
        assert not np.array_equal(R.philox4x32(c, (7, 9))[0], base)
    assert not np.array_equal(R.philox4x32(np.zeros((1, 4), dtype=np.uint64), (8, 9))[0], base)


def test_uniform_ranges():
    w = np.array([0, 255, 256, 0xFFFFFFFF], dtype=np.uint64)
    assert R.uniform_open0(w).tolist() == [2.0 ** -24, 2.0 ** -24, 2.0 ** -23, 1.0]
    assert R.uniform_open1(w).tolist() == [0.0, 0.0, 2.0 ** -24, 1.0 - 2.0 ** -24]
    u = R.uniform_open0(np.arange(0, 2 ** 32, 2 ** 20, dtype=np.uint64))
    assert np.all((u > 0) & (u <= 1)) and np.all(u * 2 ** 24 == np.round(u * 2 ** 24))


def test_normals_are_standard_and_independent():
    za, zb = R.pixel_normals(seed=2024, frame=3, n_pix=400_001)
    for z in (za, zb):
        assert sst.kstest(z, "norm").pvalue > 1e-3
        assert abs(z.mean()) < 5 / np.sqrt(z.size)
        assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert abs(np.corrcoef(za, zb)[0, 1]) < 5 / np.sqrt(za.size)
    # neighbouring pixels (same generator block, other words) are independent too
    assert abs(np.corrcoef(za[0:-1:2], za[1::2])[0, 1]) < 5 / np.sqrt(za.size / 2)


def test_streams_differ_by_seed_and_frame_and_repeat():
    a = R.pixel_normals(1, 0, 1000)[0]
    assert np.array_equal(a, R.pixel_normals(1, 0, 1000)[0])
    assert not np.allclose(a, R.pixel_normals(2, 0, 1000)[0])
    assert not np.allclose(a, R.pixel_normals(1, 1, 1000)[0])
    # a prefix of the frame draws the same numbers (pixel-addressed, not sequential)
    assert np.array_equal(a[:333], R.pixel_normals(1, 0, 333)[0])


@pytest.mark.parametrize("t", [0.0, 1.0, 2.5])
def test_truncated_draw_closed_form(t):
    """First of two independent normals at most t, else t: density
    phi(x) (1 + Q(t)) below t plus a mass Q(t)^2 at t."""
    za, zb = R.pixel_normals(seed=77, frame=0, n_pix=1_000_000)
    z = R.truncated(za, zb, t)
    Q = sst.norm.sf(t)
    assert z.max() <= t
    assert abs(np.mean(z == t) - Q * Q) < 5 * np.sqrt(Q * Q / z.size) + 1e-6
    mean = -(1 + Q) * sst.norm.pdf(t) + Q * Q * t
    assert abs(z.mean() - mean) < 5 / np.sqrt(z.size)


def _flat_profile(nb, mean, std):
    return dict(n_members=np.full(nb, 10), mean=np.full(nb, mean), std=np.full(nb, std))


def test_noisy_densify_flat_background():
    g = synth.SMALL
    m = synth.stripe_mask(g).reshape(-1)
    csr = G.csr_for(g, m)
    pos = G.position_for(g)
    prof = _flat_profile(csr.n_bins, 5.0, 2.0)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(np.nonzero(m == 0)[0], 300, replace=False))
    val = rng.uniform(50, 100, idx.size)
    dense = K.densify_noisy(idx, val, g.n_pix, m, pos, csr.centres, prof, seed=11, frame=4)
    assert np.array_equal(dense[idx], val)
    assert np.all(dense[m != 0] == 0.0)
    bg = np.ones(g.n_pix, dtype=bool)
    bg[idx] = False
    bg &= m == 0
    x = dense[bg]
    assert abs(x.mean() - 5.0) < 5 * 2.0 / np.sqrt(x.size)
    assert abs(x.std() - 2.0) < 5 * 2.0 * np.sqrt(0.5 / x.size)
    # truncated at n_pick = 3: nothing regenerated above mu + 3 sigma
    dt = K.densify_noisy(idx, val, g.n_pix, m, pos, csr.centres, prof, seed=11, frame=4, trunc=3.0)
    assert dt[bg].max() <= 5.0 + 3.0 * 2.0
    # zero spread: the noise-free densification
    p0 = _flat_profile(csr.n_bins, 5.0, 0.0)
    assert np.array_equal(K.densify_noisy(idx, val, g.n_pix, m, pos, csr.centres, p0, 11, 4),
                          K.densify(idx, val, g.n_pix, m, pos, csr.centres, p0))


def test_veto_worked_example():
    n_peaks = [0, 5, 19, 20, 21, 300]
    n_kept = [10, 20, 30, 40, 50, 60]
    v = K.veto(n_peaks, n_kept, threshold=20, hist_bins=256)
    assert v["hit"].tolist() == [False, False, False, True, True, True]
    assert (v["hits"], v["misses"], v["kept_hits"], v["kept_misses"]) == (3, 3, 150, 60)
    want = {0: 1, 5: 1, 19: 1, 20: 1, 21: 1, 255: 1}
    assert {i: int(c) for i, c in enumerate(v["hist_frames"]) if c} == want
    assert v["hist_kept"][255] == 60 and v["hist_kept"][19] == 30 and v["hist_kept"].sum() == 210


def test_veto_histogram_answers_every_threshold():
    rng = np.random.default_rng(5)
    n_peaks = rng.poisson(15, 5000)
    n_kept = rng.integers(1000, 9000, 5000)
    h = K.veto(n_peaks, n_kept, threshold=0, hist_bins=64)
    for T in range(64):
        v = K.veto(n_peaks, n_kept, threshold=T, hist_bins=64)
        assert v["misses"] == h["hist_frames"][:T].sum()
        assert v["kept_misses"] == h["hist_kept"][:T].sum()
        assert v["hits"] + v["misses"] == 5000 and v["kept_hits"] + v["kept_misses"] == n_kept.sum()
