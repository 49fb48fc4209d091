"""Pins of the oracle's raw-word correction (CPU only).

The formula is the build's reading (the paper defers it to its LImA2
reference); it is pinned here against the detector forward model of the
``synth`` package, which encodes photons into gain bits and ADC counts.
"""

import numpy as np

import synth
from synth.scene import GAIN_LEVEL_CODES
from oracle import correct as Cr


def test_round_trip_through_encoder_exhaustive():
    """Every ADC value of every gain code: a calibration with exact binary
    values makes the encoder's ADC = ped + E * gain invert exactly."""
    n = 16384
    ped = np.array([[100.0] * n, [200.0] * n, [300.0] * n], dtype=np.float32)
    gain = np.array([[4.0] * n, [2.0] * n, [0.5] * n], dtype=np.float32)
    adc = np.arange(n, dtype=np.uint16)
    for level, code in enumerate(GAIN_LEVEL_CODES):
        words = (np.uint16(code) << np.uint16(14)) | adc
        sig, bad = Cr.correct(words, ped, gain)
        photons = (adc.astype(np.float64) - ped[level, 0]) / gain[level, 0]
        assert not bad.any()
        assert np.array_equal(sig, photons.astype(np.float32))
    words = (np.uint16(2) << np.uint16(14)) | adc
    sig, bad = Cr.correct(words, ped, gain)
    assert bad.all() and np.isnan(sig).all()


def test_levels_are_per_pixel():
    ped = np.array([[10.0, 20.0], [30.0, 40.0], [50.0, 60.0]], dtype=np.float32)
    gain = np.array([[1.0, 2.0], [4.0, 8.0], [0.25, 0.5]], dtype=np.float32)
    # pixel 0 at level 1 (code 01), pixel 1 at level 2 (code 11)
    words = np.array([(1 << 14) | 70, (3 << 14) | 61], dtype=np.uint16)
    sig, bad = Cr.correct(words, ped, gain)
    assert sig.tolist() == [10.0, 2.0]


def test_recovers_photons_of_synthetic_frames():
    g = synth.JUNGFRAU4M
    ped, gain = synth.jungfrau_calibration(g)
    word, truth = synth.jungfrau_frame(g, 3)
    sig, bad = Cr.correct(word.reshape(-1), ped, gain)
    assert not bad.any()
    level = truth["level"].reshape(-1)
    adc = word.reshape(-1) & 0x3FFF
    inside = (adc > 0) & (adc < 16383)
    idx = np.arange(level.size)
    # ADC noise is N(0, 2) ADU plus rounding: 7 sigma + 0.5 ADU, in photons
    bound = (7 * 2.0 + 0.5) / gain[level, idx].astype(np.float64)
    err = np.abs(sig.astype(np.float64) - truth["photons"].reshape(-1))
    assert np.all(err[inside] <= bound[inside] + 1e-3)
    # gain mix close to the configured 95 / 4.5 / 0.5 percent
    mix = np.bincount(level, minlength=3) / level.size
    assert abs(mix[0] - 0.95) < 0.003 and abs(mix[1] - 0.045) < 0.003 and abs(mix[2] - 0.005) < 0.001
