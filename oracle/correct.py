"""Jungfrau raw-word correction (FP64, rounded to float32 at the end).

Sec. 1.2: each Jungfrau pixel switches between three gain levels and carries
three pedestals and three gains; pre-processing expands the 16-bit word to a
32-bit floating point value.  The paper defers the formula to the LImA2
reference, so this is a reading, **parity unpinned** against the paper:

* bits 15..14 of the word are the gain code, bits 13..0 the ADC value;
* codes 00, 01, 11 select gain levels 0, 1, 2; code 10 is not a valid level:
  the pixel is invalid in that frame (signal NaN, counted);
* signal = (ADC - pedestal[g]) / gain[g], gains in ADU per photon, so the
  signal is in photons (the dark-current subtraction of eq. norm);
* the corrected frame is stored as float32, the precision the paper gives
  for pre-processed data; the arithmetic before that rounding is float64.

``normalise`` applies the normalisation of eq. norm, I = signal / norm, in
float64 and stores it as a float32 frame (the corrected frame a correction
stage hands out).  The statistics and the classification do not take that
rounded frame: they take the float32 signal and norm and form I = signal /
norm in float64 themselves (``oracle.stats``, ``oracle.classify``).
"""

from __future__ import annotations

import numpy as np

CODE_TO_LEVEL = np.array([0, 1, -1, 2], dtype=np.int64)


def decode(words: np.ndarray):
    """Split raw words into (gain level, ADC); level -1 marks an invalid code."""
    w = np.asarray(words).astype(np.int64)
    return CODE_TO_LEVEL[(w >> 14) & 3], w & 0x3FFF


def correct(raw: np.ndarray, pedestal: np.ndarray, gain: np.ndarray):
    """Correct raw frames.

    raw: uint16 [..., N]; pedestal, gain: float32 [3, N] (per pixel, per level).
    Returns (signal float32 [..., N] with NaN where invalid, invalid bool).
    """
    raw = np.asarray(raw)
    shape = raw.shape
    level, adc = decode(raw.reshape(-1, shape[-1]))
    invalid = level < 0
    g = np.where(invalid, 0, level)
    pix = np.arange(shape[-1])[None, :]
    ped = pedestal.astype(np.float64)[g, pix]
    gn = gain.astype(np.float64)[g, pix]
    signal = (adc.astype(np.float64) - ped) / gn
    signal[invalid] = np.nan
    return signal.astype(np.float32).reshape(shape), invalid.reshape(shape)


def normalise(signal: np.ndarray, norm=None) -> np.ndarray:
    """Corrected intensity I = signal / norm (eq. norm) as a float32 frame."""
    s = np.asarray(signal, dtype=np.float64)
    if norm is None:
        return s.astype(np.float32)
    return (s / np.asarray(norm, dtype=np.float64)).astype(np.float32)
