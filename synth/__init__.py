"""Seeded synthetic inputs for the signal-separation path.

This package is the only code shared by the HIP path and the FP64 oracle.  It
describes the *scene* (detector shape, masks, an isotropic background with
Poisson noise, Gaussian Bragg spots, the per-pixel normalisation factors and
the Jungfrau detector's forward encoding into gain bits and ADC counts).  It
computes none of the method's steps: no binning, no CSR, no correction of raw
words, no statistics, no clipping, no classification.

Every draw comes from ``numpy.random.default_rng`` seeded with a
``SeedSequence([config_id, frame_idx])`` (calibration: ``[config_id, 999999]``;
the clip surrogate's training frames: ``[config_id, 1000000 + frame_idx]``;
the batched mixed-detector frames: ``[config_id, 2000000 + frame_idx]``;
the stored sparse frames read by densification:
``[config_id, 3000000 + frame_idx]``),
so both sides see identical bytes.
"""

from .scene import (  # noqa: F401
    Geometry,
    SMALL,
    JUNGFRAU4M,
    JUNGFRAU1M,
    JUNGFRAU16M,
    JUNGFRAU9M,
    GEOMETRIES,
    stripe_mask,
    scattering_angle_deg,
    azimuth_rad,
    normalisation,
    background_counts,
    spot_expectation,
    float_frame,
    jungfrau_calibration,
    jungfrau_frame,
    float_frames,
    jungfrau_frames,
    training_frame,
    uneven_frame,
    stored_sparse,
)
