"""Scene model for synthetic diffraction frames.

The workload follows the paper's setting (Sec. 2.1 and Sec. 3): an isotropic
background from amorphous scattering plus a few sharp Bragg spots, recorded
either as photon counts (a counting detector) or as raw Jungfrau words (an
integrating detector with three gain levels, Sec. 1.2).

Scene recipe (all lengths in metres, angles in degrees):

* scattering angle of a pixel centre (y + 1/2, x + 1/2) for a flat detector
  normal to the beam:  2theta = atan(pixel * r / distance);
* background B(2theta) = 150 exp(-2theta/8) + 400 exp(-(2theta - 20)^2 / 8)
  counts per pixel (a decaying term plus a water ring of unit-peak Gaussian
  shape, 2 degrees wide);
* per-pixel normalisation (the ``norm`` of the paper's pre-processing
  equation): 1 for the small float geometry; relative solid angle
  cos^3(2theta) times the polarisation factor
  (1 + cos^2 2theta - f cos(2 chi) sin^2 2theta) / 2 with f = 0.99 for the
  Jungfrau geometry (flat-field, absorption and flux are 1);
* Bragg spots: isotropic Gaussians of sigma = 1.2 px, integral drawn from
  LogNormal(6, 1), centres uniform over unmasked pixels, integrated exactly
  over each pixel area with the normal CDF;
* counts ~ Poisson(norm * B + spots);
* Jungfrau encoding: gain level g drawn i.i.d. with probabilities
  (0.95, 0.045, 0.005), raised while the level would saturate;
  ADC = clip(round(ped_g + E * gain_g + N(0, 2)), 0, 16383) and the 16-bit
  word is code(g) << 14 | ADC with codes 0, 1, 3 for levels 0, 1, 2.
"""

from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np
from scipy.special import ndtr

ADC_MAX = 16383
GAIN_LEVEL_CODES = (0, 1, 3)
GAIN_LEVEL_PROB = (0.95, 0.045, 0.005)


@dataclass(frozen=True)
class Geometry:
    """A flat detector normal to the beam, and its radial binning."""

    name: str
    config_id: int
    height: int
    width: int
    pixel_m: float
    dist_m: float
    centre_row: float
    centre_col: float
    wavelength_m: float
    n_bins: int
    split: str  # "none" or "bbox"
    normalised: bool  # True: norm = solid angle x polarisation; False: norm = 1
    raw: bool  # True: frames are raw Jungfrau words; False: float32 counts
    spots: tuple  # (min, max) Bragg spots per frame, inclusive
    mask_rows: tuple  # ((start, stop), ...) half-open masked row stripes
    mask_cols: tuple

    @property
    def n_pix(self) -> int:
        return self.height * self.width

    @property
    def shape(self):
        return (self.height, self.width)


# 8 float32 frames of 512x512, 256 bins, no pixel splitting, 30 spots/frame.
SMALL = Geometry(
    name="small-512", config_id=0, height=512, width=512, pixel_m=75e-6,
    dist_m=0.1, centre_row=256.3, centre_col=240.7, wavelength_m=1e-10,
    n_bins=256, split="none", normalised=False, raw=False, spots=(30, 30),
    mask_rows=((120, 133),), mask_cols=((380, 393),),
)

# 64 raw Jungfrau-4M frames of 2162x2068, 1000 bins, bbox splitting,
# 0-200 spots/frame.
JUNGFRAU4M = Geometry(
    name="jungfrau-4m", config_id=1, height=2162, width=2068, pixel_m=75e-6,
    dist_m=0.1, centre_row=1081.3, centre_col=1034.7, wavelength_m=1e-10,
    n_bins=1000, split="bbox", normalised=True, raw=True, spots=(0, 200),
    mask_rows=((514, 541), (1594, 1621)), mask_cols=((500, 526), (1540, 1566)),
)

# Further detector sizes used for mixed-geometry batches.
JUNGFRAU1M = Geometry(
    name="jungfrau-1m", config_id=2, height=1030, width=1065, pixel_m=75e-6,
    dist_m=0.1, centre_row=515.3, centre_col=532.7, wavelength_m=1e-10,
    n_bins=500, split="bbox", normalised=True, raw=True, spots=(0, 500),
    mask_rows=((514, 520),), mask_cols=((256, 262),),
)
JUNGFRAU16M = Geometry(
    name="jungfrau-16m", config_id=3, height=4150, width=4371, pixel_m=75e-6,
    dist_m=0.1, centre_row=2075.3, centre_col=2185.7, wavelength_m=1e-10,
    n_bins=2000, split="bbox", normalised=True, raw=True, spots=(0, 500),
    mask_rows=((1028, 1056), (3108, 3136)), mask_cols=((1030, 1058), (3300, 3328)),
)

JUNGFRAU9M = Geometry(
    name="jungfrau-9m", config_id=4, height=3114, width=3132, pixel_m=75e-6,
    dist_m=0.1, centre_row=1557.3, centre_col=1566.7, wavelength_m=1e-10,
    n_bins=1500, split="bbox", normalised=True, raw=True, spots=(0, 200),
    mask_rows=((1038, 1064), (2076, 2102)), mask_cols=((1044, 1070), (2088, 2114)),
)

GEOMETRIES = {g.name: g for g in (SMALL, JUNGFRAU4M, JUNGFRAU1M, JUNGFRAU16M, JUNGFRAU9M)}


def _rng(geom: Geometry, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([geom.config_id, stream]))


def stripe_mask(geom: Geometry) -> np.ndarray:
    """Static detector mask (module gaps) as uint8 [H, W], nonzero = masked."""
    m = np.zeros(geom.shape, dtype=np.uint8)
    for a, b in geom.mask_rows:
        m[a:b, :] = 1
    for a, b in geom.mask_cols:
        m[:, a:b] = 1
    return m


@functools.lru_cache(maxsize=8)
def _centre_offsets(geom: Geometry):
    dy = (np.arange(geom.height, dtype=np.float64) + 0.5 - geom.centre_row)[:, None]
    dx = (np.arange(geom.width, dtype=np.float64) + 0.5 - geom.centre_col)[None, :]
    return dy, dx


def scattering_angle_deg(geom: Geometry) -> np.ndarray:
    """Scattering angle of each pixel centre, float64 [H, W], degrees."""
    dy, dx = _centre_offsets(geom)
    r = np.hypot(dy, dx) * geom.pixel_m
    return np.degrees(np.arctan2(r, geom.dist_m))


def azimuth_rad(geom: Geometry) -> np.ndarray:
    dy, dx = _centre_offsets(geom)
    return np.arctan2(np.broadcast_to(dy, geom.shape), np.broadcast_to(dx, geom.shape))


@functools.lru_cache(maxsize=8)
def normalisation(geom: Geometry) -> np.ndarray:
    """Per-pixel normalisation factor, float32 [H, W] (read-only)."""
    if not geom.normalised:
        out = np.ones(geom.shape, dtype=np.float32)
    else:
        t = np.radians(scattering_angle_deg(geom))
        chi = azimuth_rad(geom)
        solid = np.cos(t) ** 3
        pol = 0.5 * (1.0 + np.cos(t) ** 2 - 0.99 * np.cos(2.0 * chi) * np.sin(t) ** 2)
        out = (solid * pol).astype(np.float32)
    out.setflags(write=False)
    return out


def background_counts(tth_deg: np.ndarray) -> np.ndarray:
    """Isotropic background in counts per pixel as a function of 2theta."""
    t = np.asarray(tth_deg, dtype=np.float64)
    return 150.0 * np.exp(-t / 8.0) + 400.0 * np.exp(-((t - 20.0) ** 2) / 8.0)


@functools.lru_cache(maxsize=8)
def _expected_background(geom: Geometry) -> np.ndarray:
    out = background_counts(scattering_angle_deg(geom)) * normalisation(geom)
    out.setflags(write=False)
    return out


def spot_expectation(rng: np.random.Generator, geom: Geometry, mask: np.ndarray,
                     n_spots: int, sigma_px: float = 1.2):
    """Expected counts of ``n_spots`` Gaussian spots, float64 [H, W], plus truth.

    Truth rows: (centre_row, centre_col, integral) in continuous pixel
    coordinates, where pixel (y, x) covers [y, y+1) x [x, x+1).
    """
    H, W = geom.shape
    img = np.zeros((H, W), dtype=np.float64)
    truth = []
    half = int(np.ceil(5 * sigma_px))
    while len(truth) < n_spots:
        cy = rng.uniform(0.0, H)
        cx = rng.uniform(0.0, W)
        if mask[int(cy), int(cx)]:
            continue
        integral = float(rng.lognormal(6.0, 1.0))
        y0, y1 = max(0, int(cy) - half), min(H, int(cy) + half + 1)
        x0, x1 = max(0, int(cx) - half), min(W, int(cx) + half + 1)
        ey = np.arange(y0, y1 + 1, dtype=np.float64)
        ex = np.arange(x0, x1 + 1, dtype=np.float64)
        py = np.diff(ndtr((ey - cy) / sigma_px))
        px = np.diff(ndtr((ex - cx) / sigma_px))
        img[y0:y1, x0:x1] += integral * py[:, None] * px[None, :]
        truth.append((cy, cx, integral))
    return img, np.array(truth, dtype=np.float64).reshape(-1, 3)


def _spot_count(rng: np.random.Generator, geom: Geometry) -> int:
    lo, hi = geom.spots
    return int(lo) if lo == hi else int(rng.integers(lo, hi + 1))


def _photons(geom: Geometry, frame_idx: int):
    rng = _rng(geom, frame_idx)
    mask = stripe_mask(geom)
    spots, truth = spot_expectation(rng, geom, mask, _spot_count(rng, geom))
    lam = _expected_background(geom) + spots
    return rng, rng.poisson(lam).astype(np.float64), truth


def float_frame(geom: Geometry, frame_idx: int):
    """One float32 frame of photon counts [H, W] and its spot truth."""
    _, counts, truth = _photons(geom, frame_idx)
    return counts.astype(np.float32), truth


def float_frames(geom: Geometry, n_frames: int, first: int = 0) -> np.ndarray:
    return np.stack([float_frame(geom, first + k)[0] for k in range(n_frames)])


@functools.lru_cache(maxsize=4)
def jungfrau_calibration(geom: Geometry):
    """Pedestals [3, N] (ADU) and gains [3, N] (ADU per photon), float32."""
    rng = _rng(geom, 999999)
    n = geom.n_pix
    ped = np.empty((3, n), dtype=np.float32)
    gain = np.empty((3, n), dtype=np.float32)
    ped[0] = rng.normal(1500.0, 40.0, n)
    ped[1] = rng.normal(2500.0, 60.0, n)
    ped[2] = rng.normal(3000.0, 80.0, n)
    g0 = rng.normal(20.0, 0.4, n)
    gain[0] = g0
    gain[1] = g0 / 10.0 * rng.normal(1.0, 0.01, n)
    gain[2] = g0 / 100.0 * rng.normal(1.0, 0.01, n)
    ped.setflags(write=False)
    gain.setflags(write=False)
    return ped, gain


def jungfrau_frame(geom: Geometry, frame_idx: int):
    """One raw Jungfrau frame uint16 [H, W] and its truth.

    Truth: dict(photons=float64 [H, W], level=int8 [H, W], spots=[n, 3]).
    """
    rng, photons, truth = _photons(geom, frame_idx)
    return _encode(geom, rng, photons, truth)


def training_frame(geom: Geometry, frame_idx: int):
    """One raw frame of the clip surrogate's training set, from a seed stream
    of its own (disjoint from ``jungfrau_frame``'s): the background ring
    scaled by U[0.5, 4]; a hit with probability h ~ U[0, 0.5], a hit holding
    1-500 spots (the spot model of the other frames)."""
    rng = np.random.default_rng(np.random.SeedSequence([geom.config_id, 1_000_000 + frame_idx]))
    ring = rng.uniform(0.5, 4.0)
    hit = rng.random() < rng.uniform(0.0, 0.5)
    n_spots = int(rng.integers(1, 501)) if hit else 0
    spots, truth = spot_expectation(rng, geom, stripe_mask(geom), n_spots)
    photons = rng.poisson(ring * _expected_background(geom) + spots).astype(np.float64)
    word, info = _encode(geom, rng, photons, truth)
    info.update(ring=ring, hit=hit)
    return word, info


def uneven_frame(geom: Geometry, frame_idx: int, hit_rate: float = 0.3, max_spots: int = 500):
    """One raw frame of the batched mixed-detector workload, from a seed
    stream of its own: a hit with probability ``hit_rate`` holding
    1..``max_spots`` spots, otherwise background only."""
    rng = np.random.default_rng(np.random.SeedSequence([geom.config_id, 2_000_000 + frame_idx]))
    n_spots = int(rng.integers(1, max_spots + 1)) if rng.random() < hit_rate else 0
    spots, truth = spot_expectation(rng, geom, stripe_mask(geom), n_spots)
    photons = rng.poisson(_expected_background(geom) + spots).astype(np.float64)
    return _encode(geom, rng, photons, truth)


def stored_sparse(geom: Geometry, frame_idx: int, kept_fraction: float = 0.02, empty_fraction: float = 0.05):
    """A stored sparse frame as densification reads it: a background profile
    (mean, std, member count per radial bin; about ``empty_fraction`` of the
    bins empty) and kept pixels (ascending unmasked indices, about
    ``kept_fraction`` of the pixels, with intensities well above the
    background).  Shapes only: the profile is a smooth decreasing curve with
    jitter, not the result of any statistics over a frame.
    Stream: ``[config_id, 3000000 + frame_idx]``.
    """
    rng = _rng(geom, 3_000_000 + frame_idx)
    nb = geom.n_bins
    r = np.arange(nb, dtype=np.float64) / nb
    mean = (40.0 * np.exp(-3.0 * r) + 2.0) * rng.uniform(0.97, 1.03, nb)
    std = np.sqrt(mean) * rng.uniform(0.8, 1.2, nb)
    members = rng.integers(20, 5000, nb).astype(np.int32)
    members[rng.random(nb) < empty_fraction] = 0
    members[:2] = 0  # the innermost bins (behind the beam stop) are empty
    ok = np.nonzero(stripe_mask(geom).reshape(-1) == 0)[0]
    n = int(round(kept_fraction * ok.size))
    idx = np.sort(rng.choice(ok, n, replace=False)).astype(np.int64)
    val = (mean.max() + rng.exponential(50.0, n)).astype(np.float32)
    return dict(mean=mean, std=std, n_members=members, kept_index=idx, kept_value=val)


def _encode(geom: Geometry, rng: np.random.Generator, photons: np.ndarray, truth):
    ped, gain = jungfrau_calibration(geom)
    e = photons.reshape(-1)
    u = rng.random(e.size)
    level = np.where(u < GAIN_LEVEL_PROB[0], 0,
                     np.where(u < GAIN_LEVEL_PROB[0] + GAIN_LEVEL_PROB[1], 1, 2)).astype(np.int8)
    for g in (0, 1):
        sat = (level == g) & (ped[g] + e * gain[g] > ADC_MAX)
        level[sat] = g + 1
    p = np.where(level == 0, ped[0], np.where(level == 1, ped[1], ped[2])).astype(np.float64)
    k = np.where(level == 0, gain[0], np.where(level == 1, gain[1], gain[2])).astype(np.float64)
    adc = np.clip(np.rint(p + e * k + rng.normal(0.0, 2.0, e.size)), 0, ADC_MAX).astype(np.uint16)
    code = np.asarray(GAIN_LEVEL_CODES, dtype=np.uint16)[level]
    word = (code << np.uint16(14)) | adc
    return word.reshape(geom.shape), dict(photons=photons, level=level.reshape(geom.shape), spots=truth)


def jungfrau_frames(geom: Geometry, n_frames: int, first: int = 0) -> np.ndarray:
    return np.stack([jungfrau_frame(geom, first + k)[0] for k in range(n_frames)])
