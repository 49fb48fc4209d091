"""Pixel scattering angles and the CSR pixel-to-bin matrix (FP64).

Sec. 2.2 "Azimuthal averaging": the regrouping of pixels into radial bins is a
linear map, stored as a compressed-sparse-row matrix whose rows are bins and
whose coefficient c[i, r] is the fraction of pixel i falling into bin r; with
pixel splitting disabled every coefficient is 1 and each pixel lands in one
bin.  The paper fixes neither the radial unit, the bin edges nor the splitting
rule; the readings used here:

* a flat detector normal to the beam; pixel (y, x) covers the square
  [y, y+1) x [x, x+1) in pixel units and its centre is (y + 1/2, x + 1/2);
  the beam centre (cy, cx) is given in the same coordinates;
* radial coordinate 2theta in degrees, 2theta = atan(pixel * r / distance);
* bins uniform on [0, 2theta_max], where 2theta_max is the largest corner
  angle over all pixels (independent of the mask); bin r is
  [r w, (r+1) w), the last bin closed at 2theta_max, centre (r + 1/2) w;
* no splitting: a pixel goes to the bin holding its centre angle, c = 1;
* bounding-box splitting: a pixel spans the 1-D interval [lo, hi] between
  the smallest and largest of its four corner angles (lo = 0 for the pixel
  holding the beam centre); c[i, r] is the length of the overlap of that
  interval with bin r divided by hi - lo, and zero overlaps are dropped, so
  the coefficients of an unmasked pixel sum to 1;
* masked pixels contribute no entries; within a row, entries are in
  ascending pixel index (row-major y * W + x).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Csr:
    n_bins: int
    n_pix: int
    indptr: np.ndarray  # int64 [n_bins + 1]
    indices: np.ndarray  # int64 [nnz], pixel index
    coef: np.ndarray  # float64 [nnz], c[i, r]
    tth_max: float  # degrees
    width: float  # bin width, degrees

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    @property
    def centres(self) -> np.ndarray:
        return (np.arange(self.n_bins, dtype=np.float64) + 0.5) * self.width

    def row(self, r: int):
        a, b = self.indptr[r], self.indptr[r + 1]
        return self.indices[a:b], self.coef[a:b]


def _angle_deg(dy, dx, pixel_m, dist_m):
    r = np.sqrt(dy * dy + dx * dx) * pixel_m
    return np.arctan(r / dist_m) * (180.0 / np.pi)


def centre_angle(height, width, pixel_m, dist_m, cy, cx) -> np.ndarray:
    """2theta of every pixel centre, float64 [H*W], degrees."""
    dy = np.arange(height, dtype=np.float64)[:, None] + 0.5 - cy
    dx = np.arange(width, dtype=np.float64)[None, :] + 0.5 - cx
    return _angle_deg(dy, dx, pixel_m, dist_m).reshape(-1)


def corner_angle(height, width, pixel_m, dist_m, cy, cx) -> np.ndarray:
    """2theta of every pixel corner, float64 [H+1, W+1], degrees."""
    dy = np.arange(height + 1, dtype=np.float64)[:, None] - cy
    dx = np.arange(width + 1, dtype=np.float64)[None, :] - cx
    return _angle_deg(dy, dx, pixel_m, dist_m)


def build_csr(height, width, pixel_m, dist_m, cy, cx, n_bins, split, mask=None) -> Csr:
    """CSR matrix of the radial regrouping (rows = bins)."""
    n_pix = height * width
    corners = corner_angle(height, width, pixel_m, dist_m, cy, cx)
    tth_max = float(corners.max())
    w = tth_max / n_bins
    valid = np.ones(n_pix, dtype=bool) if mask is None else (np.asarray(mask).reshape(-1) == 0)
    pix = np.arange(n_pix, dtype=np.int64)

    if split == "none":
        tc = centre_angle(height, width, pixel_m, dist_m, cy, cx)
        b = np.minimum(np.floor(tc / w).astype(np.int64), n_bins - 1)
        rows, cols, vals = b[valid], pix[valid], np.ones(int(valid.sum()))
    elif split == "bbox":
        c4 = np.stack([corners[:-1, :-1], corners[:-1, 1:], corners[1:, :-1], corners[1:, 1:]])
        lo = c4.min(axis=0).reshape(-1)
        hi = c4.max(axis=0).reshape(-1)
        # the pixel that holds the beam centre reaches 2theta = 0
        yc, xc = int(np.floor(cy)), int(np.floor(cx))
        if 0 <= yc < height and 0 <= xc < width:
            lo[yc * width + xc] = 0.0
        span = hi - lo
        first = np.floor(lo / w).astype(np.int64) - 1
        last = np.floor(hi / w).astype(np.int64) + 1
        rows, cols, vals = [], [], []
        for k in range(int((last - first).max()) + 1):
            r = first + k
            ok = valid & (r >= 0) & (r < n_bins) & (r <= last)
            rr = np.where(ok, r, 0)
            lower = rr * w
            upper = np.where(rr == n_bins - 1, tth_max, (rr + 1) * w)
            overlap = np.minimum(hi, upper) - np.maximum(lo, lower)
            ok &= overlap > 0
            rows.append(rr[ok])
            cols.append(pix[ok])
            vals.append(overlap[ok] / span[ok])
        rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    else:
        raise ValueError(f"unknown split {split!r}")

    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    indptr = np.zeros(n_bins + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_bins), out=indptr[1:])
    return Csr(n_bins, n_pix, indptr, cols.astype(np.int64), vals.astype(np.float64), tth_max, w)


def csr_for(geom, mask=None) -> Csr:
    """Convenience: the CSR of a ``synth`` geometry description."""
    return build_csr(geom.height, geom.width, geom.pixel_m, geom.dist_m,
                     geom.centre_row, geom.centre_col, geom.n_bins, geom.split, mask)


def position_for(geom) -> np.ndarray:
    return centre_angle(geom.height, geom.width, geom.pixel_m, geom.dist_m,
                        geom.centre_row, geom.centre_col)
