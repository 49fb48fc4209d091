"""Per-bin weighted statistics and iterative sigma-clipping (FP64).

Sec. 2.2 defines, for the members of one radial bin (pixel i with CSR
coefficient c and normalisation norm_i).  The frames handed to these
functions hold the pre-processed ``signal`` of eq. norm (the numerator: raw
minus dark, a 32-bit value per pixel, Sec. 1.2); every quantity below is
formed from it and from ``norm`` in float64:

  weight       omega_i = c * norm_i                          (eq. omega)
  value        v_i = signal_i / norm_i                       (eq. norm)
  Omega        = sum c norm_i,  OmegaOmega = sum omega_i^2  (eqs. omega, omegaomega)
  V            = sum c signal_i                              (eqs. avg, Vp)
  mean <I>     = V / Omega                                   (eqs. avg, weighted_avg)
  VV           = sum omega_i^2 (v_i - <I>)^2                 (eq. VVp, second pass)
  std^2        = VV / OmegaOmega                             (eqs. varA, std2)
  sem^2        = VV / Omega^2                                (eqs. varB, sem2)

The paper's own GPU merge of partial VV values is approximate; the oracle
uses the two-pass definition, never a merge.

Poisson error model (eqs. poisson, varianceP, sem).  Reading: the variance of
a pixel's signal is sigma_i^2 = max(signal_i, 0) + sigma_dark^2 and the
bin's pixel std is sqrt(sum c^2 sigma_i^2 / sum c^2 norm_i^2); the literal
denominator of eq. varianceP (sum c norm) only matches that when norm = 1,
and this form is the one consistent with eq. sem and with the two-pixel
example of Sec. 2.5 (values 1 and 199: std close to 10).  sem = sqrt(sum c^2
sigma^2) / Omega.  The hybrid model (Sec. 2.5) clips with the azimuthal std
and reports the Poisson std of the final set.

Sigma-clipping (eq. clip, Sec. 2.4), reading of the iteration:
  E_0 = all members (unmasked, finite signal);
  for k = 0 .. K-1:
      stats of E_k;  n_k = cut-off (or Chauvenet's value for |E_k|);
      D_k = members of E_k with |v - mean_k| > n_k * std_k (strict, two-sided);
      stop if D_k is empty;  E_{k+1} = E_k minus D_k;
  the reported statistics are those of the final set.
``n_iter`` counts the passes that removed something; ``converged`` is 1 when
the loop stopped because a pass removed nothing.  A set with std = 0 removes
nothing.  An empty set has mean = std = sem = 0.

Chauvenet (eq. chauvenet): n = sqrt(2 ln(size / sqrt(2 pi))) with the natural
logarithm and size = |E_k|; when size <= sqrt(2 pi) nothing is removed.
"""

from __future__ import annotations

import math
from typing import NamedTuple

import numpy as np

AZIMUTHAL, POISSON, HYBRID = 0, 1, 2
SQRT_2PI = math.sqrt(2.0 * math.pi)


def chauvenet(size) -> float:
    """Chauvenet cut-off for an ensemble of ``size`` members; inf if none applies."""
    if size <= SQRT_2PI:
        return math.inf
    return math.sqrt(2.0 * math.log(size / SQRT_2PI))


def moments(v, omega, pvar=None, csig=None):
    """Weighted statistics of one member set (two-pass).

    v: values signal/norm; omega: weights c*norm; pvar: optional c^2 sigma^2
    per member (Poisson numerator terms); csig: optional c*signal per member,
    whose sum is V of eq. avg (without it V = sum omega v, the same sum).
    Returns a dict of float64.
    """
    v = np.asarray(v, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    out = dict(n=int(v.size), Omega=0.0, OmegaOmega=0.0, V=0.0, VV=0.0,
               mean=0.0, std=0.0, sem=0.0, std_p=0.0, sem_p=0.0)
    if v.size == 0:
        return out
    Omega = float(np.sum(omega))
    OO = float(np.sum(omega * omega))
    V = float(np.sum(omega * v)) if csig is None else float(np.sum(np.asarray(csig, dtype=np.float64)))
    mean = V / Omega
    VV = float(np.sum(omega * omega * (v - mean) ** 2))
    out.update(Omega=Omega, OmegaOmega=OO, V=V, VV=VV, mean=mean,
               std=math.sqrt(VV / OO), sem=math.sqrt(VV) / Omega)
    if pvar is not None:
        S = float(np.sum(np.asarray(pvar, dtype=np.float64)))
        out.update(std_p=math.sqrt(S / OO), sem_p=math.sqrt(S) / Omega)
    return out


class Members(NamedTuple):
    """The members of one bin in one frame, aligned arrays (float64)."""

    pix: np.ndarray    # pixel index
    c: np.ndarray      # CSR coefficient c[i, r]
    v: np.ndarray      # signal / norm
    omega: np.ndarray  # c * norm
    pvar: np.ndarray   # c^2 sigma^2, sigma^2 = max(signal, 0) + sigma_dark^2
    csig: np.ndarray   # c * signal


def bin_members(signal, norm, csr, r, mask=None, dark_var=0.0) -> Members:
    """Members of bin r for one frame.

    signal: the pre-processed frame (numerator of eq. norm); norm: the
    normalisation per pixel, or None for 1.  A pixel is a member when it is
    not masked and its signal is finite.
    """
    pix, c = csr.row(r)
    s = signal[pix].astype(np.float64)
    nr = np.ones(pix.size) if norm is None else norm[pix].astype(np.float64)
    ok = np.isfinite(s)
    if mask is not None:
        ok &= mask[pix] == 0
    pix, c, s, nr = pix[ok], c[ok], s[ok], nr[ok]
    var = np.maximum(s, 0.0) + dark_var
    return Members(pix, c, s / nr, c * nr, c * c * var, c * s)


def _clip_bin(v, omega, pvar, cutoff, max_iter, model, csig=None):
    keep = np.ones(v.size, dtype=bool)
    n_iter, converged, margin = 0, 0, np.inf
    for _ in range(max_iter):
        m = moments(v[keep], omega[keep], pvar[keep], None if csig is None else csig[keep])
        n = cutoff if cutoff > 0 else chauvenet(int(keep.sum()))
        spread = m["std_p"] if model == POISSON else m["std"]
        thr = n * spread
        dev = np.abs(v - m["mean"])
        if keep.any() and np.isfinite(thr) and thr > 0:
            margin = min(margin, float(np.min(np.abs(dev[keep] - thr))) / thr)
        drop = keep & (dev > thr)
        if not drop.any():
            converged = 1
            break
        keep &= ~drop
        n_iter += 1
    return keep, n_iter, converged, margin


def sigma_clip(signal, norm, csr, mask=None, cutoff=3.0, max_iter=5,
               error_model=AZIMUTHAL, dark_var=0.0, return_keep=False, return_margin=False):
    """Sigma-clipped profile of one frame (max_iter = 0 gives the plain average).

    signal: the pre-processed frame, float [N] (NaN = invalid); norm: float
    [N] or None (= 1): v = signal / norm, weights c * norm, Poisson variance.
    With ``return_margin`` also ``margin``: per bin, the smallest relative
    distance | |v - mean_k| - n_k std_k | / (n_k std_k) of any member to the
    threshold over the passes run (inf when no pass compared anything); it
    marks bins whose clip decisions sit on the threshold within rounding.
    Returns dict of per-bin arrays: mean, std, sem, sum_w (Omega), n_members,
    n_iter, converged; with ``return_keep`` also the per-entry kept flags of
    every bin (list of bool arrays aligned with the members of that bin).
    """
    nb = csr.n_bins
    signal = np.asarray(signal).reshape(-1)
    norm = None if norm is None else np.asarray(norm).reshape(-1)
    mask = None if mask is None else np.asarray(mask).reshape(-1)
    out = dict(mean=np.zeros(nb), std=np.zeros(nb), sem=np.zeros(nb), sum_w=np.zeros(nb),
               n_members=np.zeros(nb, dtype=np.int64), n_iter=np.zeros(nb, dtype=np.int64),
               converged=np.zeros(nb, dtype=np.int64))
    keeps = []
    margins = np.full(nb, np.inf)
    for r in range(nb):
        mb = bin_members(signal, norm, csr, r, mask, dark_var)
        keep, n_iter, conv, margins[r] = _clip_bin(mb.v, mb.omega, mb.pvar, cutoff, max_iter, error_model, mb.csig)
        m = moments(mb.v[keep], mb.omega[keep], mb.pvar[keep], mb.csig[keep])
        poisson_report = error_model in (POISSON, HYBRID)
        out["mean"][r] = m["mean"]
        out["std"][r] = m["std_p"] if poisson_report else m["std"]
        out["sem"][r] = m["sem_p"] if poisson_report else m["sem"]
        out["sum_w"][r] = m["Omega"]
        out["n_members"][r] = m["n"]
        out["n_iter"][r] = n_iter
        out["converged"][r] = conv
        if return_keep:
            keeps.append((mb.pix, keep))
    if return_keep:
        out["keep"] = keeps
    if return_margin:
        out["margin"] = margins
    return out


def integrate(signal, norm, csr, mask=None, error_model=AZIMUTHAL, dark_var=0.0):
    """Azimuthal average with uncertainties, no clipping (eqs. avg .. sem2)."""
    return sigma_clip(signal, norm, csr, mask, cutoff=3.0, max_iter=0,
                      error_model=error_model, dark_var=dark_var)
