"""Densification and the peak-count veto, HIP path vs the FP64 oracle, through
the C ABI.

Inputs: stored sparse frames from ``synth.stored_sparse`` (a profile and kept
pixels), the same bytes on both sides.

Tolerances (derived from the arithmetic):
* background: the kernel reads a pixel's position as a 20-bit fraction of the
  interval between bin centres, so mu (sigma) may differ by 2^-20 of the
  largest step of the profile's mean (std) between neighbouring non-empty
  bins; rounding the float64 background to float32 adds at most one float32
  ulp (2^-23 relative);
* noise: Box-Muller in float32 (log, sqrt, sincospi of exact 24-bit
  uniforms) differs from float64 by at most 4e-6 (1 + |z|) in z
  (r <= 5.8); a pixel whose oracle normal lies within 1e-5 of the
  truncation point may take the other branch and is excused;
* kept pixels, masked pixels and the veto: bit for bit.
"""

import sys

import numpy as np
import pytest
import torch

import synth
from oracle import classify as OK
from oracle import geometry as OG
from oracle import rng as OR
from paper_2411_09515_amd import api
from paper_2411_09515_amd import binding as B

from parity import OracleScene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def scene(dev):
    g = synth.SMALL
    sc = OracleScene(g)
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), None, dev)
    stored = [synth.stored_sparse(g, k) for k in range(3)]
    return g, sc, geo, stored


def _device_inputs(stored, dev, cap=None):
    F = len(stored)
    nb = stored[0]["mean"].size
    cap = cap or max(s["kept_index"].size for s in stored)
    ki = np.zeros((F, cap), dtype=np.int32)
    kv = np.zeros((F, cap), dtype=np.float32)
    nk = np.zeros(F, dtype=np.int64)
    for f, s in enumerate(stored):
        n = s["kept_index"].size
        ki[f, :min(n, cap)] = s["kept_index"][:cap]
        kv[f, :min(n, cap)] = s["kept_value"][:cap]
        nk[f] = n
    prof = dict(mean=torch.from_numpy(np.stack([s["mean"] for s in stored])).to(dev),
                std=torch.from_numpy(np.stack([s["std"] for s in stored])).to(dev),
                n_members=torch.from_numpy(np.stack([s["n_members"] for s in stored])).to(dev))
    sparse = dict(kept_index=torch.from_numpy(ki).to(dev), kept_value=torch.from_numpy(kv).to(dev),
                  n_kept=torch.from_numpy(nk).to(dev))
    assert prof["mean"].shape == (F, nb)
    return sparse, prof


def _steps(s):
    ne = s["n_members"] > 0
    return np.abs(np.diff(s["mean"][ne])).max(), np.abs(np.diff(s["std"][ne])).max()


def _oracle_prof(s):
    return dict(mean=s["mean"], std=s["std"], n_members=s["n_members"])


def test_densify_noise_free_matches_oracle(dev, scene):
    g, sc, geo, stored = scene
    _say("case: densify noise free, small-512 x3")
    sparse, prof = _device_inputs(stored, dev)
    dense = api.densify(sparse, geo, prof).cpu().numpy()
    for f, s in enumerate(stored):
        ref = OK.densify(s["kept_index"], s["kept_value"].astype(np.float64), g.n_pix, sc.mask, sc.position,
                         sc.centres, _oracle_prof(s))
        dm, _ = _steps(s)
        tol = 2.0 ** -19 * dm + 2.0 ** -23 * np.abs(ref)
        assert np.all(np.abs(dense[f] - ref) <= tol), (f, np.max(np.abs(dense[f] - ref) - tol))
        assert np.array_equal(dense[f][s["kept_index"]], s["kept_value"])
        assert np.all(dense[f][sc.mask != 0] == 0.0)


@pytest.mark.parametrize("trunc", [3.0, float("inf")])
def test_densify_noisy_matches_oracle(dev, scene, trunc):
    g, sc, geo, stored = scene
    _say(f"case: densify with noise, trunc {trunc}")
    sparse, prof = _device_inputs(stored, dev)
    seed, frame0 = 0x1234_5678_9ABC_DEF0, 7
    dense = api.densify(sparse, geo, prof, noise=dict(seed=seed, frame0=frame0, trunc=trunc)).cpu().numpy()
    for f, s in enumerate(stored):
        ref = OK.densify_noisy(s["kept_index"], s["kept_value"].astype(np.float64), g.n_pix, sc.mask,
                               sc.position, sc.centres, _oracle_prof(s), seed, frame0 + f, trunc)
        za, zb = OR.pixel_normals(seed, frame0 + f, g.n_pix)
        z = OR.truncated(za, zb, trunc)
        mu, sd = OK.background_at(sc.position, sc.centres, _oracle_prof(s))
        dm, ds = _steps(s)
        tol = (2.0 ** -19 * (dm + ds * np.abs(z)) + 4e-6 * (1 + np.abs(z)) * sd
               + 2.0 ** -22 * (np.abs(mu) + sd * np.abs(z)))
        band = (np.abs(za - trunc) < 1e-5) | (np.abs(zb - trunc) < 1e-5)
        bad = (np.abs(dense[f] - ref) > tol) & ~band
        assert not bad.any(), (f, np.nonzero(bad)[0][:5], dense[f][bad][:5], ref[bad][:5])
        assert np.array_equal(dense[f][s["kept_index"]], s["kept_value"])
        assert np.all(dense[f][sc.mask != 0] == 0.0)
        if np.isfinite(trunc):
            bg = np.ones(g.n_pix, dtype=bool)
            bg[s["kept_index"]] = False
            bg &= sc.mask == 0
            assert np.all(dense[f][bg] <= (mu + trunc * sd)[bg] * (1 + 1e-6) + 1e-5)


def test_noise_depends_on_absolute_frame_only(dev, scene):
    """Densifying frames 1..2 with frame0 + 1 reproduces them bit for bit."""
    g, sc, geo, stored = scene
    _say("case: densify noise, batch independence")
    sparse, prof = _device_inputs(stored, dev)
    nz = dict(seed=99, frame0=10, trunc=3.0)
    full = api.densify(sparse, geo, prof, noise=nz)
    part = api.densify({k: v[1:].contiguous() for k, v in sparse.items()}, geo,
                       {k: v[1:].contiguous() for k, v in prof.items()}, noise=dict(nz, frame0=11))
    assert torch.equal(full[1:], part)


def test_densify_edge_cases(dev, scene):
    g, sc, geo, stored = scene
    _say("case: densify edge cases")
    sparse, prof = _device_inputs(stored, dev)
    # background only (capacity 0)
    bg = api.densify(None, geo, prof, n_frames=3)
    full = api.densify(sparse, geo, prof)
    keep = torch.zeros_like(full, dtype=torch.bool)
    for f, s in enumerate(stored):
        keep[f, torch.from_numpy(s["kept_index"]).to(dev)] = True
    assert torch.equal(bg[~keep], full[~keep])
    # capacity below n_kept: only the first `cap` entries return
    cap = 1000
    sp2, _ = _device_inputs(stored, dev, cap=cap)
    part = api.densify(sp2, geo, prof).cpu().numpy()
    for f, s in enumerate(stored):
        assert np.array_equal(part[f][s["kept_index"][:cap]], s["kept_value"][:cap])
        rest = s["kept_index"][cap:]
        assert np.array_equal(part[f][rest], bg[f].cpu().numpy()[rest])
    # zero frames and errors
    out0 = api.densify({k: v[:0] for k, v in sparse.items()}, geo, {k: v[:0] for k, v in prof.items()})
    assert out0.shape == (0, g.n_pix)
    with pytest.raises(B.SigsepError):
        api.densify(sparse, geo, prof, noise=dict(seed=1, trunc=float("nan")))


def test_densify_ragged_frame(dev):
    """A 7 x 9 detector: no 16-byte stores, a ragged last thread."""
    _say("case: densify ragged 7x9")
    geo = api.Geometry(7, 9, 75e-6, 0.01, 3.2, 4.1, 6, split="none", device=dev)
    rc = geo.radial()
    nb = geo.n_bins
    prof = dict(mean=torch.linspace(1, 6, nb, dtype=torch.float64, device=dev)[None].contiguous(),
                std=torch.full((1, nb), 0.5, dtype=torch.float64, device=dev),
                n_members=torch.full((1, nb), 3, dtype=torch.int32, device=dev))
    a = api.densify(None, geo, prof, n_frames=1, noise=dict(seed=5, trunc=2.0))
    b = api.densify(None, geo, prof, n_frames=1, noise=dict(seed=5, trunc=2.0))
    assert torch.equal(a, b) and rc.n_bins == nb
    csr = OG.build_csr(7, 9, 75e-6, 0.01, 3.2, 4.1, nb, "none")
    pos = OG.centre_angle(7, 9, 75e-6, 0.01, 3.2, 4.1).reshape(-1)
    hp = {k: v[0].cpu().numpy() for k, v in prof.items()}
    ref = OK.densify_noisy(np.zeros(0, np.int64), np.zeros(0), 63, None, pos, csr.centres, hp, 5, 0, 2.0)
    za, zb = OR.pixel_normals(5, 0, 63)
    z = OR.truncated(za, zb, 2.0)
    tol = 2.0 ** -19 * 5.0 / (nb - 1) + 4e-6 * (1 + np.abs(z)) * 0.5 + 2.0 ** -22 * (6 + 0.5 * np.abs(z))
    band = (np.abs(za - 2.0) < 1e-5) | (np.abs(zb - 2.0) < 1e-5)
    assert np.all((np.abs(a[0].cpu().numpy() - ref) <= tol) | band)


def test_veto_matches_oracle(dev):
    _say("case: veto counters, two calls")
    rng = np.random.default_rng(21)
    calls = [(rng.poisson(18, 3000), rng.integers(0, 20000, 3000)), (rng.integers(-2, 400, 777), None)]
    counters = api.new_veto_counters(dev)
    tot = dict(hits=0, misses=0, kept_hits=0, kept_misses=0,
               hist_frames=np.zeros(B.SS_VETO_BINS, np.int64), hist_kept=np.zeros(B.SS_VETO_BINS, np.int64))
    for n_peaks, n_kept in calls:
        nk = None if n_kept is None else torch.from_numpy(n_kept.astype(np.int64)).to(dev)
        hit, counters = api.veto(torch.from_numpy(n_peaks.astype(np.int64)).to(dev), 20, nk, counters)
        ref = OK.veto(n_peaks, np.zeros_like(n_peaks) if n_kept is None else n_kept, 20, B.SS_VETO_BINS)
        assert np.array_equal(hit.cpu().numpy().astype(bool), ref["hit"])
        for k in tot:
            tot[k] = tot[k] + ref[k]
    got = api.veto_summary(counters)
    for k in tot:
        assert np.array_equal(np.asarray(got[k]), np.asarray(tot[k])), k
