"""Tiled frame layouts on the GPU (ss_layout).

* ss_correct_tiled / ss_correct_indexed_tiled write exactly the row-major
  correction rearranged by the word formula of ss_layout (restated here),
  NaN at the words past the image edge, with the same invalid-word counts:
  vector path (width % 4 == 0, batches and one or two frames) and scalar
  path (odd width), partial tiles on both edges.
* The clip on tiled frames with the relaid CSR gives the row-major clip's
  statistics to float64 rounding (its rows are summed in another order),
  for the azimuthal and the Poisson model (whose norm is rearranged too).
* The whole path on tiled frames of the benchmark's batch (64 raw
  Jungfrau-4M frames) matches the FP64 oracle at the parity tolerance on
  sampled frames, like the row-major path.
* With the same profile the classification of tiled frames is the
  row-major one entry for entry (every threshold mode, unrolled and
  runtime patches)."""

import sys

import numpy as np
import pytest
import torch

import synth
from paper_2411_09515_amd import api

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _words_of(h, w, tw, th):
    """Word of every pixel y * w + x (the ss_layout formula)."""
    y, x = np.divmod(np.arange(h * w, dtype=np.int64), w)
    tiles_x = -(-w // tw)
    return ((y // th) * tiles_x + x // tw) * (tw * th) + (y % th) * tw + x % tw


def _raw_frames(rng, n, n_pix):
    adc = rng.integers(0, 1 << 14, size=(n, n_pix))
    code = rng.choice([0, 1, 3, 2], p=[0.9, 0.06, 0.03, 0.01], size=(n, n_pix))   # 2 = invalid
    return ((code << 14) | adc).astype(np.uint16)


@pytest.mark.parametrize("h,w,tile,n", [(37, 52, (8, 4), 5), (37, 52, (8, 4), 1), (37, 52, (4, 8), 2),
                                        (37, 53, (8, 4), 3), (64, 64, (16, 2), 4)])
def test_correct_tiled_is_the_rearranged_correction(dev, h, w, tile, n):
    _say(f"case: correct tiled {h}x{w} tiles {tile} frames {n}")
    rng = np.random.default_rng(h * 1000 + w + n)
    geo = api.Geometry(h, w, 75e-6, 0.1, h / 2 + 0.3, w / 2 - 0.2, 17, tile=tile, device=dev)
    raw = torch.from_numpy(_raw_frames(rng, n, h * w).view(np.int16)).to(dev)
    ped = torch.from_numpy(rng.uniform(900, 1100, (3, h * w)).astype(np.float32)).to(dev)
    gain = torch.from_numpy(rng.uniform(0.5, 50, (3, h * w)).astype(np.float32)).to(dev)
    norm = torch.from_numpy(rng.uniform(0.6, 1.4, h * w).astype(np.float32)).to(dev)
    flat, bad = api.correct(raw, ped, gain, norm)
    tiled, bad_t = api.correct(raw, ped, gain, norm, geom=geo)
    torch.cuda.synchronize()
    assert tiled.shape == (n, geo.frame_words)
    words = _words_of(h, w, *tile)
    t = tiled.cpu().numpy()
    assert np.array_equal(t[:, words].view(np.uint32), flat.cpu().numpy().view(np.uint32))
    edge = np.ones(geo.frame_words, dtype=bool)
    edge[words] = False
    assert edge.sum() == geo.frame_words - h * w and np.all(np.isnan(t[:, edge]))
    assert torch.equal(bad, bad_t)


def test_correct_indexed_tiled_is_the_rearranged_correction(dev):
    h, w, tile = 45, 68, (8, 4)
    _say(f"case: correct indexed tiled {h}x{w}")
    rng = np.random.default_rng(11)
    geo = api.Geometry(h, w, 75e-6, 0.1, 20.5, 30.5, 23, tile=tile, device=dev)
    ring = torch.from_numpy(_raw_frames(rng, 3, h * w).view(np.int16)).to(dev)
    ped = torch.from_numpy(rng.uniform(900, 1100, (3, h * w)).astype(np.float32)).to(dev)
    gain = torch.from_numpy(rng.uniform(0.5, 50, (3, h * w)).astype(np.float32)).to(dev)
    idx = torch.tensor([2, 0, 5, 1], dtype=torch.int64, device=dev)                 # 5: outside the ring
    flat, bad = api.correct_indexed(ring, idx, ped, gain)
    tiled, bad_t = api.correct_indexed(ring, idx, ped, gain, geom=geo)
    torch.cuda.synchronize()
    words = _words_of(h, w, *tile)
    assert np.array_equal(tiled.cpu().numpy()[:, words].view(np.uint32), flat.cpu().numpy().view(np.uint32))
    assert torch.equal(bad, bad_t) and int(bad_t[2]) == h * w


@pytest.mark.parametrize("model", ["azimuthal", "poisson"])
def test_clip_on_tiled_frames_matches_row_major(dev, model):
    g = synth.SMALL
    _say(f"case: clip on tiled frames, small-512 x8, {model}")
    norm = np.random.default_rng(5).uniform(0.6, 1.4, (g.height, g.width)).astype(np.float32)
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), norm, dev)
    geo_t = api.Geometry.from_scene(g, synth.stripe_mask(g), norm, dev, tile=(8, 4))
    frames = torch.from_numpy(synth.float_frames(g, 8).reshape(8, -1)).to(dev)
    words = torch.from_numpy(_words_of(g.height, g.width, 8, 4)).to(dev)
    frames_t = torch.full((8, geo_t.frame_words), float("nan"), device=dev)
    frames_t[:, words] = frames
    p = api.Params(error_model=model)
    ref = api.sigma_clip(frames, geo, p)
    got = api.sigma_clip(frames_t, geo_t, p)
    torch.cuda.synchronize()
    same = got["n_members"] == ref["n_members"]
    assert same.float().mean().item() >= 0.999          # decisions at a threshold within rounding may differ
    for k in ("mean", "std", "sem", "sum_w"):
        a, b = got[k][same], ref[k][same]
        assert torch.all((a - b).abs() <= 1e-9 * b.abs() + 1e-12), k


@pytest.fixture(scope="module")
def tiled_batch(dev):
    from parity import OracleScene
    g = synth.JUNGFRAU4M
    _say("setup: 16 distinct jungfrau-4m frames x4, tiled 8 x 4 geometry, oracle scene")
    distinct = synth.jungfrau_frames(g, 16).reshape(16, -1)
    raw = np.concatenate([distinct] * 4)
    sc = OracleScene(g)
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev, tile=(8, 4))
    ped, gain = (torch.from_numpy(np.array(a)).to(dev) for a in synth.jungfrau_calibration(g))
    p = api.Params()
    pipe = api.Pipeline(geo, p, 64, ped, gain, kept_capacity=1 << 18, peak_capacity=1 << 13, device=dev)
    _say("case: whole path on 64 tiled frames")
    out = pipe.run(torch.from_numpy(raw).to(dev))
    torch.cuda.synchronize()
    return g, sc, raw, pipe, out, p


@pytest.mark.parametrize("f", [0, 37, 63])
def test_tiled_path_matches_oracle(dev, tiled_batch, f):
    from test_gpu_parity import _check_classify
    g, sc, raw, pipe, out, p = tiled_batch
    _say(f"case: tiled 64-frame batch, frame {f} vs oracle")
    signal, _ = sc.signal_from_raw(raw[f:f + 1])
    words = _words_of(g.height, g.width, 8, 4)
    got = pipe.frames[f].cpu().numpy()[words]
    assert np.array_equal(got.view(np.uint32), sc.corrected(signal)[0].view(np.uint32))
    _check_classify(sc, signal[0], pipe.profile, f, out, p, f"tiled batch frame {f}")


@pytest.mark.parametrize("params", [
    dict(),
    dict(n_pick=1.0, snr=2.0, patch=5, min_count=4),
    dict(n_pick=2.0, noise=1.0, patch=1, min_count=1),
    dict(snr=-2.0, patch=7, min_count=3),
    dict(n_pick=2.5, snr=2.5, patch=15, min_count=2),
])
def test_classify_on_tiled_frames_is_the_row_major_classification(dev, params):
    """Same profile, same pixels: the classification of tiled frames (staged
    tile by tile) is the row-major one, entry for entry, for one and two
    threshold lines, a noise level, and unrolled and runtime patches."""
    g = synth.SMALL
    _say("case: classify on tiled frames, small-512 x8", params)
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev)
    geo_t = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev, tile=(8, 4))
    frames = torch.from_numpy(synth.float_frames(g, 8).reshape(8, -1)).to(dev)
    words = torch.from_numpy(_words_of(g.height, g.width, 8, 4)).to(dev)
    frames_t = torch.full((8, geo_t.frame_words), float("nan"), device=dev)
    frames_t[:, words] = frames
    p = api.Params(**params)
    prof = api.sigma_clip(frames, geo, p)
    n_pix = g.height * g.width
    ref = api.classify(frames, geo, prof, p, capacity=n_pix, peak_capacity=n_pix)
    got = api.classify(frames_t, geo_t, prof, p, capacity=n_pix, peak_capacity=n_pix)
    torch.cuda.synchronize()
    assert torch.equal(got["n_kept"], ref["n_kept"]) and torch.equal(got["n_peaks"], ref["n_peaks"])
    assert int(ref["n_peaks"].sum()) > 0
    for f in range(8):
        k, q = int(ref["n_kept"][f]), int(ref["n_peaks"][f])
        assert torch.equal(got["kept_index"][f, :k], ref["kept_index"][f, :k])
        assert torch.equal(got["kept_value"][f, :k].view(torch.int32), ref["kept_value"][f, :k].view(torch.int32))
        assert torch.equal(got["peaks"][f, :q], ref["peaks"][f, :q])
