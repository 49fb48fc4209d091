"""HIP path vs FP64 oracle, element by element, through the C ABI.

Every case builds its inputs from the seeded ``synth`` generators; the GPU
side uses the library's own geometry builder, the oracle its own.
"""

import sys

import numpy as np
import pytest
import torch

import synth
from oracle import correct as OC
from oracle import stats as OS
from paper_2411_09515_amd import api
from paper_2411_09515_amd import binding as B

import parity as P
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
def small(dev):
    g = synth.SMALL
    sc = OracleScene(g)
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), None, dev)
    frames = synth.float_frames(g, 8)
    return g, sc, geo, frames.reshape(8, -1)


@pytest.fixture(scope="module")
def jungfrau(dev):
    g = synth.JUNGFRAU4M
    sc = OracleScene(g)
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev)
    raw = synth.jungfrau_frames(g, 3, first=5)
    ped, gain = (np.array(a) for a in synth.jungfrau_calibration(g))
    return g, sc, geo, raw.reshape(3, -1), ped, gain


def _prof_host(prof, f):
    return {k: v[f].cpu().numpy() for k, v in prof.items()}


# -- correction ----------------------------------------------------------------------

def test_correct_every_word_bit_exact(dev):
    _say("case: correct, all 65536 words")
    n = 1 << 16
    rng = np.random.default_rng(11)
    raw = np.arange(n, dtype=np.uint16)[None, :]
    ped = rng.normal([[1500.0], [2500.0], [3000.0]], 40.0, (3, n)).astype(np.float32)
    gain = (rng.normal(20.0, 0.4, n)[None, :] * np.array([[1.0], [0.1], [0.01]])).astype(np.float32)
    norm = rng.uniform(0.2, 1.0, n).astype(np.float32)
    out, n_bad = api.correct(torch.from_numpy(raw).to(dev), torch.from_numpy(ped).to(dev),
                             torch.from_numpy(gain).to(dev), torch.from_numpy(norm).to(dev))
    got = out.cpu().numpy()[0]
    sig, bad = OC.correct(raw, ped, gain)
    want = OC.normalise(sig[0], norm)
    assert np.array_equal(np.isnan(got), bad[0])
    assert np.array_equal(got[~bad[0]].view(np.uint32), want[~bad[0]].view(np.uint32))
    assert int(n_bad.cpu()[0]) == n // 4


def test_correct_jungfrau_frames_bit_exact(dev, jungfrau):
    g, sc, geo, raw, ped, gain = jungfrau
    _say("case: correct, jungfrau-4m x3")
    raw = raw.copy()
    raw[1, 12345:12345 + 77] = (2 << 14) | 1000  # invalid gain code in frame 1
    out, n_bad = api.correct(torch.from_numpy(raw).to(dev), torch.from_numpy(ped).to(dev),
                             torch.from_numpy(gain).to(dev), geo.norm)
    got = out.cpu().numpy()
    sig, bad = sc.signal_from_raw(raw)
    want = sc.corrected(sig)
    assert n_bad.cpu().tolist() == [0, 77, 0]
    assert np.array_equal(np.isnan(got), bad)
    assert np.array_equal(got[~bad].view(np.uint32), want[~bad].view(np.uint32))


@pytest.mark.parametrize("n", [1, 2])
def test_correct_few_frames_bit_exact(dev, jungfrau, n):
    """One or two frames take the per-word calibration path."""
    g, sc, geo, raw, ped, gain = jungfrau
    _say("case: correct, jungfrau-4m, frames", n)
    raw = raw[:n].copy()
    raw[n - 1, 4321:4321 + 13] = (2 << 14) | 700  # invalid gain code
    out, n_bad = api.correct(torch.from_numpy(raw).to(dev), torch.from_numpy(ped).to(dev),
                             torch.from_numpy(gain).to(dev), geo.norm)
    got = out.cpu().numpy()
    sig, bad = sc.signal_from_raw(raw)
    want = sc.corrected(sig)
    assert n_bad.cpu().tolist()[-1] == 13
    assert np.array_equal(np.isnan(got), bad)
    assert np.array_equal(got[~bad].view(np.uint32), want[~bad].view(np.uint32))


def test_correct_ragged_scalar_path(dev):
    _say("case: correct, ragged 1003 pixels")
    rng = np.random.default_rng(5)
    n = 1003
    raw = rng.integers(0, 1 << 16, (2, n), dtype=np.uint16)
    ped = rng.normal(2000, 50, (3, n)).astype(np.float32)
    gain = rng.uniform(0.1, 20, (3, n)).astype(np.float32)
    out, _ = api.correct(torch.from_numpy(raw).to(dev), torch.from_numpy(ped).to(dev),
                         torch.from_numpy(gain).to(dev))
    sig, bad = OC.correct(raw, ped, gain)
    got = out.cpu().numpy()
    assert np.array_equal(np.isnan(got), bad)
    assert np.array_equal(got[~bad].view(np.uint32), sig[~bad].view(np.uint32))


# -- clipping --------------------------------------------------------------------------

def _replay(sc, prof, f, signal, p, label, **kw):
    res, counts = sc.check_profile(_prof_host(prof, f), signal, p, label, **kw)
    assert counts["unresolved"] == 0, (label, counts)
    return res, counts


def test_clip_small_config(dev, small):
    g, sc, geo, frames, = small
    p = api.Params()
    _say("case: clip, small-512 x8, default params")
    prof = api.sigma_clip(torch.from_numpy(frames).to(dev), geo, p)
    replayed = 0
    for f in range(frames.shape[0]):
        replayed += _replay(sc, prof, f, frames[f], p, f"frame {f}")[1]["replayed"]
    _say(f"  bins replayed: {replayed} of {8 * geo.n_bins}")
    assert replayed <= 2


@pytest.mark.parametrize("variant", [
    dict(cutoff=0.0),                        # Chauvenet cut-off
    dict(error_model="poisson"),
    dict(error_model="hybrid"),
    dict(max_iter=0),                        # plain average
    dict(cutoff=2.0, max_iter=12),
    dict(cutoff=1.0, max_iter=32),
])
def test_clip_variants(dev, small, variant):
    g, sc, geo, frames = small
    p = api.Params(**variant)
    _say("case: clip variant", variant)
    prof = api.sigma_clip(torch.from_numpy(frames[:2]).to(dev), geo, p)
    for f in range(2):
        _replay(sc, prof, f, frames[f], p, f"{variant} frame {f}")


@pytest.mark.parametrize("model", ["azimuthal", "poisson", "hybrid"])
def test_integrate_csr_matches_oracle(dev, small, model):
    """ss_integrate_csr: the unclipped moments, whatever max_iter says."""
    g, sc, geo, frames = small
    p = api.Params(error_model=model, max_iter=7)
    _say("case: integrate_csr", model)
    prof = api.integrate(torch.from_numpy(frames[:3]).to(dev), geo, p)
    for f in range(3):
        res, counts = _replay(sc, prof, f, frames[f], api.Params(error_model=model, max_iter=0),
                              f"integrate {model} frame {f}")
        assert counts["replayed"] == 0
        assert np.all(_prof_host(prof, f)["n_iter"] == 0)


def test_clip_extra_mask_and_long_rows(dev, small):
    """An extra mask and rows longer than the register path holds both take
    the streaming kernel."""
    g, sc, _, frames = small
    _say("case: clip, extra mask + 8 bins (rows > 24576)")
    m = synth.stripe_mask(g)
    geo8 = api.Geometry(g.height, g.width, g.pixel_m, g.dist_m, g.centre_row, g.centre_col, 8, "none", m,
                        None, dev)
    assert geo8.max_row > 1024 * 24
    from oracle import geometry as OG
    csr8 = OG.build_csr(g.height, g.width, g.pixel_m, g.dist_m, g.centre_row, g.centre_col, 8, "none",
                        m.reshape(-1))
    p = api.Params()
    prof = api.sigma_clip(torch.from_numpy(frames[:2]).to(dev), geo8, p)
    for f in range(2):
        _replay(sc, prof, f, frames[f], p, f"8 bins frame {f}", csr=csr8)
    extra = np.zeros(g.n_pix, dtype=np.uint8)
    extra[::7] = 1
    geo = api.Geometry.from_scene(g, m, None, dev)
    prof = api.sigma_clip(torch.from_numpy(frames[:2]).to(dev), geo, p, mask=torch.from_numpy(extra).to(dev))
    both = (m.reshape(-1) | extra).astype(np.uint8)
    for f in range(2):
        _replay(sc, prof, f, frames[f], p, f"extra mask frame {f}", mask=both)


# -- classification ----------------------------------------------------------------------

def _host_outputs(out, f):
    n_k = int(out["n_kept"][f])
    cap = out["kept_index"].shape[1]
    assert n_k <= cap, (n_k, cap)
    return (out["kept_index"][f, :n_k].cpu().numpy(), out["kept_value"][f, :n_k].cpu().numpy(),
            api.peaks_to_numpy(out["peaks"][f], int(out["n_peaks"][f])))


def _check_classify(sc, signal, prof_dev, f, out, p, label):
    """Profile replay, then kept pixels and peaks against the oracle with the
    resolved profile; at most 0.1 % of the valid pixels excused (their own
    decision within rounding of its threshold), no bin unresolved."""
    gpu = _prof_host(prof_dev, f)
    res, counts = _replay(sc, prof_dev, f, signal, p, label)
    ki, kv, pk = _host_outputs(out, f)
    c = sc.check_classify(signal, gpu, res, ki, kv, pk, p, label)
    _say(f"  {label}: bins replayed {counts['replayed']}/{counts['bins']}, unresolved {counts['unresolved']}; "
         f"kept {c['kept']} (excused {c['excused_keep']} px, diffs {c['kept_diffs']}), peaks {c['peaks']} "
         f"(excused {c['excused_cand']} px, diffs {c['peak_diffs']}) of {c['valid']} valid px")
    assert counts["replayed"] <= 1e-3 * counts["bins"] + 1, counts
    assert c["excused_keep"] <= 1e-3 * c["valid"] and c["excused_cand"] <= 1e-3 * c["valid"], c
    return c


@pytest.mark.parametrize("params", [
    dict(),
    dict(n_pick=1.0, snr=2.0, patch=5, min_count=4),
    dict(n_pick=2.0, noise=1.0, patch=1, min_count=1),
])
def test_classify_small_config(dev, small, params):
    g, sc, geo, frames = small
    p = api.Params(**params)
    _say("case: classify, small-512 x8", params)
    fr = torch.from_numpy(frames).to(dev)
    prof = api.sigma_clip(fr, geo, p)
    out = api.classify(fr, geo, prof, p, capacity=70000, peak_capacity=4096)
    torch.cuda.synchronize()
    for f in range(frames.shape[0]):
        _check_classify(sc, frames[f], prof, f, out, p, f"{params} frame {f}")


def test_jungfrau_path(dev, jungfrau):
    g, sc, geo, raw, ped, gain = jungfrau
    p = api.Params()
    _say("case: full path, jungfrau-4m x3")
    pipe = api.Pipeline(geo, p, raw.shape[0], torch.from_numpy(ped).to(dev), torch.from_numpy(gain).to(dev),
                        kept_capacity=1 << 18, peak_capacity=1 << 13, device=dev)
    out = pipe.run(torch.from_numpy(raw).to(dev))
    torch.cuda.synchronize()
    signal, _ = sc.signal_from_raw(raw)
    got = pipe.frames.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), sc.corrected(signal).view(np.uint32))
    for f in range(raw.shape[0]):
        _check_classify(sc, signal[f], pipe.profile, f, out, p, f"jungfrau frame {f}")


def test_capacity_overflow_reports_true_count(dev, small):
    g, sc, geo, frames = small
    p = api.Params(n_pick=1.0)
    _say("case: kept capacity overflow")
    fr = torch.from_numpy(frames[:2]).to(dev)
    prof = api.sigma_clip(fr, geo, p)
    full = api.classify(fr, geo, prof, p, capacity=100000, peak_capacity=4096)
    small_out = api.classify(fr, geo, prof, p, capacity=1000, peak_capacity=3)
    torch.cuda.synchronize()
    for f in range(2):
        n = int(full["n_kept"][f])
        assert n > 1000 and int(small_out["n_kept"][f]) == n
        assert torch.equal(small_out["kept_index"][f, :1000], full["kept_index"][f, :1000])
        npk = int(full["n_peaks"][f])
        assert int(small_out["n_peaks"][f]) == npk and npk > 3
        assert torch.equal(small_out["peaks"][f, :3], full["peaks"][f, :3])


def test_compress_and_peakfind_entry_points_match_classify(dev, small):
    g, sc, geo, frames = small
    p = api.Params()
    _say("case: split entry points")
    fr = torch.from_numpy(frames[:3]).to(dev)
    prof = api.sigma_clip(fr, geo, p)
    both = api.classify(fr, geo, prof, p, capacity=20000, peak_capacity=1024)
    k = api.compress(fr, geo, prof, p, 20000)
    pk = api.peakfind(fr, geo, prof, p, 1024)
    torch.cuda.synchronize()
    assert torch.equal(both["n_kept"], k["n_kept"]) and torch.equal(both["n_peaks"], pk["n_peaks"])
    for f in range(3):
        n = int(k["n_kept"][f])
        assert torch.equal(both["kept_index"][f, :n], k["kept_index"][f, :n])
        m = int(pk["n_peaks"][f])
        assert torch.equal(both["peaks"][f, :m], pk["peaks"][f, :m])


def test_deterministic(dev, small):
    g, sc, geo, frames = small
    p = api.Params()
    _say("case: determinism")
    fr = torch.from_numpy(frames[:4]).to(dev)
    outs = []
    for _ in range(2):
        prof = api.sigma_clip(fr, geo, p)
        cl = api.classify(fr, geo, prof, p, capacity=20000, peak_capacity=1024)
        torch.cuda.synchronize()
        outs.append((prof, cl))
    for k in outs[0][0]:
        assert torch.equal(outs[0][0][k], outs[1][0][k]), k
    a, b = outs[0][1], outs[1][1]
    assert torch.equal(a["n_kept"], b["n_kept"]) and torch.equal(a["n_peaks"], b["n_peaks"])
    for f in range(4):
        n, m = int(a["n_kept"][f]), int(a["n_peaks"][f])
        assert torch.equal(a["kept_index"][f, :n], b["kept_index"][f, :n])
        assert torch.equal(a["kept_value"][f, :n], b["kept_value"][f, :n])
        assert torch.equal(a["peaks"][f, :m], b["peaks"][f, :m])


def test_degenerate_inputs(dev, small):
    g, sc, geo, frames = small
    p = api.Params()
    _say("case: degenerate inputs")
    # a frame with every pixel invalid: every bin empty, nothing kept
    nan = torch.full((1, g.n_pix), float("nan"), device=dev)
    prof = api.sigma_clip(nan, geo, p)
    out = api.classify(nan, geo, prof, p, capacity=16, peak_capacity=16)
    torch.cuda.synchronize()
    assert int(prof["n_members"].sum()) == 0 and float(prof["mean"].abs().sum()) == 0.0
    assert int(out["n_kept"][0]) == 0 and int(out["n_peaks"][0]) == 0
    # a flat frame: std 0 everywhere, no removal, mean exact
    flat = torch.full((1, g.n_pix), 7.5, device=dev)
    prof = api.sigma_clip(flat, geo, p)
    torch.cuda.synchronize()
    ne = prof["n_members"][0] > 0
    assert torch.all(prof["mean"][0][ne] == 7.5) and torch.all(prof["std"][0][ne] == 0.0)
    assert torch.all(prof["n_iter"][0] == 0)
    # zero frames: nothing enqueued
    api.sigma_clip(torch.empty((0, g.n_pix), device=dev), geo, p)


def test_tiny_ragged_frame(dev):
    """A 37 x 53 detector: one partial tile, rows of a handful of entries."""
    _say("case: tiny ragged frame")
    H, W = 37, 53
    rng = np.random.default_rng(9)
    from oracle import geometry as OG
    from oracle import classify as OKc
    from oracle import stats as OS
    frames = rng.poisson(40.0, (2, H * W)).astype(np.float32)
    frames[0, 100] = 900.0
    frames[0, 101] = 700.0
    frames[0, 100 + W] = 800.0
    geo = api.Geometry(H, W, 75e-6, 0.01, 18.3, 26.1, 12, "bbox", None, None, dev)
    csr = OG.build_csr(H, W, 75e-6, 0.01, 18.3, 26.1, 12, "bbox")
    pos = OG.centre_angle(H, W, 75e-6, 0.01, 18.3, 26.1)
    p = api.Params()
    fr = torch.from_numpy(frames).to(dev)
    prof = api.sigma_clip(fr, geo, p)
    out = api.classify(fr, geo, prof, p, capacity=H * W, peak_capacity=64)
    torch.cuda.synchronize()
    for f in range(2):
        ref, _ = P.compare_profile(_prof_host(prof, f), frames[f], None, csr, None, p, *P.input_eps(None, "bbox"),
                                   f"tiny {f}")
        ri, _ = OKc.compress(frames[f], None, pos, csr.centres, ref, 3.0)
        n = int(out["n_kept"][f])
        assert np.array_equal(out["kept_index"][f, :n].cpu().numpy(), ri)
        rp = OKc.peakfind(frames[f], None, H, W, pos, csr.centres, ref, 3.0, 3, 3)
        gp = api.peaks_to_numpy(out["peaks"][f], int(out["n_peaks"][f]))
        assert np.array_equal(gp["index"].astype(np.int64), rp["index"])
    assert int(out["n_peaks"][0]) >= 1


@pytest.mark.parametrize("snr,patch", [(0.0, 3), (-2.0, 3), (-2.0, 5), (-2.0, 7), (-2.0, 9)])
def test_dense_candidates(dev, snr, patch):
    """Most pixels are candidates (snr <= 0): each wave's list of candidate
    core pixels holds well over 64 entries and takes several rounds of patch
    tests; unrolled (3 x 3, 5 x 5) and runtime (7 x 7, 9 x 9: a patch of more
    than 64 pixels, whose records take two rounds of the wave) patches, kept
    pixels and peaks equal to the oracle's, records within 1e-5."""
    _say("case: dense candidates", snr, patch)
    H, W = 70, 150
    rng = np.random.default_rng(31)
    from oracle import geometry as OG
    from oracle import classify as OKc
    from oracle import stats as OS
    frames = rng.poisson(40.0, (2, H * W)).astype(np.float32)
    geo = api.Geometry(H, W, 75e-6, 0.01, 18.3, 26.1, 16, "bbox", None, None, dev)
    csr = OG.build_csr(H, W, 75e-6, 0.01, 18.3, 26.1, 16, "bbox")
    pos = OG.centre_angle(H, W, 75e-6, 0.01, 18.3, 26.1)
    p = api.Params(snr=snr, patch=patch, min_count=3)
    fr = torch.from_numpy(frames).to(dev)
    prof = api.sigma_clip(fr, geo, p)
    out = api.classify(fr, geo, prof, p, capacity=H * W, peak_capacity=H * W)
    torch.cuda.synchronize()
    for f in range(2):
        ref, _ = P.compare_profile(_prof_host(prof, f), frames[f], None, csr, None, p, *P.input_eps(None, "bbox"),
                                   f"dense {f}")
        ri, _ = OKc.compress(frames[f], None, pos, csr.centres, ref, 3.0)
        n = int(out["n_kept"][f])
        assert np.array_equal(out["kept_index"][f, :n].cpu().numpy(), ri)
        rp = OKc.peakfind(frames[f], None, H, W, pos, csr.centres, ref, snr, patch, 3)
        gp = api.peaks_to_numpy(out["peaks"][f], int(out["n_peaks"][f]))
        assert np.array_equal(gp["index"].astype(np.int64), rp["index"]), (f, gp.size, rp.size)
        assert rp.size > 10, rp.size
        # with candidates below the background (snr < 0) the intensity of a
        # patch may nearly cancel, so the centroid (a ratio) is compared
        # through its numerator
        gi, ri = gp["intensity"].astype(np.float64), rp["intensity"]
        for a, b, k in ((gi, ri, "intensity"), (gp["sigma"].astype(np.float64), rp["sigma"], "sigma"),
                        (gp["y"] * gi, rp["y"] * ri, "y * intensity"), (gp["x"] * gi, rp["x"] * ri, "x * intensity")):
            assert np.allclose(a, b, rtol=2e-6, atol=1e-6 * np.abs(b).max()), (f, k)


@pytest.mark.parametrize("n_frames", [1, 3])
def test_wide_frames_match_oracle(dev, n_frames):
    """Frames 9000 pixels wide: one frame counts its compaction tiles in a
    kernel of its own (a pixel-pass tile's rows span more tiles than the
    pass counts in LDS), three frames count them in the pixel pass; kept
    pixels and peaks equal to the oracle's either way."""
    _say("case: wide frames", n_frames)
    H, W = 20, 9000
    rng = np.random.default_rng(47)
    from oracle import geometry as OG
    from oracle import classify as OKc
    frames = rng.poisson(40.0, (n_frames, H * W)).astype(np.float32)
    geo = api.Geometry(H, W, 75e-6, 0.01, 10.3, 4500.1, 16, "bbox", None, None, dev)
    csr = OG.build_csr(H, W, 75e-6, 0.01, 10.3, 4500.1, 16, "bbox")
    pos = OG.centre_angle(H, W, 75e-6, 0.01, 10.3, 4500.1)
    p = api.Params(snr=2.0, min_count=2)
    fr = torch.from_numpy(frames).to(dev)
    prof = api.sigma_clip(fr, geo, p)
    out = api.classify(fr, geo, prof, p, capacity=H * W, peak_capacity=H * W)
    torch.cuda.synchronize()
    for f in range(n_frames):
        ref, _ = P.compare_profile(_prof_host(prof, f), frames[f], None, csr, None, p, *P.input_eps(None, "bbox"),
                                   f"wide {f}")
        ri, _ = OKc.compress(frames[f], None, pos, csr.centres, ref, 3.0)
        n = int(out["n_kept"][f])
        assert n == ri.size and np.array_equal(out["kept_index"][f, :n].cpu().numpy(), ri)
        rp = OKc.peakfind(frames[f], None, H, W, pos, csr.centres, ref, 2.0, 3, 2)
        gp = api.peaks_to_numpy(out["peaks"][f], int(out["n_peaks"][f]))
        assert np.array_equal(gp["index"].astype(np.int64), rp["index"]), (f, gp.size, rp.size)
        assert rp.size > 10 and ri.size > 100, (rp.size, ri.size)


def test_correct_indexed_matches_correct(dev, jungfrau):
    """ss_correct_indexed: frames picked from a ring by a device index are
    corrected bit for bit as ss_correct corrects the same frames; an index
    outside the ring gives an all-NaN frame, every pixel counted invalid."""
    g, sc, geo, raw, ped, gain = jungfrau
    _say("case: correct_indexed, ring of 3 jungfrau-4m frames")
    ring = torch.from_numpy(raw.view(np.int16)).to(dev)
    ped_d, gain_d = torch.from_numpy(ped).to(dev), torch.from_numpy(gain).to(dev)
    for idx in ([2, 0], [1], [0, 2, 1, 1]):
        fi = torch.tensor(idx, dtype=torch.int64, device=dev)
        got, nb = api.correct_indexed(ring, fi, ped_d, gain_d, geo.norm)
        want, nw = api.correct(torch.from_numpy(raw[idx]).to(dev), ped_d, gain_d, geo.norm)
        torch.cuda.synchronize()
        assert torch.equal(nb, nw)
        assert np.array_equal(got.cpu().numpy().view(np.uint32), want.cpu().numpy().view(np.uint32)), idx
    fi = torch.tensor([1, 3, -1], dtype=torch.int64, device=dev)
    got, nb = api.correct_indexed(ring, fi, ped_d, gain_d, geo.norm)
    torch.cuda.synchronize()
    assert nb.cpu().tolist()[1:] == [g.n_pix, g.n_pix]
    assert torch.isnan(got[1:]).all() and not torch.isnan(got[0]).all()
