"""Continuous-batching service of four detectors (Jungfrau 1M, 4M, 9M, 16M):
every frame's results in the mix (batched with other frames of its
detector, batches of all detectors in flight together) are the same as when
the frame is served alone, and one served frame per detector matches the
FP64 oracle (profile through the replay, kept pixels and peaks; a tile and
sampled bins for the two largest detectors).

Tolerance: kept pixels, their values and the peaks identical; the profile
within the clip's parity tolerance (a batch and a single frame run
work-group shapes that sum in different orders)."""

import sys

import numpy as np
import pytest
import torch

import synth
from paper_2411_09515_amd import api, serve

pytestmark = pytest.mark.gpu

REL, ABS_OF_MEAN = 1e-5, 1e-7
DETS = (("1m", synth.JUNGFRAU1M), ("4m", synth.JUNGFRAU4M), ("9m", synth.JUNGFRAU9M), ("16m", synth.JUNGFRAU16M))
RING = 2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def detectors(dev):
    out = []
    for name, g in DETS:
        _say(f"setup: {name}")
        geo = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev)
        ring = np.stack([synth.uneven_frame(g, 100 + k)[0] for k in range(RING)]).reshape(RING, -1)
        ped, gain = (torch.from_numpy(np.array(a)).to(dev) for a in synth.jungfrau_calibration(g))
        out.append(serve.Detector(name, geo, ped, gain, torch.from_numpy(ring.view(np.int16)).to(dev),
                                  api.Params(cutoff=3.0, max_iter=5), max_batch=4))
    return out


def _same(a, b, label):
    assert a.n_kept == b.n_kept and a.n_peaks == b.n_peaks, label
    assert np.array_equal(a.kept_index, b.kept_index), label
    assert np.array_equal(a.kept_value.view(np.uint32), b.kept_value.view(np.uint32)), label
    assert np.array_equal(a.peaks, b.peaks), label
    tol = REL * np.abs(b.mean) + ABS_OF_MEAN * np.abs(b.mean)
    assert np.all(np.abs(a.mean - b.mean) <= tol), label
    assert np.all(np.abs(a.std - b.std) <= REL * np.abs(b.std) + ABS_OF_MEAN * np.abs(b.mean)), label
    for k in ("n_members", "n_iter", "converged"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), (label, k)


@pytest.fixture(scope="module")
def served(dev, detectors):
    """Every ring frame served alone, then mixed Poisson arrivals served with
    eager launches and with graph replays."""
    server = serve.Server(detectors, hbm_budget=12 << 30, device=dev, full_profile=True)
    _say("case: alone, one request at a time")
    alone = {}
    for d in range(len(detectors)):
        for k in range(RING):
            (r,), _ = server.run([serve.Request(det=d, ring_index=k, t_arrival=0.0)], realtime=False)
            assert r.batch_size == 1
            alone[(d, k)] = r
    mixed = {}
    for mode in ("eager launches", "graph replays"):
        if mode == "graph replays":
            _say("case: capture every slot's batch sizes as graphs")
            server.capture_graphs()
            assert all(len(s.graphs) == s.det.max_batch for s in server.slots)
            for d in range(len(detectors)):   # a graph of one frame gives the eager result bit for bit
                (r,), _ = server.run([serve.Request(det=d, ring_index=1, t_arrival=0.0)], realtime=False)
                a = alone[(d, 1)]
                assert np.array_equal(r.mean, a.mean) and np.array_equal(r.std, a.std)
                _same(r, a, ("graph alone", d))
        _say(f"case: mixed Poisson arrivals, 2000 Hz aggregate, 0.25 s, {mode}")
        reqs = serve.poisson_arrivals([900, 600, 300, 200], 0.25, [RING] * len(detectors), seed=5)
        done, stats = server.run(reqs, realtime=True)
        _say(stats)
        mixed[mode] = (done, stats, len(reqs))
    server.close()
    return alone, mixed


def test_results_are_the_same_alone_and_in_the_mix(dev, served):
    alone, mixed = served
    for mode, (done, stats, n) in mixed.items():
        assert stats["frames"] == n and all(np.isfinite(r.t_done) for r in done)
        assert stats["max_batches_in_flight"] >= 2          # batches overlap on the device
        assert max(r.batch_size for r in done) >= 2         # frames that waited were batched
        for r in done:
            _same(r, alone[(r.det, r.ring_index)], (mode, r.rid, r.det, r.ring_index, r.batch_size))


# one served frame per detector against the oracle: the whole frame for 1M
# and 4M; for 9M and 16M a 256 x 256 tile across the water ring (every bin
# its pixels interpolate between) plus the six longest rows
TILES = {"9m": True, "16m": True}


@pytest.mark.parametrize("d", range(len(DETS)))
def test_served_frame_matches_oracle(dev, served, d):
    from parity import OracleScene
    alone, mixed = served
    name, g = DETS[d]
    done, _, _ = mixed["graph replays"]
    r = next(x for x in done if x.det == d)
    _say(f"case: served {name} frame (ring {r.ring_index}, batch of {r.batch_size}) vs oracle")
    sc = OracleScene(g)
    raw = synth.uneven_frame(g, 100 + r.ring_index)[0].reshape(1, -1)
    signal, _ = sc.signal_from_raw(raw)
    gpu = {k: getattr(r, k) for k in ("mean", "std", "sem", "sum_w", "n_members", "n_iter", "converged")}
    p = api.Params(cutoff=3.0, max_iter=5)
    region = bins = None
    if TILES.get(name):
        cy, cx = int(g.centre_row), int(g.centre_col)
        region = (cy + 200, cy + 456, cx + 250, cx + 506)
        lens = np.diff(sc.csr.indptr)
        bins = np.concatenate([sc.tile_bins(region), np.argsort(lens)[-6:]])
    res, counts = sc.check_profile(gpu, signal[0], p, f"served {name}", bins=bins)
    if bins is not None:
        assert np.all(res["n_members"][sc.tile_bins(region)] > 0)   # the tile interpolates inside the sample
    c = sc.check_classify(signal[0], gpu, res, r.kept_index, r.kept_value, r.peaks, p, f"served {name}",
                          region=region)
    _say(f"  {name}: bins {counts['bins']} (replayed {counts['replayed']}), kept {c['kept']} "
         f"(excused {c['excused_keep']} px), peaks {c['peaks']} (excused {c['excused_cand']} px) "
         f"of {c['valid']} valid px")
    assert counts["unresolved"] == 0 and counts["replayed"] <= 1e-3 * counts["bins"] + 1
    assert c["excused_keep"] <= 1e-3 * c["valid"] and c["excused_cand"] <= 1e-3 * c["valid"]
    assert c["kept"] > 0


def test_packed_results_match_the_per_frame_layout(dev):
    """ss_pack_results: every frame's kept entries and peaks back to back,
    counts clamped to the capacities (one frame overflows its capacity)."""
    g = synth.SMALL
    _say("case: pack results, small-512 x5")
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), None, dev)
    fr = torch.from_numpy(synth.float_frames(g, 5).reshape(5, -1)).to(dev)
    p = api.Params(n_pick=1.5)
    prof = api.sigma_clip(fr, geo, p)
    out = api.classify(fr, geo, prof, p, capacity=20000, peak_capacity=10)
    packed = api.pack_results(out, 20000, 10)
    torch.cuda.synchronize()
    nk = out["n_kept"].cpu().numpy()
    npk = out["n_peaks"].cpu().numpy()
    assert nk.max() > 0 and npk.max() > 10          # more peaks than room
    ck, cp = np.minimum(nk, 20000), np.minimum(npk, 10)
    off = packed["offsets"].cpu().numpy()
    assert np.array_equal(off[:6], np.concatenate([[0], np.cumsum(ck)]))
    assert np.array_equal(off[6:], np.concatenate([[0], np.cumsum(cp)]))
    for f in range(5):
        assert torch.equal(packed["index"][off[f]:off[f + 1]], out["kept_index"][f, :ck[f]])
        assert torch.equal(packed["value"][off[f]:off[f + 1]], out["kept_value"][f, :ck[f]])
        assert torch.equal(packed["peaks"][off[6 + f]:off[7 + f]], out["peaks"][f, :cp[f]])
    # peaks only
    only = api.pack_results({k: out[k] for k in ("peaks", "n_peaks")}, 20000, 10)
    assert torch.equal(only["offsets"][6:], packed["offsets"][6:]) and int(only["offsets"][5]) == 0


def test_tiled_detector_served_alone_batched_and_against_oracle(dev):
    """A detector whose corrected frames are in 8 x 4 tiles (the served
    frames go through ss_correct_indexed_tiled): each result is the same
    alone and in batches, eager and as graph replays, and one served frame
    matches the FP64 oracle."""
    from parity import OracleScene
    g = synth.JUNGFRAU1M
    _say("setup: tiled 1m detector")
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev, tile=(8, 4))
    assert geo.frame_words > geo.n_pix
    ring = np.stack([synth.uneven_frame(g, 300 + k)[0] for k in range(3)]).reshape(3, -1)
    ped, gain = (torch.from_numpy(np.array(a)).to(dev) for a in synth.jungfrau_calibration(g))
    p = api.Params(cutoff=3.0, max_iter=5)
    det = serve.Detector("1m-tiled", geo, ped, gain, torch.from_numpy(ring.view(np.int16)).to(dev), p, max_batch=4)
    server = serve.Server([det], hbm_budget=4 << 30, device=dev, full_profile=True)
    _say("case: tiled detector, alone then batched (eager, graph replays)")
    alone = {}
    for k in range(3):
        (r,), _ = server.run([serve.Request(det=0, ring_index=k, t_arrival=0.0)], realtime=False)
        alone[k] = r
    for mode in ("eager", "graphs"):
        if mode == "graphs":
            server.capture_graphs()
        reqs = [serve.Request(det=0, ring_index=k % 3, t_arrival=0.0) for k in range(8)]
        done, stats = server.run(reqs, realtime=False)
        assert max(r.batch_size for r in done) >= 2, mode
        for r in done:
            _same(r, alone[r.ring_index], (mode, r.rid, r.ring_index, r.batch_size))
    server.close()
    _say("case: tiled served frame vs oracle")
    sc = OracleScene(g)
    r = alone[1]
    signal, _ = sc.signal_from_raw(ring[1:2])
    gpu = {k: getattr(r, k) for k in ("mean", "std", "sem", "sum_w", "n_members", "n_iter", "converged")}
    res, counts = sc.check_profile(gpu, signal[0], p, "served tiled 1m")
    c = sc.check_classify(signal[0], gpu, res, r.kept_index, r.kept_value, r.peaks, p, "served tiled 1m")
    _say(f"  tiled 1m: bins {counts['bins']} (replayed {counts['replayed']}), kept {c['kept']}, peaks {c['peaks']}")
    assert counts["unresolved"] == 0 and counts["replayed"] <= 1e-3 * counts["bins"] + 1
    assert c["excused_keep"] <= 1e-3 * c["valid"] and c["excused_cand"] <= 1e-3 * c["valid"] and c["kept"] > 0
