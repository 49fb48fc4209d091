"""Continuous-batching service of four detectors (Jungfrau 1M, 4M, 9M, 16M):
every frame's results in the mix (batched with other frames of its
detector, batches of all detectors in flight together) are the same as when
the frame is served alone.

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


def test_results_are_the_same_alone_and_in_the_mix(dev, detectors):
    server = serve.Server(detectors, hbm_budget=12 << 30, device=dev)
    _say("case: alone, one request at a time")
    alone = {}
    for d in range(len(detectors)):
        for k in range(RING):
            (r,), _ = server.run([serve.Request(det=d, ring_index=k, t_arrival=0.0)], realtime=False)
            assert r.batch_size == 1
            alone[(d, k)] = r
    _say("case: mixed Poisson arrivals, 2000 Hz aggregate, 0.25 s")
    reqs = serve.poisson_arrivals([900, 600, 300, 200], 0.25, [RING] * len(detectors), seed=5)
    done, stats = server.run(reqs, realtime=True)
    _say(stats)
    assert stats["frames"] == len(reqs) and all(np.isfinite(r.t_done) for r in done)
    assert stats["max_batches_in_flight"] >= 2          # batches overlap on the device
    assert max(r.batch_size for r in done) >= 2         # frames that waited were batched
    for r in done:
        _same(r, alone[(r.det, r.ring_index)], (r.rid, r.det, r.ring_index, r.batch_size))
