"""The throughput benchmark's own launch configuration against the FP64
oracle, through the C ABI: one call per stage on 64 raw Jungfrau-4M frames
(2162 x 2068, 1000 bins, bounding-box splitting), so every row-length class
runs with its default work-group shape and several frames per work-group.

* sampled frames of the batch (first, middle, last) match the oracle: the
  correction bit for bit, the profile through the replay of ``parity`` (no
  bin unresolved, at most 0.1 % replayed), the kept pixels / peaks exactly
  outside at most 0.1 % of the valid pixels;
* frames are independent inside the batch: the batch holds 16 distinct
  frames four times over (neighbouring frames always differ), and every
  repeat gives bit-identical results wherever it sits in the batch.
"""

import sys

import numpy as np
import pytest
import torch

import synth
from paper_2411_09515_amd import api

from parity import OracleScene
from test_gpu_parity import _check_classify

pytestmark = pytest.mark.gpu

N_DISTINCT, N_FRAMES = 16, 64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch(dev):
    g = synth.JUNGFRAU4M
    _say("setup: 16 distinct jungfrau-4m frames (~10 s) and the oracle geometry")
    distinct = synth.jungfrau_frames(g, N_DISTINCT).reshape(N_DISTINCT, -1)
    raw = np.concatenate([distinct] * (N_FRAMES // N_DISTINCT))
    sc = OracleScene(g)
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev)
    ped, gain = (torch.from_numpy(np.array(a)).to(dev) for a in synth.jungfrau_calibration(g))
    p = api.Params()
    pipe = api.Pipeline(geo, p, N_FRAMES, ped, gain, kept_capacity=1 << 18, peak_capacity=1 << 13, device=dev)
    _say("case: whole path on 64 frames (benchmark shapes)")
    out = pipe.run(torch.from_numpy(raw).to(dev))
    torch.cuda.synchronize()
    return g, sc, raw, pipe, out, p


@pytest.mark.parametrize("f", [0, 37, 63])
def test_sampled_frames_match_oracle(dev, batch, f):
    g, sc, raw, pipe, out, p = batch
    _say(f"case: 64-frame batch, frame {f} vs oracle")
    signal, _ = sc.signal_from_raw(raw[f:f + 1])
    got = pipe.frames[f].cpu().numpy()
    assert np.array_equal(got.view(np.uint32), sc.corrected(signal)[0].view(np.uint32))
    _check_classify(sc, signal[0], pipe.profile, f, out, p, f"bench batch frame {f}")


def test_repeated_frames_are_identical(dev, batch):
    g, sc, raw, pipe, out, p = batch
    _say("case: 64-frame batch, repeats bit for bit")
    prof = {k: v.cpu() for k, v in pipe.profile.items()}
    n_kept, n_peaks = out["n_kept"].cpu(), out["n_peaks"].cpu()
    for f in range(N_DISTINCT):
        for r in range(f + N_DISTINCT, N_FRAMES, N_DISTINCT):
            assert torch.equal(pipe.frames[f], pipe.frames[r]), (f, r)
            for k, v in prof.items():
                assert torch.equal(v[f], v[r]), (k, f, r)
            assert n_kept[f] == n_kept[r] and n_peaks[f] == n_peaks[r], (f, r)
            n, m = int(n_kept[f]), int(n_peaks[f])
            assert torch.equal(out["kept_index"][f, :n], out["kept_index"][r, :n])
            assert torch.equal(out["kept_value"][f, :n], out["kept_value"][r, :n])
            assert torch.equal(out["peaks"][f, :m], out["peaks"][r, :m])


def test_single_frame_graph_replays_match_eager(dev, batch):
    """The single-frame path captured once as a HIP graph: each replay, on a
    new frame written into its input buffer, equals the eager call bit for
    bit (eager work runs between the replays)."""
    g, sc, raw, pipe, out, p = batch
    _say("case: single-frame graph replays vs eager")
    one = api.Pipeline(pipe.geom, p, 1, pipe.pedestal, pipe.gain, kept_capacity=1 << 16, peak_capacity=1 << 12,
                       device=dev)
    ref = api.Pipeline(pipe.geom, p, 1, pipe.pedestal, pipe.gain, kept_capacity=1 << 16, peak_capacity=1 << 12,
                       device=dev)
    buf = torch.from_numpy(raw[:1].copy()).to(dev)
    one.capture(buf)
    for f in (3, 17, 3, 40):
        buf.copy_(torch.from_numpy(raw[f:f + 1]).to(dev))
        one.profile["mean"].fill_(-1.0)       # eager work between replays
        one.out["n_kept"].fill_(-1)
        torch.cuda.synchronize()
        got = one.replay()
        want = ref.run(torch.from_numpy(raw[f:f + 1]).to(dev))
        torch.cuda.synchronize()
        assert torch.equal(one.frames, ref.frames), f
        for k in one.profile:
            assert torch.equal(one.profile[k], ref.profile[k]), (f, k)
        n, m = int(want["n_kept"][0]), int(want["n_peaks"][0])
        assert int(got["n_kept"][0]) == n and int(got["n_peaks"][0]) == m, f
        assert torch.equal(got["kept_index"][0, :n], want["kept_index"][0, :n])
        assert torch.equal(got["kept_value"][0, :n], want["kept_value"][0, :n])
        assert torch.equal(got["peaks"][0, :m], want["peaks"][0, :m])
