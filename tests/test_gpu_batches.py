"""Batches of uneven detectors (Jungfrau 1M, 4M, 16M) in shared launches,
the autotuner's shape variants, and the whole path captured in a HIP graph,
through the C ABI.

* ss_sigma_clip_batches gives bit-identical profiles to one ss_sigma_clip
  call per batch (the same kernels run the same arithmetic);
* the 16M detector's longest rows (the weights-from-memory class) match the
  FP64 oracle through the replay of ``parity``, sampled bins; the 1M
  detector's frames match it in every bin, kept pixels and peaks included;
* every shape variant agrees with the default within that tolerance (the
  summation order differs);
* graph replays reproduce the eager results bit for bit, replay after
  replay, with eager work in between.
"""

import sys

import numpy as np
import pytest
import torch

import synth
from oracle import stats as OS
from paper_2411_09515_amd import api

from parity import OracleScene
from test_gpu_parity import _check_classify

pytestmark = pytest.mark.gpu

REL, ABS_OF_MEAN = 1e-5, 1e-7
MIX = ((synth.JUNGFRAU1M, 3), (synth.JUNGFRAU4M, 2), (synth.JUNGFRAU16M, 2))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def mixed(dev):
    out = []
    for g, n in MIX:
        _say(f"setup: {g.name} x{n}")
        geo = api.Geometry.from_scene(g, synth.stripe_mask(g), synth.normalisation(g), dev)
        raw = np.stack([synth.uneven_frame(g, k)[0] for k in range(n)]).reshape(n, -1)
        ped, gain = (torch.from_numpy(np.array(a)).to(dev) for a in synth.jungfrau_calibration(g))
        raw_d = torch.from_numpy(raw).to(dev)
        frames, _ = api.correct(raw_d, ped, gain, geo.norm)
        out.append(dict(g=g, geo=geo, raw=raw, raw_d=raw_d, ped=ped, gain=gain, frames=frames))
    return out


P = api.Params(cutoff=3.0, max_iter=5)


def test_batches_equal_one_call_per_batch(dev, mixed):
    _say("case: clip of 1M x3 + 4M x2 + 16M x2 in shared launches")
    assert mixed[2]["geo"].class_count[6] > 0  # the 16M detector has rows past 24 576 entries
    outs = api.sigma_clip_batches([(m["frames"], m["geo"]) for m in mixed], P)
    for m, o in zip(mixed, outs):
        ref = api.sigma_clip(m["frames"], m["geo"], P)
        for k in ref:
            assert torch.equal(o[k], ref[k]), (m["g"].name, k)


def test_longest_rows_match_oracle(dev, mixed):
    m = mixed[2]
    _say("case: 16M sampled bins vs oracle (oracle geometry build ~30 s)")
    sc = OracleScene(m["g"])
    signal, _ = sc.signal_from_raw(m["raw"])
    prof = api.sigma_clip_batches([(mm["frames"], mm["geo"]) for mm in mixed], P)[2]
    lens = np.diff(sc.csr.indptr)
    rng = np.random.default_rng(3)
    longest = np.argsort(lens)[-12:]
    bins = np.unique(np.concatenate([longest, rng.choice(sc.csr.n_bins, 12, replace=False)]))
    assert lens[longest].min() > api.B.lib().ss_class_rows(5)
    for f in range(signal.shape[0]):
        gp = {k: v[f].cpu().numpy() for k, v in prof.items()}
        _, counts = sc.check_profile(gp, signal[f], P, f"16M frame {f}", bins=bins)
        _say(f"  frame {f}: {counts['bins']} bins, replayed {counts['replayed']}")
        assert counts["unresolved"] == 0 and counts["replayed"] <= 1


def test_jungfrau1m_batch_matches_oracle(dev, mixed):
    """The 1M detector's frames of the shared launches against the oracle:
    every bin through the replay, kept pixels and peaks of the whole path."""
    m = mixed[0]
    _say("case: 1M x3 of the shared launches vs oracle")
    sc = OracleScene(m["g"])
    signal, _ = sc.signal_from_raw(m["raw"])
    prof = api.sigma_clip_batches([(mm["frames"], mm["geo"]) for mm in mixed], P)[0]
    out = api.classify(m["frames"], m["geo"], prof, P, capacity=1 << 17, peak_capacity=1 << 12)
    torch.cuda.synchronize()
    for f in range(signal.shape[0]):
        _check_classify(sc, signal[f], prof, f, out, P, f"1M frame {f}")


def test_every_shape_variant_agrees(dev, mixed):
    _say("case: shape variants 0/1/2 of every class")
    batches = [(m["frames"], m["geo"]) for m in mixed]
    ref = api.sigma_clip_batches(batches, P)
    try:
        for v in (1, 2):
            for m in mixed:
                m["geo"].shape = [v] * api.B.SS_N_CLASSES
            got = api.sigma_clip_batches(batches, P)
            for o, r in zip(got, ref):
                mref = r["mean"].abs()
                for k in ("mean", "std", "sem", "sum_w"):
                    assert torch.all((o[k] - r[k]).abs() <= REL * r[k].abs() + ABS_OF_MEAN * mref), (v, k)
                for k in ("n_members", "n_iter", "converged"):
                    assert torch.equal(o[k], r[k]), (v, k)
    finally:
        for m in mixed:
            m["geo"].shape = [0] * api.B.SS_N_CLASSES


def test_autotuner_returns_a_valid_choice(dev, mixed):
    _say("case: autotune")
    batches = [(m["frames"], m["geo"]) for m in mixed]
    best, timings = api.autotune(batches, P, reps=1)
    try:
        assert len(best) == api.B.SS_N_CLASSES and all(0 <= b <= 2 for b in best)
        assert timings and all(len(t) == 3 and min(t) > 0 for t in timings.values())
        for m in mixed:
            assert m["geo"].shape == best
    finally:
        for m in mixed:
            m["geo"].shape = [0] * api.B.SS_N_CLASSES


def test_graph_replay_matches_eager(dev, mixed):
    _say("case: whole path of the mixed batch in a HIP graph, 3 replays")
    cap = 1 << 16
    state = []
    for m in mixed:
        F, geo = m["frames"].shape[0], m["geo"]
        state.append(dict(
            frames=torch.empty_like(m["frames"]), n_invalid=torch.empty(F, dtype=torch.int64, device=dev),
            prof=api.new_profile(F, geo.n_bins, dev), ws=api.new_workspace(F, geo, dev),
            out=dict(kept_index=torch.empty((F, cap), dtype=torch.int32, device=dev),
                     kept_value=torch.empty((F, cap), dtype=torch.float32, device=dev),
                     n_kept=torch.empty(F, dtype=torch.int64, device=dev),
                     peaks=torch.empty((F, 4096, api.B.PEAK_BYTES), dtype=torch.uint8, device=dev),
                     n_peaks=torch.empty(F, dtype=torch.int64, device=dev))))

    def step():
        for m, s in zip(mixed, state):
            api.correct(m["raw_d"], m["ped"], m["gain"], m["geo"].norm, out=s["frames"], n_invalid=s["n_invalid"])
        api.sigma_clip_batches([(s["frames"], m["geo"]) for m, s in zip(mixed, state)], P,
                               [s["prof"] for s in state])
        for m, s in zip(mixed, state):
            api.classify(s["frames"], m["geo"], s["prof"], P, cap, 4096, workspace=s["ws"], out=s["out"])

    def snapshot():
        snap = []
        for s in state:
            d = {"frames": s["frames"].clone(), "n_invalid": s["n_invalid"].clone()}
            d.update({"p_" + k: v.clone() for k, v in s["prof"].items()})
            n = s["out"]["n_kept"].clone()
            d["n_kept"], d["n_peaks"] = n, s["out"]["n_peaks"].clone()
            d["kept_index"] = [s["out"]["kept_index"][f, :min(int(n[f]), cap)].clone() for f in range(n.numel())]
            d["kept_value"] = [s["out"]["kept_value"][f, :min(int(n[f]), cap)].clone() for f in range(n.numel())]
            snap.append(d)
        return snap

    def same(a, b):
        for x, y in zip(a, b):
            for k in x:
                if isinstance(x[k], list):
                    assert all(torch.equal(p, q) for p, q in zip(x[k], y[k])), k
                else:
                    assert torch.equal(x[k], y[k]), k

    step()
    torch.cuda.synchronize()
    ref = snapshot()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        for s in state:  # eager work between replays: scribble over the outputs
            s["frames"].fill_(-1.0)
            for v in s["prof"].values():
                v.fill_(7)
            s["out"]["n_kept"].fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        same(snapshot(), ref)
