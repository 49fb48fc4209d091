"""Learned clip surrogate, HIP path vs the FP64 oracle, through the C ABI:
the network's forward pass, loss gradient and Adam step, the features, the
verified clip, and what a trained network saves over the plain clip.

Tolerances (float32 arithmetic against float64):
* network outputs: |y - y_ref| <= 1e-4 (1 + |y_ref|) (three layers of
  64-term float32 dot products, float32 GELU);
* gradient: |g - g_ref| <= 1e-4 |g_ref| + 1e-5 max |g_ref| (sums over the
  samples in float32 per tile, float64 across tiles);
* Adam: |p - p_ref| <= 1e-6 (1 + |p_ref|);
* statistics: the profile tolerance of the plain clip (1e-5 relative);
* integer decisions (sketch counts, acceptance) identical except where the
  oracle puts a value within 1e-5 of a threshold (relative to the spread).
"""

import sys

import numpy as np
import pytest
import torch

import synth
from oracle import stats as OS
from oracle import surrogate as Q
from paper_2411_09515_amd import api

from parity import OracleScene

pytestmark = pytest.mark.gpu

MARGIN = 1e-5


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
    frames = synth.float_frames(g, 10).reshape(10, -1)
    return g, sc, geo, frames


def _random_params(seed):
    rng = np.random.default_rng(seed)
    p = Q.init_params(seed)
    p[Q.OFF_B1:Q.OFF_W2] = rng.normal(size=Q.N_HID) * 0.2
    p[Q.OFF_B2:Q.OFF_W3] = rng.normal(size=Q.N_HID) * 0.2
    p[Q.OFF_B3:Q.OFF_B3 + 2] = [0.1, -0.2]
    return p.astype(np.float32)


def test_mlp_forward_matches_oracle(dev):
    _say("case: mlp forward, 1000 samples")
    rng = np.random.default_rng(3)
    p = _random_params(1)
    x = rng.normal(size=(1000, Q.N_IN)).astype(np.float32)
    model = api.Surrogate(p, device=dev)
    y = model.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    ref = Q.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.all(np.abs(y - ref) <= 1e-4 * (1 + np.abs(ref))), np.max(np.abs(y - ref))
    # the float16 copy is the rounding of the float32 parameters
    assert np.array_equal(model.half_params(), Q.to_half(p))


@pytest.mark.parametrize("n", [777, 16, 5])
def test_mlp_gradient_matches_oracle(dev, n):
    _say(f"case: mlp gradient, {n} samples")
    rng = np.random.default_rng(n)
    p = _random_params(2)
    x = rng.normal(size=(n, Q.N_IN)).astype(np.float32)
    t = rng.normal(size=(n, 2)).astype(np.float32)
    use = rng.random(n) < 0.8
    use[0] = True
    model = api.Surrogate(p, device=dev)
    loss, grad = model.gradient(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev),
                                torch.from_numpy(use.astype(np.uint8)).to(dev))
    L, g = Q.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), use)
    got = grad.cpu().numpy()
    assert float(loss.cpu()[0]) == pytest.approx(L, rel=1e-5)
    tol = 1e-4 * np.abs(g) + 1e-5 * np.abs(g).max()
    bad = np.abs(got - g) > tol
    assert not bad.any(), (np.nonzero(bad)[0][:5], got[bad][:5], g[bad][:5])
    assert np.all(got[g == 0] == 0)  # padding


def test_mlp_gradient_is_deterministic(dev):
    _say("case: mlp gradient determinism")
    rng = np.random.default_rng(8)
    x = torch.from_numpy(rng.normal(size=(5000, Q.N_IN)).astype(np.float32)).to(dev)
    t = torch.from_numpy(rng.normal(size=(5000, 2)).astype(np.float32)).to(dev)
    model = api.Surrogate(_random_params(4), device=dev)
    g1 = model.gradient(x, t)[1].clone()
    g2 = model.gradient(x, t)[1].clone()
    assert torch.equal(g1, g2)


def test_adam_matches_oracle(dev):
    _say("case: adam, 5 steps")
    rng = np.random.default_rng(5)
    p = _random_params(3)
    model = api.Surrogate(p, device=dev)
    ref_p, ref_m, ref_v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for step in range(1, 6):
        g = (rng.normal(size=p.size) * 0.01).astype(np.float32)
        g[p == 0] = 0.0
        model.grad.copy_(torch.from_numpy(g))
        model.adam(lr=3e-3)
        ref_p, ref_m, ref_v, ref_h = Q.adam(ref_p, ref_m, ref_v, g.astype(np.float64), step, lr=3e-3)
    got = model.params.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref_p) <= 1e-6 * (1 + np.abs(ref_p)))
    assert np.array_equal(model.half_params(), got.astype(np.float16).astype(np.float64))


def test_features_match_oracle(dev, small):
    g, sc, geo, frames = small
    _say("case: features, small config x2")
    feats, stats0 = api.clip_features(torch.from_numpy(frames[:2]).to(dev), geo)
    feats, stats0 = feats.cpu().numpy(), stats0.cpu().numpy()
    for f in range(2):
        X, st = Q.features(frames[f], None, sc.csr, sc.mask)
        assert np.array_equal(stats0[f, :, 0], st[:, 0])
        assert np.allclose(stats0[f, :, 1:], st[:, 1:], rtol=1e-5, atol=1e-9)
        assert np.allclose(feats[f, :, :3], X[:, :3], rtol=1e-5, atol=1e-6)
        for r in range(sc.csr.n_bins):
            n = st[r, 0]
            if n == 0:
                assert np.all(feats[f, r] == 0)
                continue
            v = OS.bin_members(frames[f], None, sc.csr, r, sc.mask).v
            near = np.array([np.count_nonzero(np.abs(v - (st[r, 1] + t * st[r, 2])) <= MARGIN * st[r, 2])
                             for t in Q.THRESHOLDS])
            diff = np.abs(np.rint(feats[f, r, 3:] * n) - np.rint(X[r, 3:] * n))
            assert np.all(diff <= near), (f, r, diff, near)


def _train_small(dev, geo, frames, steps=400):
    F = frames.shape[0]
    x = torch.from_numpy(frames).to(dev)
    feats, stats0 = api.clip_features(x, geo)
    conv = api.sigma_clip(x, geo, api.Params(cutoff=3.0, max_iter=32))
    target, use = api.surrogate_targets(stats0, conv)
    model = api.Surrogate(seed=7, device=dev)
    X = feats.reshape(F * geo.n_bins, -1)
    hist = model.train(X, target, use, steps=steps, batch=2048, lr=3e-3, log_every=50)
    return model, hist


def test_trained_surrogate_matches_oracle_and_saves_passes(dev, small):
    g, sc, geo, frames = small
    _say("case: surrogate training on 8 small frames, warm-started clip on 2 others")
    model, hist = _train_small(dev, geo, frames[:8])
    assert hist[-1] < 0.5 * hist[0], hist
    p = model.half_params()
    test = frames[8:]
    x = torch.from_numpy(test).to(dev)
    params = api.Params(cutoff=3.0, max_iter=32)
    got, state = api.sigma_clip_surrogate(x, geo, params, model, widen=0.1)
    plain = api.sigma_clip(x, geo, params)
    state = state.cpu().numpy()
    n_acc = passes_plain = passes_sur = 0
    for f in range(2):
        ref = Q.surrogate_clip(test[f], None, sc.csr, p, sc.mask, 3.0, 32, 0.1)
        pl = OS.sigma_clip(test[f], None, sc.csr, sc.mask, 3.0, 32, return_margin=True)
        X, st = Q.features(test[f], None, sc.csr, sc.mask)
        y = Q.forward(p, X)
        gp = {k: v[f].cpu().numpy() for k, v in got.items()}
        for r in range(sc.csr.n_bins):
            if state[f, r] != ref["state"][r]:
                # only where a decision of the oracle sits on a threshold within rounding
                mh, sh = st[r, 1] + y[r, 0] * st[r, 2], st[r, 2] * np.exp(y[r, 1])
                half = 3.0 * 1.1 * sh
                v = OS.bin_members(test[f], None, sc.csr, r, sc.mask).v
                near = np.min(np.abs(np.abs(v - mh) - half)) / half
                m = ref if ref["state"][r] == 1 else pl
                for side in (m["mean"][r] - 3 * m["std"][r] - (mh - half), mh + half - m["mean"][r] - 3 * m["std"][r]):
                    near = min(near, abs(side) / half)
                near = min(near, pl["margin"][r])
                assert near < 1e-4, (f, r, state[f, r], ref["state"][r], near)
                continue
            if state[f, r] == 1:
                n_acc += 1
                passes_plain += plain["n_iter"][f, r].item() + plain["converged"][f, r].item()
                passes_sur += gp["n_iter"][r] + gp["converged"][r]
                for k in ("mean", "std", "sem", "sum_w"):
                    assert abs(gp[k][r] - ref[k][r]) <= 1e-5 * abs(ref[k][r]) + 1e-7 * abs(ref["mean"][r]), (f, r, k)
                assert gp["n_members"][r] == ref["n_members"][r] and gp["n_iter"][r] == ref["n_iter"][r]
            else:
                # no prediction, or refused and clipped again: exactly the plain clip
                for k in ("mean", "std", "sem", "sum_w", "n_members", "n_iter", "converged"):
                    assert gp[k][r] == plain[k][f, r].item(), (f, r, k)
    _say(f"accepted {n_acc} of {2 * geo.n_bins} bins: {passes_sur} passes instead of {passes_plain}")
    # the trained network's warm start is accepted in most bins and saves passes
    assert n_acc >= 0.5 * 2 * geo.n_bins
    assert passes_sur < passes_plain


def test_warm_start_from_given_predictions_matches_oracle(dev, small):
    """ss_sigma_clip_warm with two predictors, the plain clip's own converged
    profile (a perfect predictor) and the previous frame's profile: the
    states, statistics and passes of the oracle's warm clip with the same
    predictions; with the perfect predictor the accepted bins take fewer
    passes than the plain clip."""
    g, sc, geo, frames = small
    _say("case: warm start from given predictions, small config x3")
    params = api.Params(cutoff=3.0, max_iter=32)
    x = torch.from_numpy(frames[:3]).to(dev)
    plain = api.sigma_clip(x, geo, params)
    prev = {k: torch.roll(plain[k], 1, dims=0).contiguous() for k in ("mean", "std")}
    for name, (pm, ps) in (("own", (plain["mean"], plain["std"])), ("previous", (prev["mean"], prev["std"]))):
        got, state = api.sigma_clip_warm(x, geo, params, pm, ps, widen=0.1)
        torch.cuda.synchronize()
        state = state.cpu().numpy()
        pmh, psh = pm.cpu().numpy(), ps.cpu().numpy()
        n_acc = passes_warm = passes_plain = 0
        for f in range(3):
            ref = Q.warm_clip(frames[f], None, sc.csr, pmh[f], psh[f], sc.mask, 3.0, 32, 0.1)
            gp = {k: v[f].cpu().numpy() for k, v in got.items()}
            pl = {k: v[f].cpu().numpy() for k, v in plain.items()}
            assert np.array_equal(state[f], ref["state"]), (name, f, np.nonzero(state[f] != ref["state"])[0][:5])
            for r in range(sc.csr.n_bins):
                if state[f, r] == 1:
                    n_acc += 1
                    passes_warm += gp["n_iter"][r] + gp["converged"][r]
                    passes_plain += pl["n_iter"][r] + pl["converged"][r]
                    for k in ("mean", "std", "sem", "sum_w"):
                        tol = 1e-5 * abs(ref[k][r]) + 1e-7 * abs(ref["mean"][r])
                        assert abs(gp[k][r] - ref[k][r]) <= tol, (name, f, r, k)
                    assert gp["n_members"][r] == ref["n_members"][r] and gp["n_iter"][r] == ref["n_iter"][r]
                else:
                    for k in ("mean", "std", "sem", "sum_w", "n_members", "n_iter", "converged"):
                        assert gp[k][r] == pl[k][r], (name, f, r, k)
        _say(f"  {name}: accepted {n_acc} of {3 * geo.n_bins} bins, {passes_warm} passes instead of {passes_plain}")
        assert n_acc >= 0.5 * 3 * geo.n_bins
        if name == "own":
            assert passes_warm < passes_plain
