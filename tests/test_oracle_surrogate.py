"""Pins of the surrogate oracle: derivatives by finite differences, closed
forms of GELU and of Adam's first step, the feature sketch against the
normal distribution, and the verified clip against the plain clip's fixed
points."""

import math

import numpy as np
import pytest
from scipy.special import ndtr

from oracle import stats as S
from oracle import surrogate as Q


def test_gelu_closed_forms():
    x = np.linspace(-6, 6, 49)
    assert Q.gelu(np.array([0.0]))[0] == 0.0
    # GELU(x) - GELU(-x) = x  (erf is odd)
    assert np.allclose(Q.gelu(x) - Q.gelu(-x), x, rtol=0, atol=1e-14)
    assert abs(Q.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    h = 1e-6
    fd = (Q.gelu(x + h) - Q.gelu(x - h)) / (2 * h)
    assert np.allclose(Q.gelu_grad(x), fd, rtol=0, atol=1e-8)


def test_layout_round_trip_and_padding():
    p = Q.init_params(3)
    assert p.size == Q.N_PARAMS == 7312
    again = Q.pack(*Q.unpack(p))
    assert np.array_equal(again, p)
    W1 = p[Q.OFF_W1:Q.OFF_B1].reshape(Q.K1, Q.N_HID)
    assert np.all(W1[Q.N_IN:] == 0)
    W3 = p[Q.OFF_W3:Q.OFF_B3].reshape(Q.N_HID, Q.OUT_PAD)
    assert np.all(W3[:, Q.N_OUT:] == 0)


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(11)
    X = rng.normal(size=(9, Q.N_IN))
    T = rng.normal(size=(9, 2))
    use = np.array([1, 1, 0, 1, 1, 1, 0, 1, 1], dtype=bool)
    p = Q.init_params(5)
    p[Q.OFF_B1:Q.OFF_W2] = rng.normal(size=Q.N_HID) * 0.3
    p[Q.OFF_B3:Q.OFF_B3 + 2] = [0.2, -0.1]
    L, g = Q.loss_grad(p, X, T, use, half=False)
    # the loss itself, by its definition
    y = Q.forward(p, X, half=False)
    assert L == pytest.approx(float(np.sum(((y - T) ** 2)[use])) / use.sum(), rel=1e-14)
    W1, b1, W2, b2, W3, b3 = (np.zeros(0),) * 6  # noqa: F841
    live = [i for i in range(Q.N_PARAMS) if not (
        (Q.OFF_W1 <= i < Q.OFF_B1 and (i - Q.OFF_W1) // Q.N_HID >= Q.N_IN) or
        (Q.OFF_W3 <= i < Q.OFF_B3 and (i - Q.OFF_W3) % Q.OUT_PAD >= Q.N_OUT) or
        (i >= Q.OFF_B3 + Q.N_OUT))]
    pick = rng.choice(live, size=60, replace=False)
    h = 1e-6
    for i in pick:
        a, b = p.copy(), p.copy()
        a[i] += h
        b[i] -= h
        fd = (Q.loss_grad(a, X, T, use, half=False)[0] - Q.loss_grad(b, X, T, use, half=False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i
    dead = np.setdiff1d(np.arange(Q.N_PARAMS), live)
    assert np.all(g[dead] == 0)


def test_unused_samples_do_not_count():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(6, Q.N_IN))
    T = rng.normal(size=(6, 2))
    use = np.array([1, 0, 1, 0, 1, 1], dtype=bool)
    p = Q.init_params(1)
    L1, g1 = Q.loss_grad(p, X, T, use)
    L2, g2 = Q.loss_grad(p, X[use], T[use])
    assert L1 == pytest.approx(L2, rel=1e-14)
    assert np.allclose(g1, g2, rtol=1e-12, atol=0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-2, 1e-8
    p1, m, v, h = Q.adam(p, np.zeros(50), np.zeros(50), g, 1, lr=lr, eps=eps)
    # bias correction makes the first moments g and g^2 exactly
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-13, atol=0)
    assert np.array_equal(h, p1.astype(np.float16).astype(np.float64))
    # a constant gradient keeps moving every coordinate by about lr
    q, mm, vv = p1, m, v
    for t in range(2, 30):
        q, mm, vv, _ = Q.adam(q, mm, vv, g, t, lr=lr, eps=eps)
    assert np.allclose(p - q, 29 * lr * g / (np.abs(g) + eps), rtol=1e-9)


def test_feature_sketch_of_a_normal_sample():
    rng = np.random.default_rng(4)
    n = 200_000
    v = rng.normal(5.0, 2.0, n)
    x, (nn, m0, s0) = Q.bin_features(v, np.ones(n))
    assert nn == n and x[0] == pytest.approx(math.log1p(n))
    assert x[1] == pytest.approx(math.asinh(np.mean(v)), rel=1e-12)
    assert x[2] == pytest.approx(math.asinh(np.std(v)), rel=1e-12)
    want = ndtr(Q.THRESHOLDS)
    tol = 4 * np.sqrt(want * (1 - want) / n) + 2e-4  # binomial error + sample-moment error
    assert np.all(np.abs(x[3:] - want) <= tol)
    assert np.all(np.diff(x[3:]) >= 0)


def test_feature_sketch_counts_ties_below():
    # values on the thresholds themselves count as below (<=)
    v = np.array([0.0, 0.0, 1.0, 1.0])
    x, (n, m0, s0) = Q.bin_features(v, np.ones(4))
    assert (m0, s0) == (0.5, 0.5)
    # thresholds m0 + t s0 = 0.5 + 0.5 t: t = -1 -> 0.0 (k = 5.5, not a grid point), t = +1 -> 1.0
    k_of = {t: k for k, t in enumerate(Q.THRESHOLDS)}
    assert -1.0 not in k_of  # the grid is -3.75, -3.25, ...
    assert np.array_equal(x[3:], np.where(Q.THRESHOLDS >= 1.0, 1.0, np.where(Q.THRESHOLDS >= -1.0, 0.5, 0.0)))


def test_targets_round_trip():
    st = np.array([[10, 4.0, 2.0], [1, 3.0, 0.0], [50, -1.0, 0.5]])
    mc, sc = np.array([3.5, 3.0, -1.1]), np.array([1.5, 0.0, 0.25])
    T, use = Q.targets(st, mc, sc, [1, 1, 1], [8, 1, 40])
    assert list(use) == [True, False, True]
    back_m = st[:, 1] + T[:, 0] * st[:, 2]
    back_s = st[:, 2] * np.exp(T[:, 1])
    assert np.allclose(back_m[use], mc[use], rtol=1e-15) and np.allclose(back_s[use], sc[use], rtol=1e-15)


def _converged_plain(v, omega, cutoff):
    keep, n_iter, conv, _ = S._clip_bin(v, omega, np.zeros_like(v), cutoff, 64, S.AZIMUTHAL)
    assert conv == 1
    return keep, S.moments(v[keep], omega[keep]), n_iter


def test_warm_start_from_the_converged_answer_reproduces_the_plain_clip():
    """A prediction equal to the plain clip's converged statistics reaches
    the same member set in fewer passes, and is accepted."""
    rng = np.random.default_rng(8)
    saved = 0
    for trial in range(30):
        v = np.concatenate([rng.normal(10, 1, 400), rng.uniform(15, 60, rng.integers(0, 30))])
        omega = rng.uniform(0.5, 1.5, v.size)
        keep, m, n_plain = _converged_plain(v, omega, 3.0)
        state, kw, n_warm, conv = Q.warm_bin(v, omega, m["mean"], m["std"], 3.0, 64, 0.1)
        assert conv == 1 and np.array_equal(kw, keep)
        assert state == 1
        assert n_warm <= n_plain
        saved += n_plain - n_warm
    assert saved > 0


def test_warm_start_with_zero_widening_is_at_least_as_tight():
    rng = np.random.default_rng(10)
    v = np.concatenate([rng.normal(0, 1, 2000), rng.uniform(5, 30, 50)])
    omega = np.ones(v.size)
    keep, m, _ = _converged_plain(v, omega, 3.0)
    # a prediction a little too tight removes members the plain clip keeps: refused
    state, kw, _, _ = Q.warm_bin(v, omega, m["mean"], 0.8 * m["std"], 3.0, 64, 0.0)
    assert state == -1
    # a looser prediction removes only what the plain clip removes too
    state, kw, _, _ = Q.warm_bin(v, omega, m["mean"], 1.5 * m["std"], 3.0, 64, 0.0)
    assert state == 1 and np.array_equal(kw, keep)


def test_surrogate_clip_equals_the_plain_clip_where_refused():
    from oracle import geometry as G
    import synth
    g = synth.SMALL
    mask = synth.stripe_mask(g)
    frame = synth.float_frame(g, 0)[0]
    csr = G.csr_for(g, mask)
    p = Q.init_params(0)  # untrained
    out = Q.surrogate_clip(frame, None, csr, p, mask, 3.0, 32, 0.1)
    plain = S.sigma_clip(frame.reshape(-1), None, csr, mask.reshape(-1), 3.0, 32)
    rej = out["state"] != 1
    for k in ("mean", "std", "n_members", "n_iter", "converged"):
        assert np.array_equal(out[k][rej], plain[k][rej])
    # accepted bins hold the plain clip's member set too
    acc = ~rej
    assert np.array_equal(out["n_members"][acc], plain["n_members"][acc])
    assert np.allclose(out["mean"][acc], plain["mean"][acc], rtol=1e-12)
