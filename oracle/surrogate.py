"""Learned clip surrogate: features, the MLP, its gradient, Adam, and the
verified clip (FP64 reference).  TEST INFRASTRUCTURE ONLY.

The paper has no surrogate; its run time is set by the number of clipping
passes (Sec. 2.4: execution time grows with the iterations, three being
common).  This module states the surrogate's definitions; they are pinned
by mathematics (finite differences, closed forms, fixed points) and by the
plain clip of ``stats``, not by the paper (parity unpinned by the paper).

Features of one bin (unclipped azimuthal statistics of all members,
``stats.moments``; n members, mean m0, std s0):
  x0 = log(1 + n), x1 = asinh(m0), x2 = asinh(s0),
  x(3 + k) = #{members with v <= m0 + t_k s0} / n,  t_k = -3.75 + 0.5 k,
  k = 0 .. 15  (a 16-point sketch of the standardised value distribution).
  A bin with no member has all features 0.

Targets (the plain clip run to convergence, mean mc, std sc):
  y0 = (mc - m0) / s0,  y1 = log(sc / s0);  a prediction (y0, y1) gives
  mean_hat = m0 + y0 s0 and std_hat = s0 exp(y1).

Network: 19 -> 64 -> 64 -> 2, GELU (exact, with erf) after the two hidden
layers.  The parameters live in one float array (layout below); the network
evaluates with every parameter rounded to float16 and float32-or-better
arithmetic.  Loss: mean over the used samples of the squared error summed
over the two outputs.

Warm-started clip of one bin (cut-off c > 0, widening w >= 0):
  pass 0 of the plain clip removes the members outside the intersection of
  its own bounds (mean +- c std of all members) and the predicted bounds
  mean_hat +- c (1 + w) std_hat; the passes after it are the plain clip's
  (eq. clip, same stopping rule and pass limit).  The result is accepted
  (state 1) when the clip converged, its final bounds lie inside the
  predicted ones and the final set is exactly the members within the final
  bounds (no removed member lies within them); otherwise (state -1) the bin
  is clipped again from scratch by the plain clip.  A bin without a usable
  prediction runs the plain clip (state 0): fewer than 64 members, zero
  spread, or a predicted interval reaching zero (low counts); such bins can
  have several fixed points (for low counts, one per photon-number cluster),
  and a warm start could settle on another one.
"""

from __future__ import annotations

import math

import numpy as np

from . import stats as S

N_IN, N_HID, N_OUT = 19, 64, 2
K1 = 32            # input rows of W1 (19 used, the rest zero)
OUT_PAD = 16       # columns of W3 / entries of b3 (2 used)
THRESHOLDS = -3.75 + 0.5 * np.arange(16)
MIN_MEMBERS = 64   # smallest bin the warm start is tried on

# parameter layout (float offsets)
OFF_W1 = 0
OFF_B1 = OFF_W1 + K1 * N_HID
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID * OUT_PAD
N_PARAMS = OFF_B3 + OUT_PAD


def unpack(p):
    """Views (W1 [19][64], b1, W2 [64][64], b2, W3 [64][2], b3 [2]) of a parameter array."""
    p = np.asarray(p, dtype=np.float64)
    W1 = p[OFF_W1:OFF_B1].reshape(K1, N_HID)[:N_IN]
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(N_HID, N_HID)
    b2 = p[OFF_B2:OFF_W3]
    W3 = p[OFF_W3:OFF_B3].reshape(N_HID, OUT_PAD)[:, :N_OUT]
    b3 = p[OFF_B3:OFF_B3 + N_OUT]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    p = np.zeros(N_PARAMS)
    p[OFF_W1:OFF_B1].reshape(K1, N_HID)[:N_IN] = W1
    p[OFF_B1:OFF_W2] = b1
    p[OFF_W2:OFF_B2] = np.asarray(W2).reshape(-1)
    p[OFF_B2:OFF_W3] = b2
    p[OFF_W3:OFF_B3].reshape(N_HID, OUT_PAD)[:, :N_OUT] = W3
    p[OFF_B3:OFF_B3 + N_OUT] = b3
    return p


def to_half(p):
    """The parameters as the network uses them: rounded to float16."""
    return np.asarray(p, dtype=np.float64).astype(np.float16).astype(np.float64)


def init_params(seed=0):
    """Seeded initial parameters (uniform +-1/sqrt(fan_in) weights, zero biases)."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (N_IN, N_HID)) / math.sqrt(N_IN)
    W2 = rng.uniform(-1, 1, (N_HID, N_HID)) / math.sqrt(N_HID)
    W3 = rng.uniform(-1, 1, (N_HID, N_OUT)) / math.sqrt(N_HID)
    return pack(W1, np.zeros(N_HID), W2, np.zeros(N_HID), W3, np.zeros(N_OUT))


# ---------------------------------------------------------------- features

def bin_features(v, omega, cutoff_unused=None):
    """Features (19,) and unclipped (n, mean, std) of one member set."""
    m = S.moments(v, omega)
    n = m["n"]
    x = np.zeros(N_IN)
    if n == 0:
        return x, (0, 0.0, 0.0)
    m0, s0 = m["mean"], m["std"]
    x[0] = math.log1p(n)
    x[1] = math.asinh(m0)
    x[2] = math.asinh(s0)
    v = np.asarray(v, dtype=np.float64)
    for k, t in enumerate(THRESHOLDS):
        x[3 + k] = np.count_nonzero(v <= m0 + t * s0) / n
    return x, (n, m0, s0)


def features(frame, norm, csr, mask=None):
    """Per-bin features [n_bins][19] and unclipped stats [n_bins][3] of one frame."""
    frame = np.asarray(frame).reshape(-1)
    norm = None if norm is None else np.asarray(norm).reshape(-1)
    mask = None if mask is None else np.asarray(mask).reshape(-1)
    X = np.zeros((csr.n_bins, N_IN))
    st = np.zeros((csr.n_bins, 3))
    for r in range(csr.n_bins):
        mb = S.bin_members(frame, norm, csr, r, mask)
        X[r], st[r] = bin_features(mb.v, mb.omega)
    return X, st


def targets(stats0, mean_c, std_c, converged, n_members):
    """Training targets [n][2] and the mask of usable samples."""
    n0, m0, s0 = (np.asarray(stats0)[:, i] for i in range(3))
    use = (n0 >= 2) & (s0 > 0) & (np.asarray(converged) == 1) & (np.asarray(n_members) >= 2) & \
          (np.asarray(std_c) > 0)
    T = np.zeros((len(n0), 2))
    T[use, 0] = (np.asarray(mean_c)[use] - m0[use]) / s0[use]
    T[use, 1] = np.log(np.asarray(std_c)[use] / s0[use])
    return T, use


# ---------------------------------------------------------------- network

def gelu(u):
    from scipy.special import erf
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def forward(p, X, keep=False, half=True):
    """Network outputs [n][2] for features X [n][19] (parameters rounded to
    float16 unless ``half`` is False)."""
    W1, b1, W2, b2, W3, b3 = unpack(to_half(p) if half else p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    y = h2 @ W3 + b3
    if keep:
        return y, (X, z1, h1, z2, h2)
    return y


def loss_grad(p, X, T, use=None, half=True):
    """Loss and its gradient with respect to the (float16-rounded) parameters.

    L = (1 / n_used) sum over used samples of sum_o (y_o - t_o)^2.  The
    gradient is laid out like the parameters (zero in the padding).  With
    ``half`` False the parameters are used as given (for derivative checks).
    """
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    use = np.ones(len(X), dtype=bool) if use is None else np.asarray(use, dtype=bool)
    n_used = int(use.sum())
    W1, b1, W2, b2, W3, b3 = unpack(to_half(p) if half else p)
    y, (x, z1, h1, z2, h2) = forward(p, X, keep=True, half=half)
    if n_used == 0:
        return 0.0, np.zeros(N_PARAMS)
    r = (y - T) * use[:, None]
    L = float(np.sum(r * r)) / n_used
    dy = 2.0 * r / n_used
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * gelu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    return L, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(p, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, 2015) on float parameters; step counts from 1.

    Returns updated (p, m, v) and the float16 copy the network uses.
    """
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    p = np.asarray(p, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v, to_half(p)


# ---------------------------------------------------------------- verified clip

def warm_bin(v, omega, mean_hat, std_hat, cutoff, max_iter, widen):
    """(state, keep, n_iter, converged) of the warm-started clip of one bin."""
    v = np.asarray(v, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    keep = np.ones(v.size, dtype=bool)
    n_iter, converged = 0, 0
    half = cutoff * (1.0 + widen) * std_hat
    for k in range(max_iter):
        m = S.moments(v[keep], omega[keep])
        dev = np.abs(v - m["mean"])
        drop = keep & (dev > cutoff * m["std"])
        if k == 0:
            drop |= keep & (np.abs(v - mean_hat) > half)
        if not drop.any():
            converged = 1
            break
        keep &= ~drop
        n_iter += 1
    m = S.moments(v[keep], omega[keep])
    inside = (m["mean"] - cutoff * m["std"] >= mean_hat - half) and (m["mean"] + cutoff * m["std"] <= mean_hat + half)
    exact = np.array_equal(np.abs(v - m["mean"]) <= cutoff * m["std"], keep)
    state = 1 if (converged and inside and exact) else -1
    return state, keep, n_iter, converged


def warm_clip(frame, norm, csr, mean_hat, std_hat, mask=None, cutoff=3.0, max_iter=32, widen=0.1, stats0=None):
    """Profile of one frame from the clip warm-started by given per-bin
    predictions of the converged mean and std (``mean_hat``, ``std_hat``
    [n_bins]: the network's, or any other predictor's), plain clip as the
    fallback.  A bin gets a warm start when it has at least MIN_MEMBERS
    members, a positive unclipped std, a positive predicted std and a
    predicted interval mean_hat - cutoff (1 + widen) std_hat above zero.

    Returns the dict of ``stats.sigma_clip`` plus ``state`` per bin (1 warm
    start accepted, 0 no warm start, -1 clipped again from scratch).
    """
    frame = np.asarray(frame).reshape(-1)
    normf = None if norm is None else np.asarray(norm).reshape(-1)
    maskf = None if mask is None else np.asarray(mask).reshape(-1)
    plain = S.sigma_clip(frame, normf, csr, maskf, cutoff, max_iter)
    st = features(frame, normf, csr, maskf)[1] if stats0 is None else stats0
    out = {k: np.array(val, copy=True) for k, val in plain.items()}
    out["state"] = np.zeros(csr.n_bins, dtype=np.int64)
    for r in range(csr.n_bins):
        n0, m0, s0 = st[r]
        if n0 < 2 or not (s0 > 0) or max_iter < 1:
            continue
        mh, sh = float(mean_hat[r]), float(std_hat[r])
        if n0 < MIN_MEMBERS or not (sh > 0) or not (mh - cutoff * (1.0 + widen) * sh > 0):
            continue
        mb = S.bin_members(frame, normf, csr, r, maskf)
        v, omega = mb.v, mb.omega
        state, keep, n_iter, conv = warm_bin(v, omega, mh, sh, cutoff, max_iter, widen)
        out["state"][r] = state
        if state != 1:
            continue
        m = S.moments(v[keep], omega[keep])
        out["mean"][r], out["std"][r], out["sem"][r] = m["mean"], m["std"], m["sem"]
        out["sum_w"][r], out["n_members"][r] = m["Omega"], m["n"]
        out["n_iter"][r], out["converged"][r] = n_iter, conv
    return out


def surrogate_clip(frame, norm, csr, p, mask=None, cutoff=3.0, max_iter=32, widen=0.1):
    """Profile of one frame from the warm-started clip, the network's
    prediction from the bin's features (``warm_clip``), plain clip as the
    fallback."""
    frame = np.asarray(frame).reshape(-1)
    normf = None if norm is None else np.asarray(norm).reshape(-1)
    maskf = None if mask is None else np.asarray(mask).reshape(-1)
    X, st = features(frame, normf, csr, maskf)
    y = forward(p, X)
    mean_hat = st[:, 1] + y[:, 0] * st[:, 2]
    std_hat = st[:, 2] * np.exp(y[:, 1])
    return warm_clip(frame, normf, csr, mean_hat, std_hat, maskf, cutoff, max_iter, widen, stats0=st)
