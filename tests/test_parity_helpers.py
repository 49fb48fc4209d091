"""The parity helpers themselves, on the CPU: the replay of band decisions,
the derived band and the classification comparison, exercised with the
oracle and with an emulation of the GPU's float32 inputs (oracle arithmetic
on RN32(signal / norm) values and RN32(c norm) weights), and shown to reject
planted mistakes."""

import math

import numpy as np
import pytest

import synth
from oracle import classify as OK
from oracle import geometry as OG
from oracle import stats as OS

import parity as P
from paper_2411_09515_amd import api


class _OneRow:
    def __init__(self, c):
        self.n_bins = 1
        self.n_pix = len(c)
        self.indptr = np.array([0, len(c)])
        self.indices = np.arange(len(c))
        self.coef = np.asarray(c, dtype=np.float64)

    def row(self, r):
        return self.indices, self.coef


def _bin_with_member_at_threshold(delta, n=3.0):
    """200 members around 100 and one member x with |x - m| - n s = delta
    (relative to n s) for the statistics of all 201 (bisection in float64)."""
    rng = np.random.default_rng(4)
    base = rng.normal(100.0, 5.0, 200)

    def d(x):
        v = np.append(base, x)
        m = v.mean()
        return abs(x - m) - n * v.std(), n * v.std()

    lo, hi = 100.0, 200.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if d(mid)[0] > 0:
            hi = mid
        else:
            lo = mid
    x = hi
    thr = d(x)[1]
    x = x + delta * thr
    return np.append(base, x)


def _gpu_like(g):
    return {k: np.array([g[k]]) for k in ("mean", "std", "sem", "sum_w", "n_members", "n_iter", "converged")}


def test_band_member_gives_both_outcomes():
    v = _bin_with_member_at_threshold(1e-9)
    mb = OS.bin_members(v, None, _OneRow(np.ones(v.size)), 0)
    out, complete = P.clip_outcomes(mb, 3.0, 5, OS.AZIMUTHAL, P.U32, P.U32)
    assert complete
    # the member (the last one) stays in one outcome and goes in another
    assert any(k[-1] for k, _, _ in out) and any(not k[-1] for k, _, _ in out)
    # far outside the band: one outcome only
    v = _bin_with_member_at_threshold(1e-3)
    mb = OS.bin_members(v, None, _OneRow(np.ones(v.size)), 0)
    out, complete = P.clip_outcomes(mb, 3.0, 5, OS.AZIMUTHAL, P.U32, P.U32)
    assert complete and len(out) == 1


def test_replay_accepts_the_flipped_outcome_and_nothing_else():
    # 1e-6 of the threshold: inside the band of float32 inputs (~7e-6 here),
    # outside the float64 allowance alone (~1e-7)
    v = _bin_with_member_at_threshold(1e-6)
    csr = _OneRow(np.ones(v.size))
    p = api.Params()
    ref = OS.sigma_clip(v, None, csr, cutoff=3.0, max_iter=5)
    # the other decision for the band member: it stays (or goes) in pass 0
    mb = OS.bin_members(v, None, csr, 0)
    outs, _ = P.clip_outcomes(mb, 3.0, 5, OS.AZIMUTHAL, P.U32, P.U32)
    other = [o for o in outs if int(o[0].sum()) != int(ref["n_members"][0])]
    assert other
    keep, n_iter, conv = other[0]
    m = OS.moments(mb.v[keep], mb.omega[keep])
    gpu = _gpu_like(dict(mean=m["mean"], std=m["std"], sem=m["sem"], sum_w=m["Omega"], n_members=m["n"],
                         n_iter=n_iter, converged=conv))
    res, counts = P.compare_profile(gpu, v, None, csr, None, p, P.U32, P.U32, "flip")
    assert counts["replayed"] == 1 and counts["unresolved"] == 0
    assert res["n_members"][0] == m["n"]
    # without the band (exact inputs) the flipped outcome is refused
    with pytest.raises(AssertionError):
        P.compare_profile(gpu, v, None, csr, None, p, 0.0, 0.0, "no band")
    # a statistic off by 1e-4 is refused whatever the band
    bad = {k: a.copy() for k, a in gpu.items()}
    bad["mean"] = bad["mean"] * (1 + 1e-4)
    with pytest.raises(AssertionError):
        P.compare_profile(bad, v, None, csr, None, p, P.U32, P.U32, "off")


@pytest.fixture(scope="module")
def emulated():
    """A Jungfrau-1M frame through the oracle, and through the oracle's
    arithmetic on the GPU's float32 inputs (values RN32(signal / norm),
    weights RN32(c norm)): the profile and lists a correct GPU could give."""
    g = synth.JUNGFRAU1M
    sc = P.OracleScene(g)
    raw = synth.jungfrau_frames(g, 1, first=2).reshape(1, -1)
    signal, _ = sc.signal_from_raw(raw)
    signal = signal[0]
    v32 = sc.corrected(signal[None, :])[0]
    w32 = OG.Csr(sc.csr.n_bins, sc.csr.n_pix, sc.csr.indptr, sc.csr.indices,
                 (sc.csr.coef * sc.norm.astype(np.float64)[sc.csr.indices]).astype(np.float32).astype(np.float64),
                 sc.csr.tth_max, sc.csr.width)
    p = api.Params()
    gpu = OS.sigma_clip(v32, None, w32, sc.mask, cutoff=3.0, max_iter=5)
    ki, kv = OK.compress(v32, sc.mask, sc.position, sc.centres, gpu, 3.0)
    pk = OK.peakfind(v32, sc.mask, g.height, g.width, sc.position, sc.centres, gpu, 3.0, 3, 3)
    return sc, signal, p, gpu, ki, kv.astype(np.float32), pk


def test_emulated_gpu_inputs_pass_the_replay(emulated):
    sc, signal, p, gpu, ki, kv, pk = emulated
    res, counts = sc.check_profile(gpu, signal, p, "emulated 1M")
    assert counts["unresolved"] == 0
    assert counts["replayed"] <= 2, counts   # float32 inputs flip a decision very rarely
    c = sc.check_classify(signal, gpu, res, ki, kv, pk, p, "emulated 1M")
    assert c["excused_keep"] <= 1e-3 * c["valid"] and c["excused_cand"] <= 1e-3 * c["valid"], c
    assert c["kept"] > 1000 and c["peaks"] > 0


def test_planted_list_mistakes_are_caught(emulated):
    sc, signal, p, gpu, ki, kv, pk = emulated
    res, _ = sc.check_profile(gpu, signal, p, "emulated 1M")
    # one kept pixel missing (the middle one: far from the band)
    drop = np.arange(ki.size) != ki.size // 2
    with pytest.raises(AssertionError):
        sc.check_classify(signal, gpu, res, ki[drop], kv[drop], pk, p, "missing kept")
    # one kept value off by one float32 ulp
    kv2 = kv.copy()
    kv2[3] = np.nextafter(kv2[3], np.float32(np.inf))
    with pytest.raises(AssertionError):
        sc.check_classify(signal, gpu, res, ki, kv2, pk, p, "kept value")
    # a peak dropped
    if pk.size:
        with pytest.raises(AssertionError):
            sc.check_classify(signal, gpu, res, ki, kv, pk[1:], p, "missing peak")


def test_band_is_tight_for_float32_frames():
    """With exact inputs (float32 frames, unit weights) the band is the
    float64 allowance alone: well under 1e-7 of the threshold for counts."""
    rng = np.random.default_rng(8)
    v = rng.poisson(100.0, 5000).astype(np.float64)
    mb = OS.bin_members(v, None, _OneRow(np.ones(v.size)), 0)
    keep = np.ones(v.size, dtype=bool)
    m = OS.moments(mb.v, mb.omega)
    tau = P.clip_band(mb, keep, m, m["std"], 3.0, OS.AZIMUTHAL, 0.0, 0.0)
    assert np.all(tau <= 1e-7 * 3.0 * m["std"])
    tau32 = P.clip_band(mb, keep, m, m["std"], 3.0, OS.AZIMUTHAL, P.U32, P.U32)
    assert tau32.max() > 10 * tau.max()
    assert math.isfinite(tau32.max())
