"""Pins of the oracle's per-bin statistics and sigma-clipping (CPU only)."""

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import geometry as G
from oracle import stats as S


class _OneRowCsr:
    """A CSR with a single row holding pixels 0..n-1 with coefficients c."""

    def __init__(self, c):
        self.n_bins = 1
        self.n_pix = len(c)
        self.indptr = np.array([0, len(c)])
        self.indices = np.arange(len(c))
        self.coef = np.asarray(c, dtype=np.float64)

    def row(self, r):
        return self.indices, self.coef


def _clip(values, c=None, norm=None, **kw):
    values = np.asarray(values, dtype=np.float64)
    c = np.ones(values.size) if c is None else c
    return S.sigma_clip(values, norm, _OneRowCsr(c), **kw)


# -- the paper's worked examples -------------------------------------------

def test_two_pixel_example(golden):
    gd = golden("two_pixel_example.txt")
    v = np.array(gd["values"])
    m = S.moments(v, np.ones(2), np.maximum(v, 0))
    assert m["mean"] == gd["mean"]
    # population std (ddof = 0) is 99, "close to 100"; ddof = 1 would be 140
    assert m["std"] == pytest.approx(99.0, abs=1e-12)
    assert abs(m["std"] - gd["azimuthal_std_approx"]) <= 1.0
    assert abs(m["std_p"] - gd["poisson_std_approx"]) <= 0.1
    dev = np.abs(v - m["mean"])
    assert np.allclose(dev / m["std"], gd["azimuthal_deviation_sigma"])
    assert np.allclose(dev / m["std_p"], gd["poisson_deviation_sigma_approx"], rtol=0.02)


def test_two_pixel_example_clipping():
    # azimuthal model: both pixels sit exactly at 1 sigma: nothing goes at n >= 1
    out = _clip([1, 199], cutoff=3.0, max_iter=5)
    assert out["n_members"][0] == 2 and out["converged"][0] == 1 and out["n_iter"][0] == 0
    out = _clip([1, 199], cutoff=1.0, max_iter=5)
    assert out["n_members"][0] == 2
    # ... and both go below 1 sigma, leaving an empty bin
    out = _clip([1, 199], cutoff=0.9, max_iter=5)
    assert out["n_members"][0] == 0 and out["mean"][0] == 0.0 and out["n_iter"][0] == 1
    # Poisson model: both pixels at ~10 sigma: the bin is emptied (the
    # artefact that motivated the azimuthal model)
    out = _clip([1, 199], cutoff=3.0, max_iter=5, error_model=S.POISSON)
    assert out["n_members"][0] == 0
    # hybrid: clip with the azimuthal spread, report the Poisson one
    out = _clip([1, 199], cutoff=3.0, max_iter=5, error_model=S.HYBRID)
    assert out["n_members"][0] == 2 and out["std"][0] == pytest.approx(10.0)


def test_chauvenet_values(golden):
    gd = golden("chauvenet.txt")
    assert round(S.chauvenet(100), 1) == gd["size_100_cutoff_1dp"]
    assert round(S.chauvenet(1000), 1) == gd["size_1000_cutoff_1dp"]
    assert S.chauvenet(2) == math.inf
    assert S.chauvenet(100) == pytest.approx(2.7152, abs=1e-4)
    assert S.chauvenet(1000) == pytest.approx(3.4609, abs=1e-4)


def _lambda1_ensemble(size, top):
    """Integers with mean exactly 1 and population std exactly 1, holding one
    value ``top`` and one ``top - 1``, the rest in {0, 1, 2}."""
    rest = size - 2
    s1 = size - (2 * top - 1)
    s2 = 2 * size - (top * top + (top - 1) ** 2)
    c2 = (s2 - s1) // 2
    c1 = s1 - 2 * c2
    c0 = rest - c1 - c2
    v = np.array([0] * c0 + [1] * c1 + [2] * c2 + [top - 1, top], dtype=np.float64)
    assert v.size == size and v.mean() == 1.0 and v.std() == 1.0
    return v


def test_chauvenet_lambda1_example(golden):
    gd = golden("chauvenet.txt")
    for size, key in ((100, "size_100_lambda1_smallest_discarded"), (1000, "size_1000_lambda1_smallest_discarded")):
        top = int(gd[key])
        v = _lambda1_ensemble(size, top)
        out = S.sigma_clip(v, None, _OneRowCsr(np.ones(size)), cutoff=0.0, max_iter=1,
                           return_keep=True)
        _, keep = out["keep"][0]
        assert np.all(keep[v < top]) and not np.any(keep[v >= top])


# -- closed forms and identities ---------------------------------------------

def test_unit_weights_reduce_to_numpy(rng):
    for n in (1, 2, 7, 100, 1001):
        v = rng.normal(50.0, 7.0, n)
        m = S.moments(v, np.ones(n))
        assert m["mean"] == pytest.approx(np.mean(v), rel=1e-13)
        assert m["std"] == pytest.approx(np.std(v), rel=1e-12, abs=1e-12)
        assert m["sem"] == pytest.approx(np.std(v) / math.sqrt(n), rel=1e-12, abs=1e-12)


def _grow_with_union(v, w):
    """VV grown one member at a time with eq. union_variance1."""
    Om, V, VV = w[0], w[0] * v[0], 0.0
    for b in range(1, len(v)):
        mean_a = V / Om
        Om2, V2 = Om + w[b], V + w[b] * v[b]
        VV = VV + w[b] ** 2 * (v[b] - mean_a) * (v[b] - V2 / Om2)
        Om, V = Om2, V2
    return Om, V, VV


def test_union_formula_builds_the_same_vv(rng):
    """With equal weights, VV grown with the paper's single-member union
    (eq. union_variance1) equals the two-pass VV; with unequal weights the
    union is only approximate (the paper calls its merge approximate), which
    is why the two-pass definition is the oracle."""
    for n in (2, 5, 50, 400):
        v = rng.normal(100.0, 10.0, n)
        w = np.full(n, 0.7)
        Om, V, VV = _grow_with_union(v, w)
        m = S.moments(v, w)
        assert m["Omega"] == pytest.approx(Om, rel=1e-13)
        assert m["V"] == pytest.approx(V, rel=1e-13)
        assert m["VV"] == pytest.approx(VV, rel=1e-10)
    v = rng.normal(100.0, 10.0, 400)
    w = rng.uniform(0.05, 1.0, 400)
    _, _, VV = _grow_with_union(v, w)
    err = abs(VV - S.moments(v, w)["VV"]) / S.moments(v, w)["VV"]
    assert 1e-6 < err < 0.5


def test_sem_forms_agree(rng):
    """eq. sem (std * sqrt(sum w^2) / sum w) equals eq. sem2 (sqrt(VV) / Omega)."""
    v = rng.normal(10.0, 2.0, 300)
    w = rng.uniform(0.1, 2.0, 300)
    m = S.moments(v, w)
    assert m["sem"] == pytest.approx(m["std"] * math.sqrt(np.sum(w * w)) / np.sum(w), rel=1e-13)


def test_weighted_mean_is_ratio_of_sums(rng):
    """eq. avg: sum c * signal / sum c * norm, via the CSR members."""
    n = 200
    signal = rng.uniform(10, 100, n)
    norm = rng.uniform(0.3, 1.0, n)
    c = rng.uniform(0.05, 1.0, n)
    out = S.integrate(signal, norm, _OneRowCsr(c))
    assert out["mean"][0] == pytest.approx(np.dot(c, signal) / np.dot(c, norm), rel=1e-14)
    assert out["sum_w"][0] == pytest.approx(np.dot(c, norm), rel=1e-14)


def test_statistics_use_the_unrounded_quotient():
    """The float32 signal and norm enter eq. avg and the deviations in
    float64: the result is the exact-arithmetic value of the definition, not
    the one of a float32-rounded corrected frame (which is off by up to 2^-24
    per value).  Exact rational arithmetic decides."""
    rng = np.random.default_rng(77)
    n = 64
    signal = rng.uniform(10, 100, n).astype(np.float32)
    norm = (1.0 / rng.integers(3, 11, n)).astype(np.float32)   # quotients far from float32 values
    c = rng.uniform(0.05, 1.0, n)
    out = S.integrate(signal, norm, _OneRowCsr(c))
    fc = [Fraction(float(x)) for x in c]
    fs = [Fraction(float(x)) for x in signal]
    fn = [Fraction(float(x)) for x in norm]
    mean = sum(a * b for a, b in zip(fc, fs)) / sum(a * b for a, b in zip(fc, fn))
    vv = sum((a * b) ** 2 * (s / b - mean) ** 2 for a, b, s in zip(fc, fn, fs))
    oo = sum((a * b) ** 2 for a, b in zip(fc, fn))
    assert abs(Fraction(out["mean"][0]) - mean) <= Fraction(1, 10 ** 14) * mean
    assert out["std"][0] == pytest.approx(math.sqrt(vv / oo), rel=1e-13)
    # the float32 corrected frame gives a measurably different mean
    v32 = (signal.astype(np.float64) / norm).astype(np.float32).astype(np.float64)
    w = c * norm.astype(np.float64)
    m32 = np.dot(w, v32) / np.sum(w)
    assert abs(m32 - float(mean)) > 1e3 * abs(out["mean"][0] - float(mean))


def test_flat_image_any_split():
    """signal = k * norm gives mean k and std 0 in every non-empty bin."""
    for split in ("none", "bbox"):
        H, W = 40, 44
        csr = G.build_csr(H, W, 75e-6, 0.003, 19.2, 20.7, 30, split)
        norm = np.linspace(0.5, 1.0, H * W)
        k = 37.25
        out = S.integrate(k * norm, norm, csr)
        ne = out["n_members"] > 0
        assert ne.all()
        assert np.allclose(out["mean"][ne], k, rtol=1e-14)
        assert np.all(out["std"][ne] <= 1e-12 * k)


def test_piecewise_constant_profile_no_split():
    H, W, nb = 30, 30, 20
    csr = G.build_csr(H, W, 75e-6, 0.003, 14.5, 15.5, nb, "none")
    rows = np.repeat(np.arange(nb), np.diff(csr.indptr))
    image = np.zeros(H * W)
    image[csr.indices] = 3.0 * rows + 1.0
    out = S.integrate(image, None, csr)
    ne = out["n_members"] > 0
    assert np.array_equal(out["mean"][ne], 3.0 * np.arange(nb)[ne] + 1.0)
    assert np.all(out["std"][ne] == 0.0)


def test_empty_bin_is_zero():
    out = _clip([np.nan, np.nan], max_iter=5)
    assert out["n_members"][0] == 0 and out["mean"][0] == 0 and out["std"][0] == 0


def test_zero_spread_removes_nothing():
    out = _clip([5.0] * 10, cutoff=0.5, max_iter=5)
    assert out["n_members"][0] == 10 and out["converged"][0] == 1


# -- exact brute force on tiny bins ------------------------------------------

def _exact_clip(values, weights, n, max_iter):
    """The iteration of Sec. 2.4 in exact rational arithmetic."""
    members = list(range(len(values)))
    history = []
    for _ in range(max_iter):
        if not members:
            history.append(set())
            break
        Om = sum(weights[i] for i in members)
        OO = sum(weights[i] ** 2 for i in members)
        m = sum(weights[i] * values[i] for i in members) / Om
        VV = sum(weights[i] ** 2 * (values[i] - m) ** 2 for i in members)
        drop = {i for i in members if (values[i] - m) ** 2 > n * n * VV / OO}
        margin = min((abs((values[i] - m) ** 2 - n * n * VV / OO) for i in members), default=1)
        history.append(drop)
        if not drop:
            break
        members = [i for i in members if i not in drop]
    return members, history, margin


def test_clip_matches_exact_rational(rng):
    checked = 0
    for case in range(400):
        size = int(rng.integers(1, 9))
        vals = [Fraction(int(x)) for x in rng.integers(0, 40, size)]
        if rng.random() < 0.3:
            vals[int(rng.integers(size))] = Fraction(int(rng.integers(100, 400)))
        ws = [Fraction(int(x), 8) for x in rng.integers(1, 17, size)]
        n = Fraction(int(rng.integers(4, 13)), 4)
        members, hist, margin = _exact_clip(vals, ws, n, 5)
        if margin != 0 and margin < Fraction(1, 10 ** 9):
            continue
        v = np.array([float(x) for x in vals])
        c = np.array([float(x) for x in ws])
        out = S.sigma_clip(v, None, _OneRowCsr(c), cutoff=float(n), max_iter=5, return_keep=True)
        _, keep = out["keep"][0]
        assert sorted(np.nonzero(keep)[0].tolist()) == members, (case, vals, ws, n)
        assert out["n_iter"][0] == sum(1 for d in hist if d)
        checked += 1
    assert checked > 300


def test_converged_set_is_fixed_point(rng):
    v = np.concatenate([rng.normal(100, 10, 3000), rng.uniform(200, 2000, 40)])
    out = _clip(v, cutoff=3.0, max_iter=50, return_keep=True)
    assert out["converged"][0] == 1
    _, keep = out["keep"][0]
    again = _clip(v[keep], cutoff=3.0, max_iter=1)
    assert again["n_members"][0] == keep.sum() and again["n_iter"][0] == 0


def test_gaussian_with_outliers_converges_fast(rng):
    iters = []
    for _ in range(10):
        v = np.concatenate([rng.normal(100, 10, 5000), rng.uniform(300, 3000, 50)])
        out = _clip(v, cutoff=3.0, max_iter=20)
        iters.append(out["n_iter"][0])
        assert out["mean"][0] == pytest.approx(100.0, abs=4 * 10 / math.sqrt(5000))
        assert out["std"][0] == pytest.approx(10.0 * 0.987, rel=0.04)
    assert max(iters) <= 6 and np.median(iters) <= 4


def test_poisson_and_azimuthal_agree_on_pure_poisson(rng):
    """Fig. fig_std: on a pure Poisson background both models give a similar
    amplitude when many pixels share the bin."""
    lam = 100.0
    v = rng.poisson(lam, 20000).astype(np.float64)
    out_a = _clip(v, max_iter=0)
    out_p = _clip(v, max_iter=0, error_model=S.POISSON)
    assert out_a["std"][0] == pytest.approx(10.0, rel=0.03)
    assert out_p["std"][0] == pytest.approx(10.0, rel=0.03)
