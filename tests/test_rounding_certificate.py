"""The correction kernel's rounding certificate, replayed on the host.

The kernel divides a = adc - pedestal (exact in float64) by a float32 gain
(and the float32 result by the norm) as q = a * float64(1 / b), and returns
float32(q) when the 29 fraction bits of q below float32 precision lie more
than 8 from the half-way pattern 2^28; otherwise it divides exactly.  The
method's value is float32(float64(a / b)) (the oracle's definition).  Here
the same test runs in NumPy float64 on random quotients and on quotients
placed next to float32 half-way points: wherever it certifies, float32(q)
must equal float32(a / b), and it must refuse rarely on random input."""

import numpy as np


def _certified(q):
    below = q.view(np.uint64).astype(np.uint64) & np.uint64(0x1FFFFFFF)
    return (below.astype(np.int64) - (0x10000000 - 8)).astype(np.uint64) > np.uint64(16)


def _check(a, b):
    b = b.astype(np.float32)
    r = 1.0 / b.astype(np.float64)
    q = a * r
    ok = _certified(q)
    want = (a / b.astype(np.float64)).astype(np.float32)
    got = q.astype(np.float32)
    assert np.array_equal(got[ok].view(np.uint32), want[ok].view(np.uint32))
    return ok


def test_random_quotients_certify_and_agree():
    rng = np.random.default_rng(11)
    n = 2_000_000
    adc = rng.integers(0, 1 << 14, n).astype(np.float64)
    ped = rng.uniform(0.0, 16000.0, n).astype(np.float32).astype(np.float64)
    gain = rng.uniform(0.01, 60.0, n).astype(np.float32)
    ok = _check(adc - ped, gain)
    assert ok.mean() > 1 - 1e-5, ok.mean()
    # the second division: a float32 signal by a float32 norm
    sig = ((adc - ped) / gain.astype(np.float64)).astype(np.float32).astype(np.float64)
    norm = rng.uniform(0.3, 1.7, n).astype(np.float32)
    ok = _check(sig, norm)
    assert ok.mean() > 1 - 1e-5, ok.mean()


def test_quotients_next_to_half_way_points():
    """Targets a float32 half-way point h and numerators a = h * b nudged by
    a few float64 units: the certificate must refuse whatever it cannot
    decide, and agree wherever it decides."""
    rng = np.random.default_rng(12)
    n = 200_000
    m = rng.integers(1 << 23, 1 << 24, n).astype(np.float64)
    e = rng.integers(-10, 10, n).astype(np.float64)
    h = (m + 0.5) * np.exp2(e - 23)                    # half-way between two float32 values
    b = rng.uniform(0.5, 40.0, n).astype(np.float32)
    a = h * b.astype(np.float64)
    a = a + np.spacing(a) * rng.integers(-40, 41, n)
    ok = _check(a, b)
    assert 0 < ok.mean() < 1
