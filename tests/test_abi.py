"""C-ABI library checks that need no GPU: exported symbols, the host-side
geometry builder against the oracle's independent one, and argument errors
detected before any launch."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import geometry as G
from paper_2411_09515_amd import binding as B
from paper_2411_09515_amd import api

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sigsep.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|int32_t|int64_t|size_t|const char \*)\s*(ss_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) == len(B.EXPORTED) and set(names) == set(B.EXPORTED)
    L = B.lib()
    for n in names:
        assert getattr(L, n) is not None
    assert L.ss_version() >= 100
    assert B.strerror(B.SS_OK) == "ok" and B.strerror(B.SS_EINVAL) == "invalid argument"


def _compare_csr(host, ref, norm=None):
    assert host["nnz"] == ref.nnz
    assert np.array_equal(host["indptr"], ref.indptr)
    assert np.array_equal(host["indices"].astype(np.int64), ref.indices)
    want = ref.coef * (1.0 if norm is None else norm.reshape(-1).astype(np.float64)[ref.indices])
    # the float32 weight is the rounding of c * norm to within one half-ulp (the
    # input bound eps_w the parity band of tests/parity.py rests on)
    assert np.all(np.abs(host["weight"].astype(np.float64) - want) <= 2.0 ** -24 * (1 + 2.0 ** -20) * want)
    assert host["max_row"] == int(np.diff(ref.indptr).max())
    assert host["tth_max"] == pytest.approx(ref.tth_max, rel=1e-13)


def test_host_csr_matches_oracle_no_split():
    g = synth.SMALL
    m = synth.stripe_mask(g)
    host = api.build_csr_host(g.height, g.width, g.pixel_m, g.dist_m, g.centre_row, g.centre_col,
                              g.n_bins, "none", m)
    _compare_csr(host, G.csr_for(g, m))


def test_host_csr_matches_oracle_bbox_with_norm():
    g = synth.JUNGFRAU1M
    m = synth.stripe_mask(g)
    norm = synth.normalisation(g)
    host = api.build_csr_host(g.height, g.width, g.pixel_m, g.dist_m, g.centre_row, g.centre_col,
                              g.n_bins, "bbox", m, norm)
    _compare_csr(host, G.csr_for(g, m), norm)


def test_radial_coords_decode_to_oracle_angles():
    g = synth.JUNGFRAU1M
    m = synth.stripe_mask(g).reshape(-1)
    host = api.build_csr_host(g.height, g.width, g.pixel_m, g.dist_m, g.centre_row, g.centre_col,
                              g.n_bins, "bbox", m)
    rc = host["rcoord"]
    assert np.all(rc[m != 0] == B.SS_RC_MASKED)
    ok = m == 0
    t = (rc[ok] >> B.SS_RC_FRAC_BITS).astype(np.int64) - 1
    frac = (rc[ok] & ((1 << B.SS_RC_FRAC_BITS) - 1)) / float(1 << B.SS_RC_FRAC_BITS)
    pos = G.position_for(g)[ok]
    w = host["width"]
    assert host["centre0"] == pytest.approx(w / 2, rel=1e-14)
    inner = (t >= 0) & (t <= g.n_bins - 2)
    decoded = host["centre0"] + (t[inner] + frac[inner]) * w
    assert np.abs(decoded - pos[inner]).max() <= 2.0 ** -B.SS_RC_FRAC_BITS * w * 1.01
    # outside the centre range the interval index is clamped
    assert np.all(pos[t == -1] < host["centre0"] + 1e-12)
    assert np.all(pos[t == g.n_bins - 1] >= host["centre0"] + (g.n_bins - 1) * w - 1e-12)


def test_host_builder_argument_errors():
    L = B.lib()
    nnz, mr, tm = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
    r = L.ss_build_csr(10, 10, 75e-6, 0.1, 5.0, 5.0, 10, 7, None, None, None, None, None, 0,
                       ctypes.byref(nnz), ctypes.byref(mr), ctypes.byref(tm))
    assert r == B.SS_EINVAL
    r = L.ss_build_csr(10, 10, 75e-6, 0.1, 5.0, 5.0, B.SS_MAX_BINS + 1, 0, None, None, None, None, None, 0,
                       ctypes.byref(nnz), ctypes.byref(mr), ctypes.byref(tm))
    assert r == B.SS_ESIZE
    r = L.ss_build_csr(0, 10, 75e-6, 0.1, 5.0, 5.0, 10, 0, None, None, None, None, None, 0,
                       ctypes.byref(nnz), ctypes.byref(mr), ctypes.byref(tm))
    assert r == B.SS_ESIZE
    r = L.ss_build_csr(10, 10, 75e-6, 0.1, 5.0, 5.0, 10, 0, None, None, None, None, None, 0,
                       ctypes.byref(nnz), ctypes.byref(mr), ctypes.byref(tm))
    assert r == B.SS_OK and nnz.value == 100
    ip = np.zeros(11, dtype=np.int64)
    ix = np.zeros(10, dtype=np.int32)
    wt = np.zeros(10, dtype=np.float32)
    r = L.ss_build_csr(10, 10, 75e-6, 0.1, 5.0, 5.0, 10, 0, None, None, ip.ctypes.data, ix.ctypes.data,
                       wt.ctypes.data, 10, ctypes.byref(nnz), ctypes.byref(mr), ctypes.byref(tm))
    assert r == B.SS_ESIZE  # capacity 10 < nnz 100


def test_device_calls_reject_bad_arguments_before_launch():
    """Host-side validation returns before anything reaches the HIP runtime."""
    L = B.lib()
    fake = ctypes.c_void_p(4096)
    assert L.ss_correct(None, 1, 16, fake, fake, None, fake, None, None) == B.SS_EINVAL
    assert L.ss_correct(fake, -1, 16, fake, fake, None, fake, None, None) == B.SS_ESIZE
    assert L.ss_correct(fake, 1, 1 << 31, fake, fake, None, fake, None, None) == B.SS_ESIZE
    assert L.ss_correct(fake, 0, 16, fake, fake, None, fake, None, None) == B.SS_OK
    csr = B.Csr(10, 5, 100, 50, 4096, 4096, 4096, None)
    prof = B.Profile(*([4096] * 7))
    good = B.Params(3.0, 5, 0, 0.0, 3.0, 0.0, 3.0, 3, 3)
    bad_iter = B.Params(3.0, B.SS_MAX_ITER + 1, 0, 0.0, 3.0, 0.0, 3.0, 3, 3)
    bad_model = B.Params(3.0, 5, 7, 0.0, 3.0, 0.0, 3.0, 3, 3)
    ref = ctypes.byref
    assert L.ss_sigma_clip(fake, None, None, 1, ref(csr), ref(bad_iter), ref(prof), None) == B.SS_ESIZE
    assert L.ss_sigma_clip(fake, None, None, 1, ref(csr), ref(bad_model), ref(prof), None) == B.SS_EINVAL
    assert L.ss_sigma_clip(None, None, None, 1, ref(csr), ref(good), ref(prof), None) == B.SS_EINVAL
    assert L.ss_sigma_clip(fake, None, None, 0, ref(csr), ref(good), ref(prof), None) == B.SS_OK
    big = B.Csr(B.SS_MAX_BINS + 1, 5, 100, 50, 4096, 4096, 4096, None)
    assert L.ss_sigma_clip(fake, None, None, 1, ref(big), ref(good), ref(prof), None) == B.SS_ESIZE
    # integrate ignores max_iter
    assert L.ss_integrate_csr(fake, None, None, 0, ref(csr), ref(bad_iter), ref(prof), None) == B.SS_OK

    rad = B.Radial(10, 0.05, 0.1, 4096)
    need = L.ss_classify_workspace(2, 100, 10)
    assert need > 0
    even = B.Params(3.0, 5, 0, 0.0, 3.0, 0.0, 3.0, 4, 3)
    args = (fake, None, 2, 10, 10, ref(rad), ref(prof))
    assert L.ss_classify(*args, ref(even), fake, fake, 8, fake, None, 0, None, fake, need, None) == B.SS_EINVAL
    assert L.ss_classify(*args, ref(good), fake, fake, 8, fake, None, 0, None, fake, need - 1,
                         None) == B.SS_ESIZE
    assert L.ss_classify(*args, ref(good), fake, None, 8, fake, None, 0, None, fake, need,
                         None) == B.SS_EINVAL
    assert L.ss_classify(*args, ref(good), fake, fake, -1, fake, None, 0, None, fake, need,
                         None) == B.SS_ESIZE
    assert L.ss_compress(*args, ref(good), None, fake, 8, fake, fake, need, None) == B.SS_EINVAL
    assert L.ss_peakfind(*args, ref(good), None, 8, fake, fake, need, None) == B.SS_EINVAL


def test_schedule_groups_rows_by_class():
    L = B.lib()
    rng = np.random.default_rng(4)
    n_bins = 300
    lens = rng.integers(0, 30000, n_bins)
    indptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    order = np.zeros(n_bins, dtype=np.int32)
    counts = np.zeros(B.SS_N_CLASSES, dtype=np.int32)
    assert L.ss_csr_schedule(indptr.ctypes.data, n_bins, order.ctypes.data, counts.ctypes.data) == B.SS_OK
    assert sorted(order.tolist()) == list(range(n_bins)) and counts.sum() == n_bins
    limits = [L.ss_class_rows(c) for c in range(B.SS_N_CLASSES - 1)] + [1 << 40]
    assert limits[:6] == [1024, 2048, 4096, 8192, 16384, 24576]
    at = 0
    for c in range(B.SS_N_CLASSES - 1, -1, -1):
        chunk = order[at: at + counts[c]]
        at += counts[c]
        assert np.all(np.diff(chunk) > 0)
        lo = 0 if c == 0 else limits[c - 1]
        assert np.all((lens[chunk] > lo) | (c == 0)) and np.all(lens[chunk] <= limits[c])
    assert L.ss_csr_schedule(indptr.ctypes.data, 0, order.ctypes.data, counts.ctypes.data) == B.SS_ESIZE
    # a schedule whose class sizes do not add up to n_bins is refused before launch
    bad = B.Csr(10, 5, 100, 50, 4096, 4096, 4096, 4096, (ctypes.c_int32 * B.SS_N_CLASSES)(1, 2, 0, 0, 0, 0, 0))
    prof = B.Profile(*([4096] * 7))
    good = B.Params(3.0, 5, 0, 0.0, 3.0, 0.0, 3.0, 3, 3)
    ref = ctypes.byref
    assert L.ss_sigma_clip(ctypes.c_void_p(4096), None, None, 1, ref(bad), ref(good), ref(prof), None) == B.SS_EINVAL


def test_densify_veto_and_pack_reject_bad_arguments_before_launch():
    """Host-side validation of the densification, veto and packing entry
    points (nothing reaches the HIP runtime)."""
    L = B.lib()
    fake = ctypes.c_void_p(4096)
    ref = ctypes.byref
    rad = B.Radial(10, 0.05, 0.1, 4096)
    prof = B.Profile(*([4096] * 7))
    need = L.ss_densify_workspace(2, 10)
    assert need > 0 and L.ss_densify_workspace(-1, 10) == 0
    noise = B.Noise(7, 0, 3.0)
    nan_noise = B.Noise(7, 0, float("nan"))
    assert L.ss_densify(fake, fake, 8, fake, None, 2, 100, None, ref(prof), None, fake, fake, need,
                        None) == B.SS_EINVAL
    assert L.ss_densify(fake, fake, 8, fake, None, -1, 100, ref(rad), ref(prof), None, fake, fake, need,
                        None) == B.SS_ESIZE
    assert L.ss_densify(fake, fake, 8, fake, None, 0, 100, ref(rad), ref(prof), None, fake, fake, need,
                        None) == B.SS_OK
    assert L.ss_densify(fake, fake, 8, fake, None, 2, 100, ref(rad), ref(prof), ref(nan_noise), fake, fake, need,
                        None) == B.SS_EINVAL
    assert L.ss_densify(None, fake, 8, fake, None, 2, 100, ref(rad), ref(prof), ref(noise), fake, fake, need,
                        None) == B.SS_EINVAL
    assert L.ss_densify(fake, fake, 8, fake, None, 2, 100, ref(rad), ref(prof), None, None, fake, need,
                        None) == B.SS_EINVAL
    assert L.ss_densify(fake, fake, 8, fake, None, 2, 100, ref(rad), ref(prof), None, fake, fake, need - 1,
                        None) == B.SS_ESIZE
    big = B.Radial(B.SS_MAX_BINS + 1, 0.05, 0.1, 4096)
    assert L.ss_densify(fake, fake, 8, fake, None, 2, 100, ref(big), ref(prof), None, fake, fake, need,
                        None) == B.SS_ESIZE
    assert L.ss_veto(fake, fake, -1, 20, fake, fake, None) == B.SS_ESIZE
    assert L.ss_veto(fake, fake, 0, 20, fake, fake, None) == B.SS_OK
    assert L.ss_veto(None, fake, 4, 20, fake, fake, None) == B.SS_EINVAL
    assert L.ss_veto(fake, fake, 4, 20, fake, None, None) == B.SS_EINVAL
    assert L.ss_pack_results(fake, fake, 8, fake, fake, 4, fake, -1, fake, fake, fake, fake, None) == B.SS_ESIZE
    assert L.ss_pack_results(fake, fake, 8, fake, fake, 4, fake, 2, None, fake, fake, fake, None) == B.SS_EINVAL
    assert L.ss_pack_results(fake, fake, 8, fake, None, 4, fake, 2, fake, fake, fake, fake, None) == B.SS_EINVAL
    assert L.ss_pack_results(fake, None, 8, fake, None, 4, None, 2, fake, fake, fake, None, None) == B.SS_EINVAL


def test_classify_noalloc_refuses_oversize_before_any_device_call():
    """Sizes beyond the library's array are refused on the host; a call with
    no frames enqueues nothing."""
    L = B.lib()
    g = synth.JUNGFRAU4M
    ref = ctypes.byref
    radial = B.Radial(g.n_bins, 0.025, 0.05, 4096)
    prof = B.Profile(4096, 4096, 4096, 4096, 4096, 4096, 4096)
    p = api.Params().c()
    assert int(L.ss_classify_workspace(16, g.n_pix, g.n_bins)) > B.SS_CLASSIFY_SCRATCH_BYTES
    args = (ctypes.c_void_p(4096), None, 16, g.height, g.width, ref(radial), ref(prof), ref(p),
            ctypes.c_void_p(4096), ctypes.c_void_p(4096), 16, ctypes.c_void_p(4096), None, 0, None, None)
    assert L.ss_classify_noalloc(*args) == B.SS_ESIZE
    big = (ctypes.c_void_p(4096), None, 1, 1 << 15, 1 << 15) + args[5:]
    assert L.ss_classify_noalloc(*big) == B.SS_ESIZE
    none = (ctypes.c_void_p(4096), None, 0) + args[3:]
    assert L.ss_classify_noalloc(*none) == B.SS_OK
    assert L.ss_classify_noalloc(None, None, 1, 4, 4, None, ref(prof), ref(p), None, None, 0, None, None, 0,
                                 None, None) == B.SS_EINVAL


def test_wrappers_refuse_bad_dtypes_and_shapes_before_launch():
    """Every torch-facing wrapper checks dtype and shape against the geometry
    and the frame count and raises ValueError before any launch (a wrongly
    shaped buffer would be read past its end on the device)."""
    import torch
    g = synth.SMALL
    geo = api.Geometry.from_scene(g, synth.stripe_mask(g), None, "cpu")
    N, nb = geo.n_pix, geo.n_bins
    p = api.Params()
    f32 = torch.zeros((2, N), dtype=torch.float32)

    def bad(fn, *a, what, **kw):
        with pytest.raises(ValueError) as e:
            fn(*a, **kw)
        assert what in str(e.value), str(e.value)

    raw = torch.zeros((2, N), dtype=torch.uint16)
    ped = torch.zeros((3, N), dtype=torch.float32)
    bad(api.correct, raw.to(torch.int32), ped, ped, what="raw: dtype")
    bad(api.correct, raw, ped[:2], ped, what="pedestal: shape")
    bad(api.correct, raw, ped, ped.double(), what="gain: dtype")
    bad(api.correct, raw, ped, ped, torch.zeros(N - 1), what="norm: shape")
    bad(api.correct, raw, ped, ped, what="device")           # right types, host memory
    bad(api.sigma_clip, f32.double(), geo, p, what="frames: dtype")
    bad(api.sigma_clip, f32[:, :-1].contiguous(), geo, p, what="frames: shape")
    bad(api.sigma_clip, f32, geo, p, mask=torch.zeros(N, dtype=torch.bool), what="mask: dtype")
    prof = api.new_profile(2, nb, "cpu")
    prof["n_iter"] = prof["n_iter"].long()
    bad(api.sigma_clip, f32, geo, p, out=prof, what="out['n_iter']: dtype")
    prof = api.new_profile(2, nb - 1, "cpu")
    bad(api.classify, f32, geo, prof, p, capacity=8, what="profile['mean']: shape")
    prof = api.new_profile(2, nb, "cpu")
    bad(api.classify, f32, geo, prof, p, capacity=8, workspace=torch.zeros(16, dtype=torch.uint8),
        what="workspace")
    out = dict(kept_index=torch.zeros((2, 4), dtype=torch.int32), kept_value=torch.zeros((2, 4)),
               n_kept=torch.zeros(2, dtype=torch.int64), peaks=torch.zeros((2, 4, B.PEAK_BYTES), dtype=torch.uint8),
               n_peaks=torch.zeros(2, dtype=torch.int64))
    bad(api.classify_noalloc, f32, geo, prof, p, out, 8, 4, what="capacity")
    bad(api.veto, torch.zeros(3, dtype=torch.int32), 2, what="n_peaks: dtype")
    bad(api.veto, torch.zeros(3, dtype=torch.int64), 2, counters=torch.zeros(5, dtype=torch.int64),
        what="counters: shape")
    model_x = torch.zeros((5, B.SS_MLP_IN + 1))
    bad(api.Surrogate.forward, None, model_x, what="x: shape")


def test_tiled_layout_calls_reject_bad_arguments_before_launch():
    """The tiled correction entries and a classification naming a tiled
    layout refuse bad layouts and pointers on the host; the torch wrappers
    check frame shapes against a tiled geometry's frame length."""
    import torch
    L = B.lib()
    fake = ctypes.c_void_p(4096)
    ref = ctypes.byref
    good = B.Layout(37, 52, 8, 4)
    odd_tiles = B.Layout(37, 52, 3, 4)
    assert L.ss_correct_tiled(fake, 1, None, fake, fake, None, fake, None, None) == B.SS_EINVAL
    assert L.ss_correct_tiled(fake, 1, ref(odd_tiles), fake, fake, None, fake, None, None) == B.SS_ESIZE
    assert L.ss_correct_tiled(fake, -1, ref(good), fake, fake, None, fake, None, None) == B.SS_ESIZE
    assert L.ss_correct_tiled(None, 1, ref(good), fake, fake, None, fake, None, None) == B.SS_EINVAL
    assert L.ss_correct_tiled(fake, 1, ref(good), fake, None, None, fake, None, None) == B.SS_EINVAL
    assert L.ss_correct_tiled(fake, 0, ref(good), fake, fake, None, fake, None, None) == B.SS_OK
    assert L.ss_correct_indexed_tiled(fake, 3, None, 2, ref(good), fake, fake, None, fake, None, None) == B.SS_EINVAL
    assert L.ss_correct_indexed_tiled(fake, -1, fake, 2, ref(good), fake, fake, None, fake, None, None) == B.SS_ESIZE
    assert L.ss_correct_indexed_tiled(fake, 3, fake, 2, ref(odd_tiles), fake, fake, None, fake, None, None) == \
        B.SS_ESIZE
    # classification: a radial naming tiles that ss_layout refuses
    prof = B.Profile(*([4096] * 7))
    p = B.Params(3.0, 5, 0, 0.0, 3.0, 0.0, 3.0, 3, 3)
    need = L.ss_classify_workspace(2, 100, 10)
    for tw, th in ((3, 4), (8, 3), (128, 1)):
        rad = B.Radial(10, 0.05, 0.1, 4096, tw, th)
        assert L.ss_classify(fake, None, 2, 10, 10, ref(rad), ref(prof), ref(p), fake, fake, 8, fake, None, 0, None,
                             fake, need, None) == B.SS_ESIZE, (tw, th)

    geo = api.Geometry(37, 53, 75e-6, 0.1, 18.3, 26.1, 17, device="cpu", tile=(8, 4))
    assert geo.frame_words == 7 * 10 * 32 and geo.n_pix == 37 * 53
    N = geo.n_pix
    raw = torch.zeros((2, N), dtype=torch.uint16)
    ped = torch.zeros((3, N), dtype=torch.float32)
    with pytest.raises(ValueError, match="raw: expected"):
        api.correct(raw[:, :-4].contiguous(), ped[:, :-4].contiguous(), ped[:, :-4].contiguous(), geom=geo)
    with pytest.raises(ValueError, match="out: shape"):
        api.correct(raw, ped, ped, out=torch.zeros((2, N), dtype=torch.float32), geom=geo)
    with pytest.raises(ValueError, match="frames: shape"):
        api.sigma_clip(torch.zeros((2, N), dtype=torch.float32), geo, api.Params())   # row-major frames
    with pytest.raises(ValueError, match="tile"):
        api.Geometry(37, 53, 75e-6, 0.1, 18.3, 26.1, 17, device="cpu", tile=(6, 4))
