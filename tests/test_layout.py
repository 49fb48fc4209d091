"""Tiled frame layouts on the host (no GPU): ss_layout_words, ss_csr_relayout
and ss_layout_scatter against the word formula that include/sigsep.h states
for ss_layout, restated here, on an odd-sized masked geometry."""

import ctypes

import numpy as np
import pytest

from paper_2411_09515_amd import api
from paper_2411_09515_amd import binding as B


def _word(y, x, width, tw, th):
    """Word of pixel (y, x): tiles of tw x th, tiles row-major, pixels row-major inside a tile."""
    tiles_x = -(-width // tw)
    return ((y // th) * tiles_x + x // tw) * (tw * th) + (y % th) * tw + x % tw


def _layout(h, w, tw, th):
    return B.Layout(h, w, tw, th)


def test_layout_words_and_refusals():
    L = B.lib()
    assert L.ss_layout_words(ctypes.byref(_layout(2162, 2068, 0, 0))) == 2162 * 2068
    assert L.ss_layout_words(ctypes.byref(_layout(2162, 2068, 8, 4))) == 259 * 541 * 32
    assert L.ss_layout_words(ctypes.byref(_layout(37, 53, 4, 8))) == 14 * 5 * 32
    for tw, th in ((3, 4), (8, 3), (2, 4), (128, 1), (8, 128), (0, 4), (8, 0), (-8, 4)):
        assert L.ss_layout_words(ctypes.byref(_layout(64, 64, tw, th))) == B.SS_ESIZE, (tw, th)
    assert L.ss_layout_words(ctypes.byref(_layout(0, 64, 8, 4))) == B.SS_ESIZE
    assert L.ss_layout_words(ctypes.byref(_layout(1 << 16, 1 << 15, 8, 4))) == B.SS_ESIZE
    assert L.ss_layout_words(None) == B.SS_EINVAL


@pytest.mark.parametrize("tile", [(8, 4), (4, 8), (16, 2), (64, 1), (4, 1)])
def test_csr_relayout_maps_and_sorts_every_row(tile):
    h, w, nb = 37, 53, 17
    rng = np.random.default_rng(3)
    mask = (rng.random((h, w)) < 0.08).astype(np.uint8)
    norm = (0.5 + rng.random((h, w))).astype(np.float32)
    host = api.build_csr_host(h, w, 75e-6, 0.1, 10.3, 40.7, nb, "bbox", mask, norm)
    ip, ind0, wt0 = host["indptr"], host["indices"].copy(), host["weight"].copy()
    ind, wt = ind0.copy(), wt0.copy()
    lay = _layout(h, w, *tile)
    assert B.lib().ss_csr_relayout(ctypes.byref(lay), nb, api._host_ptr(ip), api._host_ptr(ind),
                                   api._host_ptr(wt)) == B.SS_OK
    words = B.lib().ss_layout_words(ctypes.byref(lay))
    # every pixel has its own word inside the frame
    yy, xx = np.divmod(np.arange(h * w), w)
    all_words = _word(yy, xx, w, *tile)
    assert len(np.unique(all_words)) == h * w and all_words.max() < words
    for r in range(nb):
        a, b = ip[r], ip[r + 1]
        want = sorted(zip(all_words[ind0[a:b]].tolist(), wt0[a:b].tolist()))
        got = list(zip(ind[a:b].tolist(), wt[a:b].tolist()))
        assert np.all(np.diff(ind[a:b]) > 0), r          # ascending word offsets
        assert got == want, r                            # the same (pixel, weight) entries, moved together


def test_csr_relayout_refuses_without_touching_the_arrays():
    ip = np.array([0, 2, 3], dtype=np.int64)
    ind = np.array([0, 5, 99], dtype=np.int32)          # 99 is outside a 6 x 7 image
    wt = np.ones(3, dtype=np.float32)
    keep = ind.copy()
    lay = _layout(6, 7, 4, 2)
    L = B.lib()
    assert L.ss_csr_relayout(ctypes.byref(lay), 2, api._host_ptr(ip), api._host_ptr(ind), api._host_ptr(wt)) == \
        B.SS_EINVAL
    assert np.array_equal(ind, keep)
    bad = np.array([0, 2, 1], dtype=np.int64)            # a row that does not ascend
    assert L.ss_csr_relayout(ctypes.byref(lay), 2, api._host_ptr(bad), api._host_ptr(ind), api._host_ptr(wt)) == \
        B.SS_EINVAL
    assert L.ss_csr_relayout(ctypes.byref(_layout(6, 7, 3, 2)), 2, api._host_ptr(ip), api._host_ptr(ind),
                             api._host_ptr(wt)) == B.SS_ESIZE


def test_layout_scatter_puts_every_pixel_at_its_word():
    h, w, tile = 21, 30, (8, 4)
    src = np.arange(h * w, dtype=np.float32) + 0.5
    lay = _layout(h, w, *tile)
    words = B.lib().ss_layout_words(ctypes.byref(lay))
    dst = np.zeros(words, dtype=np.float32)
    assert B.lib().ss_layout_scatter(ctypes.byref(lay), api._host_ptr(src), np.float32(-7.0),
                                     api._host_ptr(dst)) == B.SS_OK
    yy, xx = np.divmod(np.arange(h * w), w)
    assert np.array_equal(dst[_word(yy, xx, w, *tile)], src)
    assert np.count_nonzero(dst == -7.0) == words - h * w
