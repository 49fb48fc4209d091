"""Torch-facing wrappers over the C ABI: device memory and streams come from
PyTorch, every step of the path runs in the library's HIP kernels."""

from __future__ import annotations

import ctypes
import gc
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B

SPLITS = {"none": B.SS_SPLIT_NONE, "bbox": B.SS_SPLIT_BBOX}
MODELS = {"azimuthal": B.SS_AZIMUTHAL, "poisson": B.SS_POISSON, "hybrid": B.SS_HYBRID}

PEAK_DTYPE = np.dtype([("index", np.uint32), ("y", np.float32), ("x", np.float32),
                       ("intensity", np.float32), ("sigma", np.float32)])


def _p(t):
    """Device pointer of a tensor handed to the C ABI (None for None); the
    tensor must be a contiguous device tensor."""
    if t is None:
        return None
    _need_device(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _need_device(*tensors):
    for t in tensors:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("device tensors must be contiguous CUDA/HIP tensors")


def _arg(t, name, dtypes, shape=None, min_numel=None):
    """Check one tensor argument before anything is launched: dtype (one of
    ``dtypes``), shape (a tuple, None for any extent) or a minimum size.  A
    mismatch raises ValueError: a wrongly shaped buffer would otherwise be
    read past its end by a kernel.  (Device and contiguity are checked when
    the pointer is taken, ``_p``.)"""
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a tensor, got {type(t).__name__}")
    dtypes = dtypes if isinstance(dtypes, tuple) else (dtypes,)
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
    if shape is not None:
        if t.dim() != len(shape) or any(e is not None and int(a) != int(e) for a, e in zip(t.shape, shape)):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {min_numel} needed")


def _profile_args(prof, F, nb, name="profile", keys=None):
    for k in keys or ("mean", "std", "sem", "sum_w", "n_members", "n_iter", "converged"):
        if k not in prof or prof[k] is None:
            raise ValueError(f"{name}: missing '{k}'")
        dt = torch.float64 if k in ("mean", "std", "sem", "sum_w") else torch.int32
        _arg(prof[k], f"{name}['{k}']", dt, (F, nb))


def _frames_arg(frames, geom, name="frames"):
    if not isinstance(frames, torch.Tensor) or frames.dim() != 2:
        raise ValueError(f"{name}: expected a [F, n_pix] tensor")
    _arg(frames, name, torch.float32, (None, geom.frame_words))
    return frames.shape[0]


def _outputs_args(out, F, capacity, peak_capacity):
    if out.get("kept_index") is not None or out.get("kept_value") is not None or out.get("n_kept") is not None:
        _arg(out.get("kept_index"), "kept_index", (torch.int32, torch.uint32), (F, None))
        _arg(out.get("kept_value"), "kept_value", torch.float32, (F, None))
        _arg(out.get("n_kept"), "n_kept", torch.int64, (F,))
        for k in ("kept_index", "kept_value"):
            if out.get(k) is None or out[k].shape[1] < max(capacity, 1):
                raise ValueError(f"{k}: needs [F, >= capacity] with capacity {capacity}")
    if out.get("peaks") is not None or out.get("n_peaks") is not None:
        _arg(out.get("peaks"), "peaks", torch.uint8, (F, None, B.PEAK_BYTES))
        _arg(out.get("n_peaks"), "n_peaks", torch.int64, (F,))
        if out.get("peaks") is None or out["peaks"].shape[1] < max(peak_capacity, 1):
            raise ValueError(f"peaks: needs [F, >= peak_capacity, {B.PEAK_BYTES}]")


@dataclass
class Params:
    """Parameters of the path (see ss_params in include/sigsep.h)."""

    cutoff: float = 3.0
    max_iter: int = 5
    error_model: str = "azimuthal"
    dark_var: float = 0.0
    n_pick: float = 3.0
    noise: float = 0.0
    snr: float = 3.0
    patch: int = 3
    min_count: int = 3

    def c(self) -> B.Params:
        return B.Params(self.cutoff, self.max_iter, MODELS[self.error_model], self.dark_var, self.n_pick,
                        self.noise, self.snr, self.patch, self.min_count)


# -- geometry (host builder, device-resident result) -------------------------------

def build_csr_host(height, width, pixel_m, dist_m, centre_row, centre_col, n_bins, split="bbox",
                   mask=None, norm=None):
    """CSR of the radial regrouping built by the library's host code (numpy)."""
    L = B.lib()
    mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    norm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32).reshape(-1)
    nnz, max_row, tmax = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
    args = (height, width, pixel_m, dist_m, centre_row, centre_col, n_bins, SPLITS[split],
            _host_ptr(mask), _host_ptr(norm))
    B.check("ss_build_csr", L.ss_build_csr(*args, None, None, None, 0, ctypes.byref(nnz),
                                           ctypes.byref(max_row), ctypes.byref(tmax)))
    indptr = np.zeros(n_bins + 1, dtype=np.int64)
    indices = np.zeros(max(nnz.value, 1), dtype=np.int32)
    weight = np.zeros(max(nnz.value, 1), dtype=np.float32)
    B.check("ss_build_csr", L.ss_build_csr(*args, _host_ptr(indptr), _host_ptr(indices), _host_ptr(weight),
                                           nnz.value, ctypes.byref(nnz), ctypes.byref(max_row),
                                           ctypes.byref(tmax)))
    order = np.zeros(n_bins, dtype=np.int32)
    counts = np.zeros(B.SS_N_CLASSES, dtype=np.int32)
    B.check("ss_csr_schedule", L.ss_csr_schedule(_host_ptr(indptr), n_bins, _host_ptr(order), _host_ptr(counts)))
    rc = np.zeros(height * width, dtype=np.uint32)
    c0, w = ctypes.c_double(), ctypes.c_double()
    B.check("ss_radial_coords", L.ss_radial_coords(height, width, pixel_m, dist_m, centre_row, centre_col,
                                                   n_bins, tmax.value, _host_ptr(mask), _host_ptr(rc),
                                                   ctypes.byref(c0), ctypes.byref(w)))
    return dict(indptr=indptr, indices=indices[: nnz.value], weight=weight[: nnz.value], nnz=nnz.value,
                max_row=max_row.value, tth_max=tmax.value, rcoord=rc, centre0=c0.value, width=w.value,
                bin_order=order, class_count=counts)


class Geometry:
    """Device-resident detector geometry: CSR with weights c * norm, packed
    radial coordinates, normalisation and static mask.

    ``tile=(tile_w, tile_h)`` selects a tiled layout for the corrected
    frames (see ss_layout): ``correct(..., geom=)`` writes it, the CSR
    indices address it and classification reads it; ``frame_words`` is the
    frame length in that layout (``n_pix`` for row-major frames)."""

    def __init__(self, height, width, pixel_m, dist_m, centre_row, centre_col, n_bins, split="bbox",
                 mask=None, norm=None, device="cuda", tile=None):
        h = build_csr_host(height, width, pixel_m, dist_m, centre_row, centre_col, n_bins, split, mask, norm)
        self.height, self.width, self.n_bins = int(height), int(width), int(n_bins)
        self.n_pix = self.height * self.width
        self.tile = None if tile is None else (int(tile[0]), int(tile[1]))
        self.frame_words = self.n_pix
        clip_norm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32).reshape(-1)
        if self.tile is not None:
            L = B.lib()
            lay = self.layout_c()
            words = L.ss_layout_words(ctypes.byref(lay))
            if words < 0:
                raise ValueError(f"tile {tile}: {B.strerror(int(words))}")
            self.frame_words = int(words)
            h = dict(h, indices=h["indices"].copy(), weight=h["weight"].copy())
            B.check("ss_csr_relayout", L.ss_csr_relayout(ctypes.byref(lay), self.n_bins, _host_ptr(h["indptr"]),
                                                         _host_ptr(h["indices"]), _host_ptr(h["weight"])))
            if clip_norm is not None:
                tiled = np.empty(self.frame_words, dtype=np.float32)
                B.check("ss_layout_scatter", L.ss_layout_scatter(ctypes.byref(lay), _host_ptr(clip_norm), 1.0,
                                                                 _host_ptr(tiled)))
                clip_norm = tiled
        self.nnz, self.max_row, self.tth_max = h["nnz"], h["max_row"], h["tth_max"]
        self.centre0, self.bin_width = h["centre0"], h["width"]
        dev = torch.device(device)
        self.indptr = torch.from_numpy(h["indptr"]).to(dev)
        self.indices = torch.from_numpy(np.ascontiguousarray(h["indices"])).to(dev)
        self.weight = torch.from_numpy(np.ascontiguousarray(h["weight"])).to(dev)
        self.rcoord = torch.from_numpy(h["rcoord"].view(np.int32)).to(dev)
        self.bin_order = torch.from_numpy(h["bin_order"]).to(dev)
        self.class_count = h["class_count"]
        self.shape = [0] * B.SS_N_CLASSES   # work-group shape variant per class (see autotune)
        self.scheduled = True
        self.norm = None if norm is None else torch.from_numpy(
            np.array(norm, dtype=np.float32).reshape(-1)).to(dev)
        # the norm indexed like the frames (the clip's Poisson variance)
        self.clip_norm = self.norm if self.tile is None or clip_norm is None else torch.from_numpy(clip_norm).to(dev)
        self.mask = None if mask is None else torch.from_numpy(
            np.array(mask, dtype=np.uint8).reshape(-1)).to(dev)
        self.host = h

    @classmethod
    def from_scene(cls, geom, mask=None, norm=None, device="cuda", tile=None):
        """Geometry of a ``synth.Geometry`` description."""
        return cls(geom.height, geom.width, geom.pixel_m, geom.dist_m, geom.centre_row, geom.centre_col,
                   geom.n_bins, geom.split, mask, norm, device, tile)

    def layout_c(self) -> B.Layout:
        tw, th = self.tile if self.tile is not None else (0, 0)
        return B.Layout(self.height, self.width, tw, th)

    def csr(self) -> B.Csr:
        """The C struct; with ``scheduled`` the clip launches per row-length class."""
        counts = (ctypes.c_int32 * B.SS_N_CLASSES)(*[int(c) for c in self.class_count])
        shape = (ctypes.c_int32 * B.SS_N_CLASSES)(*[int(c) for c in self.shape])
        return B.Csr(self.n_bins, self.max_row, self.frame_words, self.nnz, self.indptr.data_ptr(),
                     self.indices.data_ptr(), self.weight.data_ptr(),
                     self.bin_order.data_ptr() if self.scheduled else None, counts, shape)

    def radial(self) -> B.Radial:
        tw, th = self.tile if self.tile is not None else (0, 0)
        return B.Radial(self.n_bins, self.centre0, self.bin_width, self.rcoord.data_ptr(), tw, th)

    @property
    def bin_centres(self) -> np.ndarray:
        return self.centre0 + self.bin_width * np.arange(self.n_bins)


# -- correction ------------------------------------------------------------------------

def correct(raw, pedestal, gain, norm=None, out=None, n_invalid=None, geom=None):
    """Raw Jungfrau words [F, N] uint16 -> corrected intensity [F, N] float32,
    or [F, geom.frame_words] in the layout of a tiled ``geom``."""
    if not isinstance(raw, torch.Tensor) or raw.dim() != 2:
        raise ValueError("raw: expected a [F, N] tensor of 16-bit words")
    F, N = raw.shape
    if geom is not None and geom.tile is not None:
        if N != geom.n_pix:
            raise ValueError(f"raw: expected {geom.n_pix} pixels per frame, got {N}")
        return _correct_tiled(raw, None, pedestal, gain, norm, out, n_invalid, geom)
    _arg(raw, "raw", (torch.uint16, torch.int16), (F, N))
    _arg(pedestal, "pedestal", torch.float32, (3, N))
    _arg(gain, "gain", torch.float32, (3, N))
    if pedestal is None or gain is None:
        raise ValueError("pedestal and gain are required")
    _arg(norm, "norm", torch.float32, (N,))
    _arg(out, "out", torch.float32, (F, N))
    _arg(n_invalid, "n_invalid", torch.int64, (F,))
    if out is None:
        out = torch.empty((F, N), dtype=torch.float32, device=raw.device)
    if n_invalid is None:
        n_invalid = torch.empty(F, dtype=torch.int64, device=raw.device)
    B.check("ss_correct", B.lib().ss_correct(_p(raw), F, N, _p(pedestal), _p(gain), _p(norm), _p(out),
                                             _p(n_invalid), _stream()))
    return out, n_invalid


def correct_indexed(ring, frame_index, pedestal, gain, norm=None, out=None, n_invalid=None, geom=None):
    """Correction of ring frames picked by a device index: ring [K, N] of
    16-bit words, frame_index [F] int64 on the device -> out [F, N] float32,
    or [F, geom.frame_words] for a tiled ``geom`` (an index outside the ring
    gives an all-invalid frame)."""
    if not isinstance(ring, torch.Tensor) or ring.dim() != 2:
        raise ValueError("ring: expected a [K, N] tensor of 16-bit words")
    K, N = ring.shape
    if geom is not None and geom.tile is not None:
        if N != geom.n_pix:
            raise ValueError(f"ring: expected {geom.n_pix} pixels per frame, got {N}")
        return _correct_tiled(ring, frame_index, pedestal, gain, norm, out, n_invalid, geom)
    _arg(ring, "ring", (torch.uint16, torch.int16), (K, N))
    _arg(frame_index, "frame_index", torch.int64, (None,))
    F = frame_index.shape[0]
    _arg(pedestal, "pedestal", torch.float32, (3, N))
    _arg(gain, "gain", torch.float32, (3, N))
    if pedestal is None or gain is None:
        raise ValueError("pedestal and gain are required")
    _arg(norm, "norm", torch.float32, (N,))
    if out is None:
        out = torch.empty((F, N), dtype=torch.float32, device=ring.device)
    if n_invalid is None:
        n_invalid = torch.empty(F, dtype=torch.int64, device=ring.device)
    _arg(out, "out", torch.float32, (F, N))
    _arg(n_invalid, "n_invalid", torch.int64, (F,))
    B.check("ss_correct_indexed", B.lib().ss_correct_indexed(_p(ring), K, _p(frame_index), F, N, _p(pedestal),
                                                             _p(gain), _p(norm), _p(out), _p(n_invalid), _stream()))
    return out, n_invalid


def _correct_tiled(raw, frame_index, pedestal, gain, norm, out, n_invalid, geom):
    """ss_correct_tiled / ss_correct_indexed_tiled (raw or ring [K, N])."""
    K, N = raw.shape
    _arg(raw, "raw", (torch.uint16, torch.int16), (K, N))
    if frame_index is not None:
        _arg(frame_index, "frame_index", torch.int64, (None,))
    F = K if frame_index is None else frame_index.shape[0]
    if pedestal is None or gain is None:
        raise ValueError("pedestal and gain are required")
    _arg(pedestal, "pedestal", torch.float32, (3, N))
    _arg(gain, "gain", torch.float32, (3, N))
    _arg(norm, "norm", torch.float32, (N,))
    if out is None:
        out = torch.empty((F, geom.frame_words), dtype=torch.float32, device=raw.device)
    if n_invalid is None:
        n_invalid = torch.empty(F, dtype=torch.int64, device=raw.device)
    _arg(out, "out", torch.float32, (F, geom.frame_words))
    _arg(n_invalid, "n_invalid", torch.int64, (F,))
    lay = geom.layout_c()
    if frame_index is None:
        B.check("ss_correct_tiled", B.lib().ss_correct_tiled(_p(raw), F, ctypes.byref(lay), _p(pedestal), _p(gain),
                                                             _p(norm), _p(out), _p(n_invalid), _stream()))
    else:
        B.check("ss_correct_indexed_tiled", B.lib().ss_correct_indexed_tiled(
            _p(raw), K, _p(frame_index), F, ctypes.byref(lay), _p(pedestal), _p(gain), _p(norm), _p(out),
            _p(n_invalid), _stream()))
    return out, n_invalid


# -- statistics -------------------------------------------------------------------------

def new_profile(n_frames, n_bins, device="cuda"):
    d = dict(device=device)
    return dict(mean=torch.empty((n_frames, n_bins), dtype=torch.float64, **d),
                std=torch.empty((n_frames, n_bins), dtype=torch.float64, **d),
                sem=torch.empty((n_frames, n_bins), dtype=torch.float64, **d),
                sum_w=torch.empty((n_frames, n_bins), dtype=torch.float64, **d),
                n_members=torch.empty((n_frames, n_bins), dtype=torch.int32, **d),
                n_iter=torch.empty((n_frames, n_bins), dtype=torch.int32, **d),
                converged=torch.empty((n_frames, n_bins), dtype=torch.int32, **d))


def profile_c(prof) -> B.Profile:
    return B.Profile(*(_p(prof[k]).value if prof.get(k) is not None else None
                       for k in ("mean", "std", "sem", "sum_w", "n_members", "n_iter", "converged")))


def sigma_clip(frames, geom: Geometry, params: Params, out=None, norm=None, mask=None, integrate_only=False):
    """Per-bin clipped profile of frames [F, geom.frame_words] float32
    (corrected intensity; norm and mask, if given, indexed like the frames)."""
    F = _frames_arg(frames, geom)
    _arg(norm, "norm", torch.float32, (geom.frame_words,))
    _arg(mask, "mask", torch.uint8, (geom.frame_words,))
    if out is None:
        out = new_profile(F, geom.n_bins, frames.device)
    _profile_args(out, F, geom.n_bins, "out")
    if norm is None and params.error_model != "azimuthal":
        norm = geom.clip_norm
    fn = B.lib().ss_integrate_csr if integrate_only else B.lib().ss_sigma_clip
    B.check("ss_sigma_clip", fn(_p(frames), _p(norm), _p(mask), F, ctypes.byref(geom.csr()),
                                ctypes.byref(params.c()), ctypes.byref(profile_c(out)), _stream()))
    return out


def sigma_clip_batches(batches, params: Params, outs=None):
    """Clipped profiles of several batches with their own geometries in one
    launch per row-length class: ``batches`` is a list of (frames [F, N],
    Geometry); returns one profile dict per batch."""
    outs = [new_profile(f.shape[0], g.n_bins, f.device) for f, g in batches] if outs is None else outs
    keep = []   # the ctypes structs must outlive the call
    arr = (B.ClipBatch * len(batches))()
    for i, ((frames, geom), out) in enumerate(zip(batches, outs)):
        F = _frames_arg(frames, geom, f"batches[{i}] frames")
        _profile_args(out, F, geom.n_bins, f"outs[{i}]")
        csr, prof = geom.csr(), profile_c(out)
        keep += [csr, prof]
        norm = geom.clip_norm if params.error_model != "azimuthal" else None
        arr[i] = B.ClipBatch(_p(frames).value, None if norm is None else _p(norm).value, frames.shape[0],
                             ctypes.addressof(csr), ctypes.addressof(prof))
    B.check("ss_sigma_clip_batches", B.lib().ss_sigma_clip_batches(arr, len(batches), ctypes.byref(params.c()),
                                                                   _stream()))
    return outs


def autotune(batches, params: Params, reps=3, geometries=None):
    """Pick, per row-length class, the fastest of the clip's work-group shapes
    on the given batches (list of (frames, Geometry)), timing each variant
    with HIP events on the current stream; the choice is stored in every
    Geometry (``shape``) and returned with the timings (ms)."""
    geoms = geometries or [g for _, g in batches]
    n_var = 3
    timings = {}
    best = [0] * B.SS_N_CLASSES
    stream = torch.cuda.current_stream()
    outs = [new_profile(f.shape[0], g.n_bins, f.device) for f, g in batches]
    for c in range(B.SS_N_CLASSES - 2):       # classes with alternative shapes
        if not any(g.class_count[c] for g in geoms):
            continue
        row = []
        for v in range(n_var):
            for g in geoms:
                g.shape[c] = v
            # time this class alone: the other classes are held at their choice
            sigma_clip_batches(batches, params, outs)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                sigma_clip_batches(batches, params, outs)
            b.record(stream)
            b.synchronize()
            row.append(a.elapsed_time(b) / reps)
        best[c] = int(np.argmin(row))
        timings[c] = row
        for g in geoms:
            g.shape[c] = best[c]
    return best, timings


def integrate(frames, geom: Geometry, params: Params, out=None, norm=None, mask=None):
    return sigma_clip(frames, geom, params, out, norm, mask, integrate_only=True)


# -- learned clip surrogate ---------------------------------------------------------------

def clip_features(frames, geom: Geometry, norm=None):
    """Surrogate inputs [F, nb, 19] (float32) and unclipped (n, mean, std) [F, nb, 3] (float64)."""
    F = _frames_arg(frames, geom)
    _arg(norm, "norm", torch.float32, (geom.frame_words,))
    feats = torch.empty((F, geom.n_bins, B.SS_MLP_IN), dtype=torch.float32, device=frames.device)
    stats0 = torch.empty((F, geom.n_bins, 3), dtype=torch.float64, device=frames.device)
    B.check("ss_clip_features", B.lib().ss_clip_features(_p(frames), _p(norm), None, F, ctypes.byref(geom.csr()),
                                                         _p(feats), _p(stats0), _stream()))
    return feats, stats0


def surrogate_targets(stats0, profile):
    """Training targets [n, 2] and use flags [n] from unclipped stats and a converged clip."""
    _arg(stats0, "stats0", torch.float64, (None, None, 3))
    _profile_args(profile, stats0.shape[0], stats0.shape[1])
    n = stats0.numel() // 3
    target = torch.empty((n, 2), dtype=torch.float32, device=stats0.device)
    use = torch.empty(n, dtype=torch.uint8, device=stats0.device)
    B.check("ss_surrogate_targets", B.lib().ss_surrogate_targets(_p(stats0), ctypes.byref(profile_c(profile)), n,
                                                                 _p(target), _p(use), _stream()))
    return target, use


def init_mlp_params(seed=0):
    """Seeded initial parameters in the library's layout: weights uniform in
    +-1/sqrt(fan_in), biases and padding zero (float32, host)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(B.SS_MLP_PARAMS, dtype=np.float32)
    w1 = p[B.SS_MLP_OFF_W1:B.SS_MLP_OFF_B1].reshape(B.SS_MLP_K1, B.SS_MLP_HID)
    w1[:B.SS_MLP_IN] = rng.uniform(-1, 1, (B.SS_MLP_IN, B.SS_MLP_HID)) / np.sqrt(B.SS_MLP_IN)
    p[B.SS_MLP_OFF_W2:B.SS_MLP_OFF_B2] = (rng.uniform(-1, 1, (B.SS_MLP_HID, B.SS_MLP_HID)) /
                                          np.sqrt(B.SS_MLP_HID)).reshape(-1)
    w3 = p[B.SS_MLP_OFF_W3:B.SS_MLP_OFF_B3].reshape(B.SS_MLP_HID, B.SS_MLP_OUT_PAD)
    w3[:, :B.SS_MLP_OUT] = rng.uniform(-1, 1, (B.SS_MLP_HID, B.SS_MLP_OUT)) / np.sqrt(B.SS_MLP_HID)
    return p


class Surrogate:
    """The network's parameters on the device: float32 master copy with Adam
    moments, and the float16 copy (as int16 bits) the kernels use."""

    def __init__(self, params=None, device="cuda", seed=0):
        p = init_mlp_params(seed) if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if p.size != B.SS_MLP_PARAMS:
            raise ValueError(f"expected {B.SS_MLP_PARAMS} parameters")
        self.params = torch.from_numpy(p.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.w16 = torch.from_numpy(p.astype(np.float16).view(np.int16)).to(device)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step = 0
        self._ws = None

    def half_params(self) -> np.ndarray:
        """The float16 parameters as float64 (host)."""
        return self.w16.cpu().numpy().view(np.float16).astype(np.float64)

    def forward(self, x):
        _arg(x, "x", torch.float32, (None, B.SS_MLP_IN))
        n = x.shape[0]
        y = torch.empty((n, B.SS_MLP_OUT), dtype=torch.float32, device=x.device)
        B.check("ss_mlp_forward", B.lib().ss_mlp_forward(_p(self.w16), _p(x), n, _p(y), _stream()))
        return y

    def gradient(self, x, target, use=None):
        """Loss and gradient (into self.loss / self.grad) on samples x [n, 19]."""
        _arg(x, "x", torch.float32, (None, B.SS_MLP_IN))
        n = x.shape[0]
        _arg(target, "target", torch.float32, (n, B.SS_MLP_OUT))
        _arg(use, "use", torch.uint8, (n,))
        need = int(B.lib().ss_mlp_grad_workspace(n))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=x.device)
        B.check("ss_mlp_grad", B.lib().ss_mlp_grad(_p(self.w16), _p(x), _p(target), _p(use), n, _p(self.grad),
                                                   _p(self.loss), _p(self._ws), self._ws.numel(), _stream()))
        return self.loss, self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        B.check("ss_mlp_adam", B.lib().ss_mlp_adam(_p(self.params), _p(self.m), _p(self.v), _p(self.grad), self.step,
                                                   lr, beta1, beta2, eps, _p(self.w16), _stream()))

    def train(self, x, target, use=None, steps=1000, batch=8192, lr=2e-3, seed=0, log_every=0):
        """Adam on shuffled minibatches of the samples; returns the loss history (host floats,
        one per logged step)."""
        n = x.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        for s in range(steps):
            idx = torch.randint(0, n, (min(batch, n),), generator=g).to(x.device)
            self.gradient(x[idx].contiguous(), target[idx].contiguous(),
                          None if use is None else use[idx].contiguous())
            self.adam(lr=lr)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append(float(self.loss.item()))
        return hist


def sigma_clip_surrogate(frames, geom: Geometry, params: Params, model: Surrogate, out=None, widen=0.1,
                         state=None, norm=None):
    """The clip warm-started by the surrogate; ``state`` [F, nb] int32 receives
    1 (accepted), 0 (no prediction) or -1 (refused, clipped again from scratch)."""
    F = _frames_arg(frames, geom)
    _arg(norm, "norm", torch.float32, (geom.frame_words,))
    _arg(state, "state", torch.int32, (F, geom.n_bins))
    if out is None:
        out = new_profile(F, geom.n_bins, frames.device)
    _profile_args(out, F, geom.n_bins, "out")
    if state is None:
        state = torch.empty((F, geom.n_bins), dtype=torch.int32, device=frames.device)
    B.check("ss_sigma_clip_surrogate",
            B.lib().ss_sigma_clip_surrogate(_p(frames), _p(norm), None, F, ctypes.byref(geom.csr()),
                                            ctypes.byref(params.c()), _p(model.w16), widen,
                                            ctypes.byref(profile_c(out)), _p(state), _stream()))
    return out, state


def sigma_clip_warm(frames, geom: Geometry, params: Params, pred_mean, pred_std, out=None, widen=0.1, state=None):
    """The clip warm-started from given per-bin predictions of the converged
    mean and std (float64 [F, nb], e.g. the previous frame's profile), with
    the surrogate's verification; ``state`` [F, nb] int32 receives 1
    (accepted), 0 (no warm start) or -1 (refused, clipped again)."""
    F = _frames_arg(frames, geom)
    _arg(pred_mean, "pred_mean", torch.float64, (F, geom.n_bins))
    _arg(pred_std, "pred_std", torch.float64, (F, geom.n_bins))
    _arg(state, "state", torch.int32, (F, geom.n_bins))
    if out is None:
        out = new_profile(F, geom.n_bins, frames.device)
    _profile_args(out, F, geom.n_bins, "out")
    if state is None:
        state = torch.empty((F, geom.n_bins), dtype=torch.int32, device=frames.device)
    B.check("ss_sigma_clip_warm",
            B.lib().ss_sigma_clip_warm(_p(frames), None, None, F, ctypes.byref(geom.csr()), ctypes.byref(params.c()),
                                       _p(pred_mean), _p(pred_std), widen, ctypes.byref(profile_c(out)), _p(state),
                                       _stream()))
    return out, state


# -- classification ----------------------------------------------------------------------

def workspace_bytes(n_frames, n_pix, n_bins) -> int:
    return int(B.lib().ss_classify_workspace(n_frames, n_pix, n_bins))


def new_workspace(n_frames, geom: Geometry, device="cuda"):
    return torch.empty(workspace_bytes(n_frames, geom.n_pix, geom.n_bins), dtype=torch.uint8, device=device)


def classify(frames, geom: Geometry, profile, params: Params, capacity=0, peak_capacity=0, keep=True,
             peaks=True, mask=None, workspace=None, out=None):
    """Sparsification and/or peak finding of frames [F, N] against a profile."""
    F = _frames_arg(frames, geom)
    _arg(mask, "mask", torch.uint8, (geom.n_pix,))
    _arg(workspace, "workspace", torch.uint8, min_numel=workspace_bytes(F, geom.n_pix, geom.n_bins))
    _profile_args(profile, F, geom.n_bins, keys=("mean", "std", "n_members"))
    dev = frames.device
    if workspace is None:
        workspace = new_workspace(F, geom, dev)
    if out is None:
        out = {}
        if keep:
            out["kept_index"] = torch.empty((F, max(capacity, 1)), dtype=torch.int32, device=dev)
            out["kept_value"] = torch.empty((F, max(capacity, 1)), dtype=torch.float32, device=dev)
            out["n_kept"] = torch.empty(F, dtype=torch.int64, device=dev)
        if peaks:
            out["peaks"] = torch.empty((F, max(peak_capacity, 1), B.PEAK_BYTES), dtype=torch.uint8, device=dev)
            out["n_peaks"] = torch.empty(F, dtype=torch.int64, device=dev)
    _outputs_args(out, F, capacity if keep else 0, peak_capacity if peaks else 0)
    args = (_p(frames), _p(mask), F, geom.height, geom.width, ctypes.byref(geom.radial()),
            ctypes.byref(profile_c(profile)), ctypes.byref(params.c()))
    B.check("ss_classify", B.lib().ss_classify(
        *args, _p(out.get("kept_index")), _p(out.get("kept_value")), capacity, _p(out.get("n_kept")),
        _p(out.get("peaks")), peak_capacity, _p(out.get("n_peaks")), _p(workspace), workspace.numel(),
        _stream()))
    return out


def classify_noalloc(frames, geom: Geometry, profile, params: Params, out, capacity, peak_capacity, mask=None):
    """``classify`` through ss_classify_noalloc: the library's own device array
    serves as workspace (nothing is allocated); ``out`` holds the caller's
    output tensors (kept_index, kept_value, n_kept, peaks, n_peaks)."""
    F = _frames_arg(frames, geom)
    _arg(mask, "mask", torch.uint8, (geom.n_pix,))
    _profile_args(profile, F, geom.n_bins, keys=("mean", "std", "n_members"))
    _outputs_args(out, F, capacity, peak_capacity)
    args = (_p(frames), _p(mask), F, geom.height, geom.width, ctypes.byref(geom.radial()),
            ctypes.byref(profile_c(profile)), ctypes.byref(params.c()))
    B.check("ss_classify_noalloc", B.lib().ss_classify_noalloc(
        *args, _p(out.get("kept_index")), _p(out.get("kept_value")), capacity, _p(out.get("n_kept")),
        _p(out.get("peaks")), peak_capacity, _p(out.get("n_peaks")), _stream()))
    return out


def compress(frames, geom, profile, params, capacity, mask=None, workspace=None):
    F = _frames_arg(frames, geom)
    _arg(mask, "mask", torch.uint8, (geom.n_pix,))
    _arg(workspace, "workspace", torch.uint8, min_numel=workspace_bytes(F, geom.n_pix, geom.n_bins))
    _profile_args(profile, F, geom.n_bins, keys=("mean", "std", "n_members"))
    dev = frames.device
    if workspace is None:
        workspace = new_workspace(F, geom, dev)
    out = dict(kept_index=torch.empty((F, max(capacity, 1)), dtype=torch.int32, device=dev),
               kept_value=torch.empty((F, max(capacity, 1)), dtype=torch.float32, device=dev),
               n_kept=torch.empty(F, dtype=torch.int64, device=dev))
    B.check("ss_compress", B.lib().ss_compress(
        _p(frames), _p(mask), F, geom.height, geom.width, ctypes.byref(geom.radial()),
        ctypes.byref(profile_c(profile)), ctypes.byref(params.c()), _p(out["kept_index"]),
        _p(out["kept_value"]), capacity, _p(out["n_kept"]), _p(workspace), workspace.numel(), _stream()))
    return out


def peakfind(frames, geom, profile, params, peak_capacity, mask=None, workspace=None):
    F = _frames_arg(frames, geom)
    _arg(mask, "mask", torch.uint8, (geom.n_pix,))
    _arg(workspace, "workspace", torch.uint8, min_numel=workspace_bytes(F, geom.n_pix, geom.n_bins))
    _profile_args(profile, F, geom.n_bins, keys=("mean", "std", "n_members"))
    dev = frames.device
    if workspace is None:
        workspace = new_workspace(F, geom, dev)
    out = dict(peaks=torch.empty((F, max(peak_capacity, 1), B.PEAK_BYTES), dtype=torch.uint8, device=dev),
               n_peaks=torch.empty(F, dtype=torch.int64, device=dev))
    B.check("ss_peakfind", B.lib().ss_peakfind(
        _p(frames), _p(mask), F, geom.height, geom.width, ctypes.byref(geom.radial()),
        ctypes.byref(profile_c(profile)), ctypes.byref(params.c()), _p(out["peaks"]), peak_capacity,
        _p(out["n_peaks"]), _p(workspace), workspace.numel(), _stream()))
    return out


def densify(sparse, geom: Geometry, profile, n_frames=None, noise=None, mask=None, out=None, workspace=None):
    """Dense frames [F, N] float32 from kept pixels and their profile (Sec. 3.2).

    ``sparse``: dict with kept_index [F, cap] int32, kept_value [F, cap]
    float32 and n_kept [F] int64 (the layout ``compress`` returns), or None
    for background only (then give ``n_frames``).  ``profile``: dict with
    mean, std [F, nb] float64 and n_members [F, nb] int32.  ``noise``: None
    (noise free) or dict(seed=int, frame0=int, trunc=float) -- the draw
    convention is that of ``ss_densify``.
    """
    ref = profile["mean"]
    F = int(n_frames if sparse is None else sparse["n_kept"].shape[0])
    dev = ref.device
    _profile_args(profile, F, geom.n_bins, keys=("mean", "std", "n_members"))
    _arg(mask, "mask", torch.uint8, (geom.n_pix,))
    _arg(out, "out", torch.float32, (F, geom.n_pix))
    _arg(workspace, "workspace", torch.uint8, min_numel=int(B.lib().ss_densify_workspace(F, geom.n_bins)))
    if sparse is not None:
        _arg(sparse["kept_index"], "kept_index", (torch.int32, torch.uint32), (F, None))
        _arg(sparse["kept_value"], "kept_value", torch.float32, (F, sparse["kept_index"].shape[1]))
        _arg(sparse["n_kept"], "n_kept", torch.int64, (F,))
    if out is None:
        out = torch.empty((F, geom.n_pix), dtype=torch.float32, device=dev)
    if workspace is None:
        workspace = torch.empty(int(B.lib().ss_densify_workspace(F, geom.n_bins)), dtype=torch.uint8, device=dev)
    cap = 0 if sparse is None else sparse["kept_index"].shape[1]
    nz = None
    if noise is not None:
        nz = B.Noise(int(noise.get("seed", 0)) & ((1 << 64) - 1), int(noise.get("frame0", 0)),
                     float(noise.get("trunc", float("inf"))))
    B.check("ss_densify", B.lib().ss_densify(
        _p(None if sparse is None else sparse["kept_index"]), _p(None if sparse is None else sparse["kept_value"]),
        cap, _p(None if sparse is None else sparse["n_kept"]), _p(mask), F, geom.n_pix,
        ctypes.byref(geom.radial()), ctypes.byref(profile_c(profile)),
        None if nz is None else ctypes.byref(nz), _p(out), _p(workspace), workspace.numel(), _stream()))
    return out


def new_veto_counters(device="cuda"):
    """Zeroed counters for ``veto`` (they accumulate over calls)."""
    return torch.zeros(B.SS_VETO_COUNTERS, dtype=torch.int64, device=device)


def veto(n_peaks, threshold, n_kept=None, counters=None, hit=None):
    """Peak-count veto (Sec. 4): hit [F] uint8 and the accumulated counters."""
    _arg(n_peaks, "n_peaks", torch.int64, (None,))
    F = n_peaks.numel()
    _arg(n_kept, "n_kept", torch.int64, (F,))
    _arg(counters, "counters", torch.int64, (B.SS_VETO_COUNTERS,))
    _arg(hit, "hit", torch.uint8, (F,))
    if counters is None:
        counters = new_veto_counters(n_peaks.device)
    if hit is None:
        hit = torch.empty(F, dtype=torch.uint8, device=n_peaks.device)
    B.check("ss_veto", B.lib().ss_veto(_p(n_peaks), _p(n_kept), F, int(threshold), _p(hit), _p(counters),
                                       _stream()))
    return hit, counters


def veto_summary(counters):
    """Host view of the veto counters."""
    c = counters.cpu().numpy()
    nb = B.SS_VETO_BINS
    return dict(hits=int(c[0]), misses=int(c[1]), kept_hits=int(c[2]), kept_misses=int(c[3]),
                hist_frames=c[4:4 + nb].copy(), hist_kept=c[4 + nb:4 + 2 * nb].copy())


def pack_results(out, capacity, peak_capacity, packed=None):
    """Kept entries and peaks of the frames of ``out`` (the dict ``classify``
    fills) packed back to back on the device; returns the dict of packed
    buffers with ``offsets`` [2 (F + 1)] (kept, then peaks)."""
    F = out["n_kept"].shape[0] if "n_kept" in out else out["n_peaks"].shape[0]
    dev = (out.get("n_kept") if out.get("n_kept") is not None else out["n_peaks"]).device
    if packed is None:
        packed = dict(offsets=torch.empty(2 * (F + 1), dtype=torch.int64, device=dev),
                      index=torch.empty(max(F * capacity, 1), dtype=torch.int32, device=dev),
                      value=torch.empty(max(F * capacity, 1), dtype=torch.float32, device=dev),
                      peaks=torch.empty((max(F * peak_capacity, 1), B.PEAK_BYTES), dtype=torch.uint8, device=dev))
    keep = out.get("n_kept") is not None
    pk = out.get("n_peaks") is not None
    _outputs_args(out, F, capacity if keep else 0, peak_capacity if pk else 0)
    _arg(packed["offsets"], "offsets", torch.int64, min_numel=2 * (F + 1))
    if keep:
        _arg(packed["index"], "packed index", (torch.int32, torch.uint32), min_numel=F * capacity)
        _arg(packed["value"], "packed value", torch.float32, min_numel=F * capacity)
    if pk:
        _arg(packed["peaks"], "packed peaks", torch.uint8, min_numel=F * peak_capacity * B.PEAK_BYTES)
    B.check("ss_pack_results", B.lib().ss_pack_results(
        _p(out.get("kept_index")) if keep else None, _p(out.get("kept_value")) if keep else None, capacity,
        _p(out.get("n_kept")) if keep else None, _p(out.get("peaks")) if pk else None, peak_capacity,
        _p(out.get("n_peaks")) if pk else None, F, _p(packed["offsets"]),
        _p(packed["index"]) if keep else None, _p(packed["value"]) if keep else None,
        _p(packed["peaks"]) if pk else None, _stream()))
    return packed


def peaks_to_numpy(peaks_u8, n):
    """Host copy of the first n peak records of one frame as a structured array."""
    raw = peaks_u8[: max(int(n), 0)].cpu().numpy()
    return raw.reshape(-1).view(PEAK_DTYPE).copy() if raw.size else np.zeros(0, dtype=PEAK_DTYPE)


# -- graph lifetimes -------------------------------------------------------------------------

# A captured graph must not be destroyed while another capture is open on the
# device: the destruction is an operation the capture forbids, and the
# runtime aborts.  Captures therefore run inside ``capturing()``, which
# pauses cyclic garbage collection (a collected object could own a graph)
# and defers every graph released through ``release_graphs`` until no
# capture is open.  Objects that capture (Pipeline, serve.Server) own their
# graphs until ``close()``.
_open_captures = 0
_deferred_graphs = []


class capturing:
    """Context of one graph capture (re-entrant)."""

    def __enter__(self):
        global _open_captures
        if _open_captures == 0:
            gc.collect()
            self._gc = gc.isenabled()
            gc.disable()
        _open_captures += 1
        return self

    def __exit__(self, *exc):
        global _open_captures
        _open_captures -= 1
        if _open_captures == 0:
            if getattr(self, "_gc", False):
                gc.enable()
            _deferred_graphs.clear()   # no capture open: the deferred graphs may go now
        return False


def release_graphs(graphs):
    """Drop references to captured graphs (a list or dict of them, emptied);
    while a capture is open they are kept until it closes."""
    items = list(graphs.values()) if isinstance(graphs, dict) else list(graphs)
    graphs.clear()
    if _open_captures:
        _deferred_graphs.extend(items)


# -- the whole path ------------------------------------------------------------------------

class Pipeline:
    """correct -> sigma_clip -> classify for batches of raw frames, with every
    buffer allocated once up front and every step enqueued on the current
    stream."""

    def __init__(self, geom: Geometry, params: Params, n_frames, pedestal=None, gain=None,
                 kept_capacity=1 << 16, peak_capacity=1024, device="cuda"):
        self.geom, self.params, self.n_frames = geom, params, n_frames
        self.pedestal, self.gain = pedestal, gain
        self.kept_capacity, self.peak_capacity = kept_capacity, peak_capacity
        self.frames = torch.empty((n_frames, geom.frame_words), dtype=torch.float32, device=device)
        self.n_invalid = torch.empty(n_frames, dtype=torch.int64, device=device)
        self.profile = new_profile(n_frames, geom.n_bins, device)
        self.workspace = new_workspace(n_frames, geom, device)
        self.out = dict(kept_index=torch.empty((n_frames, kept_capacity), dtype=torch.int32, device=device),
                        kept_value=torch.empty((n_frames, kept_capacity), dtype=torch.float32, device=device),
                        n_kept=torch.empty(n_frames, dtype=torch.int64, device=device),
                        peaks=torch.empty((n_frames, peak_capacity, B.PEAK_BYTES), dtype=torch.uint8,
                                          device=device),
                        n_peaks=torch.empty(n_frames, dtype=torch.int64, device=device))

    def correct(self, raw):
        return correct(raw, self.pedestal, self.gain, self.geom.norm, self.frames, self.n_invalid, geom=self.geom)

    def separate(self, frames=None):
        frames = self.frames if frames is None else frames
        return sigma_clip(frames, self.geom, self.params, self.profile)

    def classify(self, frames=None):
        frames = self.frames if frames is None else frames
        return classify(frames, self.geom, self.profile, self.params, self.kept_capacity, self.peak_capacity,
                        workspace=self.workspace, out=self.out)

    def run(self, raw=None, frames=None):
        """One pass of the path over the batch; returns the output tensors."""
        if raw is not None:
            self.correct(raw)
            frames = self.frames
        self.separate(frames)
        self.classify(frames)
        return self.out

    def capture(self, raw):
        """Capture one pass over the raw frames in ``raw`` (a fixed device
        buffer the caller refills) as a HIP graph; ``replay`` then runs the
        whole path with one launch.  The graph holds no memory sets and is
        owned by the pipeline until ``close()`` (or the next capture)."""
        with capturing():
            self.close()
            side = torch.cuda.Stream(device=raw.device)
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                self.run(raw)                   # eager first: nothing initialised inside the capture
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize(raw.device)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                self.run(raw)
            self._graphs = [g]
        return g

    @property
    def graph(self):
        return self._graphs[0] if getattr(self, "_graphs", None) else None

    def replay(self):
        """The captured pass, on the current stream; returns the output tensors."""
        self.graph.replay()
        return self.out

    def close(self):
        """Release the captured graph (deferred while a capture is open)."""
        if getattr(self, "_graphs", None):
            torch.cuda.synchronize()
            release_graphs(self._graphs)
