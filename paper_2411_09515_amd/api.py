"""Torch-facing wrappers over the C ABI: device memory and streams come from
PyTorch, every step of the path runs in the library's HIP kernels."""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B

SPLITS = {"none": B.SS_SPLIT_NONE, "bbox": B.SS_SPLIT_BBOX}
MODELS = {"azimuthal": B.SS_AZIMUTHAL, "poisson": B.SS_POISSON, "hybrid": B.SS_HYBRID}

PEAK_DTYPE = np.dtype([("index", np.uint32), ("y", np.float32), ("x", np.float32),
                       ("intensity", np.float32), ("sigma", np.float32)])


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _need_device(*tensors):
    for t in tensors:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("device tensors must be contiguous CUDA/HIP tensors")


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
    radial coordinates, normalisation and static mask."""

    def __init__(self, height, width, pixel_m, dist_m, centre_row, centre_col, n_bins, split="bbox",
                 mask=None, norm=None, device="cuda"):
        h = build_csr_host(height, width, pixel_m, dist_m, centre_row, centre_col, n_bins, split, mask, norm)
        self.height, self.width, self.n_bins = int(height), int(width), int(n_bins)
        self.n_pix = self.height * self.width
        self.nnz, self.max_row, self.tth_max = h["nnz"], h["max_row"], h["tth_max"]
        self.centre0, self.bin_width = h["centre0"], h["width"]
        dev = torch.device(device)
        self.indptr = torch.from_numpy(h["indptr"]).to(dev)
        self.indices = torch.from_numpy(np.ascontiguousarray(h["indices"])).to(dev)
        self.weight = torch.from_numpy(np.ascontiguousarray(h["weight"])).to(dev)
        self.rcoord = torch.from_numpy(h["rcoord"].view(np.int32)).to(dev)
        self.bin_order = torch.from_numpy(h["bin_order"]).to(dev)
        self.class_count = h["class_count"]
        self.scheduled = True
        self.norm = None if norm is None else torch.from_numpy(
            np.array(norm, dtype=np.float32).reshape(-1)).to(dev)
        self.mask = None if mask is None else torch.from_numpy(
            np.array(mask, dtype=np.uint8).reshape(-1)).to(dev)
        self.host = h

    @classmethod
    def from_scene(cls, geom, mask=None, norm=None, device="cuda"):
        """Geometry of a ``synth.Geometry`` description."""
        return cls(geom.height, geom.width, geom.pixel_m, geom.dist_m, geom.centre_row, geom.centre_col,
                   geom.n_bins, geom.split, mask, norm, device)

    def csr(self) -> B.Csr:
        """The C struct; with ``scheduled`` the clip launches per row-length class."""
        counts = (ctypes.c_int32 * B.SS_N_CLASSES)(*[int(c) for c in self.class_count])
        return B.Csr(self.n_bins, self.max_row, self.n_pix, self.nnz, self.indptr.data_ptr(),
                     self.indices.data_ptr(), self.weight.data_ptr(),
                     self.bin_order.data_ptr() if self.scheduled else None, counts)

    def radial(self) -> B.Radial:
        return B.Radial(self.n_bins, self.centre0, self.bin_width, self.rcoord.data_ptr())

    @property
    def bin_centres(self) -> np.ndarray:
        return self.centre0 + self.bin_width * np.arange(self.n_bins)


# -- correction ------------------------------------------------------------------------

def correct(raw, pedestal, gain, norm=None, out=None, n_invalid=None):
    """Raw Jungfrau words [F, N] uint16 -> corrected intensity [F, N] float32."""
    _need_device(raw, pedestal, gain, norm, out, n_invalid)
    F, N = raw.shape
    if out is None:
        out = torch.empty((F, N), dtype=torch.float32, device=raw.device)
    if n_invalid is None:
        n_invalid = torch.empty(F, dtype=torch.int64, device=raw.device)
    B.check("ss_correct", B.lib().ss_correct(_p(raw), F, N, _p(pedestal), _p(gain), _p(norm), _p(out),
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
    return B.Profile(*(prof[k].data_ptr() for k in ("mean", "std", "sem", "sum_w", "n_members", "n_iter",
                                                    "converged")))


def sigma_clip(frames, geom: Geometry, params: Params, out=None, norm=None, mask=None, integrate_only=False):
    """Per-bin clipped profile of frames [F, N] float32 (corrected intensity)."""
    _need_device(frames, norm, mask)
    F = frames.shape[0]
    if out is None:
        out = new_profile(F, geom.n_bins, frames.device)
    if norm is None and params.error_model != "azimuthal":
        norm = geom.norm
    fn = B.lib().ss_integrate if integrate_only else B.lib().ss_sigma_clip
    B.check("ss_sigma_clip", fn(_p(frames), _p(norm), _p(mask), F, ctypes.byref(geom.csr()),
                                ctypes.byref(params.c()), ctypes.byref(profile_c(out)), _stream()))
    return out


def integrate(frames, geom: Geometry, params: Params, out=None, norm=None, mask=None):
    return sigma_clip(frames, geom, params, out, norm, mask, integrate_only=True)


# -- classification ----------------------------------------------------------------------

def workspace_bytes(n_frames, n_pix, n_bins) -> int:
    return int(B.lib().ss_classify_workspace(n_frames, n_pix, n_bins))


def new_workspace(n_frames, geom: Geometry, device="cuda"):
    return torch.empty(workspace_bytes(n_frames, geom.n_pix, geom.n_bins), dtype=torch.uint8, device=device)


def classify(frames, geom: Geometry, profile, params: Params, capacity=0, peak_capacity=0, keep=True,
             peaks=True, mask=None, workspace=None, out=None):
    """Sparsification and/or peak finding of frames [F, N] against a profile."""
    _need_device(frames, mask, workspace)
    F = frames.shape[0]
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
    args = (_p(frames), _p(mask), F, geom.height, geom.width, ctypes.byref(geom.radial()),
            ctypes.byref(profile_c(profile)), ctypes.byref(params.c()))
    B.check("ss_classify", B.lib().ss_classify(
        *args, _p(out.get("kept_index")), _p(out.get("kept_value")), capacity, _p(out.get("n_kept")),
        _p(out.get("peaks")), peak_capacity, _p(out.get("n_peaks")), _p(workspace), workspace.numel(),
        _stream()))
    return out


def compress(frames, geom, profile, params, capacity, mask=None, workspace=None):
    _need_device(frames, mask, workspace)
    F = frames.shape[0]
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
    _need_device(frames, mask, workspace)
    F = frames.shape[0]
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


def peaks_to_numpy(peaks_u8, n):
    """Host copy of the first n peak records of one frame as a structured array."""
    raw = peaks_u8[: max(int(n), 0)].cpu().numpy()
    return raw.reshape(-1).view(PEAK_DTYPE).copy() if raw.size else np.zeros(0, dtype=PEAK_DTYPE)


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
        self.frames = torch.empty((n_frames, geom.n_pix), dtype=torch.float32, device=device)
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
        return correct(raw, self.pedestal, self.gain, self.geom.norm, self.frames, self.n_invalid)

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
