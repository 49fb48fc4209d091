"""ctypes binding of libsigsep.so (argument marshalling only).

Every function takes torch tensors for device buffers, passes their data
pointers and the current HIP stream to the C ABI declared in
``include/sigsep.h``, and raises ``SigsepError`` on a nonzero return code.
There is no fallback: if the library is missing the import fails loudly.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "_lib", "libsigsep.so")

SS_OK, SS_EINVAL, SS_ESIZE, SS_EHIP = 0, -1, -2, -3
SS_AZIMUTHAL, SS_POISSON, SS_HYBRID = 0, 1, 2
SS_SPLIT_NONE, SS_SPLIT_BBOX = 0, 1
SS_RC_FRAC_BITS = 20
SS_RC_MASKED = 0xFFFFFFFF
SS_MAX_BINS = 4094
SS_MAX_ITER = 32
SS_MAX_PATCH = 15
SS_N_CLASSES = 8
SS_SURROGATE_MAX_CLASS = 5
SS_MLP_IN, SS_MLP_HID, SS_MLP_OUT = 19, 64, 2
SS_MLP_K1, SS_MLP_OUT_PAD = 32, 16
SS_MLP_OFF_W1, SS_MLP_OFF_B1, SS_MLP_OFF_W2 = 0, 2048, 2112
SS_MLP_OFF_B2, SS_MLP_OFF_W3, SS_MLP_OFF_B3 = 6208, 6272, 7296
SS_MLP_PARAMS = 7312
SS_VETO_BINS = 256
SS_VETO_COUNTERS = 4 + 2 * SS_VETO_BINS
SS_CLASSIFY_SCRATCH_BYTES = 64 << 20

EXPORTED = (
    "ss_strerror", "ss_version", "ss_build_csr", "ss_csr_schedule", "ss_class_rows", "ss_radial_coords",
    "ss_layout_words", "ss_csr_relayout", "ss_layout_scatter",
    "ss_correct", "ss_correct_indexed", "ss_correct_tiled", "ss_correct_indexed_tiled",
    "ss_integrate_csr", "ss_sigma_clip", "ss_classify_workspace", "ss_classify", "ss_classify_noalloc",
    "ss_compress", "ss_peakfind",
    "ss_clip_features", "ss_surrogate_targets", "ss_mlp_forward", "ss_mlp_grad_workspace", "ss_mlp_grad",
    "ss_mlp_adam", "ss_sigma_clip_surrogate", "ss_sigma_clip_warm", "ss_sigma_clip_batches",
    "ss_densify_workspace", "ss_densify", "ss_veto", "ss_pack_results",
)


class SigsepError(RuntimeError):
    def __init__(self, name, code):
        super().__init__(f"{name} failed: {code} ({strerror(code)})")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("max_row", ctypes.c_int32), ("n_pix", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("bin_order", ctypes.c_void_p),
                ("class_count", ctypes.c_int32 * SS_N_CLASSES), ("shape", ctypes.c_int32 * SS_N_CLASSES)]


class ClipBatch(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_void_p), ("norm", ctypes.c_void_p), ("n_frames", ctypes.c_int32),
                ("csr", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("cutoff", ctypes.c_float), ("max_iter", ctypes.c_int32), ("error_model", ctypes.c_int32),
                ("dark_var", ctypes.c_float), ("n_pick", ctypes.c_float), ("noise", ctypes.c_float),
                ("snr", ctypes.c_float), ("patch", ctypes.c_int32), ("min_count", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("std", ctypes.c_void_p), ("sem", ctypes.c_void_p),
                ("sum_w", ctypes.c_void_p), ("n_members", ctypes.c_void_p), ("n_iter", ctypes.c_void_p),
                ("converged", ctypes.c_void_p)]


class Radial(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int32), ("centre0", ctypes.c_double), ("width", ctypes.c_double),
                ("rcoord", ctypes.c_void_p), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32)]


class Layout(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32)]


class Peak(ctypes.Structure):
    _fields_ = [("index", ctypes.c_uint32), ("y", ctypes.c_float), ("x", ctypes.c_float),
                ("intensity", ctypes.c_float), ("sigma", ctypes.c_float)]


class Noise(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("frame0", ctypes.c_int64), ("trunc", ctypes.c_float)]


PEAK_BYTES = ctypes.sizeof(Peak)

_lib = None


def lib():
    """The loaded library (loads it on first use; raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_09515_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        P = ctypes.POINTER
        L.ss_strerror.restype = ctypes.c_char_p
        L.ss_strerror.argtypes = [ctypes.c_int]
        L.ss_version.restype = ctypes.c_int
        L.ss_version.argtypes = []
        L.ss_build_csr.restype = ctypes.c_int
        L.ss_build_csr.argtypes = [i32, i32, f64, f64, f64, f64, i32, i32, vp, vp, vp, vp, vp, i64,
                                   P(i64), P(i32), P(f64)]
        L.ss_csr_schedule.restype = ctypes.c_int
        L.ss_csr_schedule.argtypes = [vp, i32, vp, vp]
        L.ss_class_rows.restype = ctypes.c_int32
        L.ss_class_rows.argtypes = [i32]
        L.ss_radial_coords.restype = ctypes.c_int
        L.ss_radial_coords.argtypes = [i32, i32, f64, f64, f64, f64, i32, f64, vp, vp, P(f64), P(f64)]
        L.ss_layout_words.restype = i64
        L.ss_layout_words.argtypes = [P(Layout)]
        L.ss_csr_relayout.restype = ctypes.c_int
        L.ss_csr_relayout.argtypes = [P(Layout), i32, vp, vp, vp]
        L.ss_layout_scatter.restype = ctypes.c_int
        L.ss_layout_scatter.argtypes = [P(Layout), vp, ctypes.c_float, vp]
        L.ss_correct.restype = ctypes.c_int
        L.ss_correct.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp]
        L.ss_correct_indexed.restype = ctypes.c_int
        L.ss_correct_indexed.argtypes = [vp, i64, vp, i32, i64, vp, vp, vp, vp, vp, vp]
        L.ss_correct_tiled.restype = ctypes.c_int
        L.ss_correct_tiled.argtypes = [vp, i32, P(Layout), vp, vp, vp, vp, vp, vp]
        L.ss_correct_indexed_tiled.restype = ctypes.c_int
        L.ss_correct_indexed_tiled.argtypes = [vp, i64, vp, i32, P(Layout), vp, vp, vp, vp, vp, vp]
        for name in ("ss_integrate_csr", "ss_sigma_clip"):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [vp, vp, vp, i32, P(Csr), P(Params), P(Profile), vp]
        L.ss_classify_workspace.restype = sz
        L.ss_classify_workspace.argtypes = [i32, i64, i32]
        L.ss_classify.restype = ctypes.c_int
        L.ss_classify.argtypes = [vp, vp, i32, i32, i32, P(Radial), P(Profile), P(Params), vp, vp, i64, vp,
                                  vp, i64, vp, vp, sz, vp]
        L.ss_classify_noalloc.restype = ctypes.c_int
        L.ss_classify_noalloc.argtypes = [vp, vp, i32, i32, i32, P(Radial), P(Profile), P(Params), vp, vp, i64,
                                          vp, vp, i64, vp, vp]
        L.ss_compress.restype = ctypes.c_int
        L.ss_compress.argtypes = [vp, vp, i32, i32, i32, P(Radial), P(Profile), P(Params), vp, vp, i64, vp,
                                  vp, sz, vp]
        L.ss_peakfind.restype = ctypes.c_int
        L.ss_peakfind.argtypes = [vp, vp, i32, i32, i32, P(Radial), P(Profile), P(Params), vp, i64, vp,
                                  vp, sz, vp]
        f32 = ctypes.c_float
        L.ss_clip_features.restype = ctypes.c_int
        L.ss_clip_features.argtypes = [vp, vp, vp, i32, P(Csr), vp, vp, vp]
        L.ss_surrogate_targets.restype = ctypes.c_int
        L.ss_surrogate_targets.argtypes = [vp, P(Profile), i64, vp, vp, vp]
        L.ss_mlp_forward.restype = ctypes.c_int
        L.ss_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.ss_mlp_grad_workspace.restype = sz
        L.ss_mlp_grad_workspace.argtypes = [i64]
        L.ss_mlp_grad.restype = ctypes.c_int
        L.ss_mlp_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, sz, vp]
        L.ss_mlp_adam.restype = ctypes.c_int
        L.ss_mlp_adam.argtypes = [vp, vp, vp, vp, i32, f32, f32, f32, f32, vp, vp]
        L.ss_sigma_clip_surrogate.restype = ctypes.c_int
        L.ss_sigma_clip_surrogate.argtypes = [vp, vp, vp, i32, P(Csr), P(Params), vp, f32, P(Profile), vp, vp]
        L.ss_sigma_clip_warm.restype = ctypes.c_int
        L.ss_sigma_clip_warm.argtypes = [vp, vp, vp, i32, P(Csr), P(Params), vp, vp, f32, P(Profile), vp, vp]
        L.ss_sigma_clip_batches.restype = ctypes.c_int
        L.ss_sigma_clip_batches.argtypes = [vp, i32, P(Params), vp]
        L.ss_densify_workspace.restype = sz
        L.ss_densify_workspace.argtypes = [i32, i32]
        L.ss_densify.restype = ctypes.c_int
        L.ss_densify.argtypes = [vp, vp, i64, vp, vp, i32, i64, P(Radial), P(Profile), P(Noise), vp, vp, sz, vp]
        L.ss_veto.restype = ctypes.c_int
        L.ss_veto.argtypes = [vp, vp, i32, i64, vp, vp, vp]
        L.ss_pack_results.restype = ctypes.c_int
        L.ss_pack_results.argtypes = [vp, vp, i64, vp, vp, i64, vp, i32, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().ss_strerror(code).decode()


def check(name: str, code: int) -> None:
    if code != SS_OK:
        raise SigsepError(name, code)
