"""MI355X (gfx950) per-frame signal separation: Jungfrau correction, CSR
azimuthal regrouping, iterative sigma-clipping, sparsification and peak
finding as hand-written HIP kernels behind the C ABI of include/sigsep.h.

The compiled library is required: importing the package works without it,
but every call raises ImportError until ``python -m
paper_2411_09515_amd.build`` has produced ``_lib/libsigsep.so``.
"""

from .binding import SigsepError, lib  # noqa: F401
from .api import (  # noqa: F401
    Params,
    Geometry,
    Pipeline,
    build_csr_host,
    correct,
    sigma_clip,
    integrate,
    classify,
    compress,
    peakfind,
    new_profile,
    new_workspace,
    peaks_to_numpy,
    PEAK_DTYPE,
)
