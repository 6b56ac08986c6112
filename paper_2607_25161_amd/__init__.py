"""MI355X-native fast Stokesian dynamics for suspensions of rigid bead aggregates.

The compute path is libfsd.so (HIP kernels for gfx950 behind the C ABI of
include/fsd.h).  This package is a thin ctypes binding with the same names:
argument marshalling only.  Importing it on a machine where the library has
not been built raises ImportError; there is no CPU fallback.
"""
from ._capi import (  # noqa: F401
    Batch, FSD_FP64, FSD_MIXED, FsdError, Info, Params, SolveInfo, System, default_params,
    estimate_bytes, fft3d, fft3d_noalloc, lib, library_path, normals, philox4x64, TIMER_NAMES,
)
