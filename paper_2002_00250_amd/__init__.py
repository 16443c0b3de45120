"""fgs: RGB-D foreground segmentation (GMM and PBAS background models) on MI355X.

The compute path is libfgs.so (hand-written HIP kernels for gfx950, C ABI in
include/fgs.h); ``paper_2002_00250_amd.fgs`` is its ctypes binding.
"""
from . import fgs  # noqa: F401
from .fgs import FGS_GMM, FGS_PBAS, FgsError, Model  # noqa: F401
