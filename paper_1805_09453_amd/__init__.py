"""G-prox PDHG for ROF denoising and L1 EMD on MI355X: Python binding of libgprox.

Every call forwards to the HIP library (include/gprox.h) through ctypes; this
module only checks tensor shapes/dtypes/devices and passes device pointers and
the current HIP stream.  There is no CPU fallback: if the library is missing or
no GPU is present, the calls raise.
"""
from .api import (  # noqa: F401
    GPError,
    Context,
    Options,
    WarmStart,
    dct_poisson_noalloc,
    emd_step_rule_singular,
    lib_path,
    ws_downsample,
    ws_upsample,
)
