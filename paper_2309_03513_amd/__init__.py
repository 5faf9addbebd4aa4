"""MI355X (gfx950) Liouville-apply library for Gamma-point Tamm-Dancoff hybrid TDDFT.

The compute path is the HIP library ``libwtd.so`` (C ABI in include/wtd.h);
``wtd`` is its ctypes binding and ``autograd`` wraps the apply for PyTorch.
"""
from .wtd import (  # noqa: F401
    FP32, FP64, TERM_ALL, TERM_D, TERM_K1D, TERM_K1E, Liouville, WtdError, load_library,
    LIB_PATH, EXPORTS,
)
