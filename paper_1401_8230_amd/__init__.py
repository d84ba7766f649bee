"""libprngd for MI355X: PRNGD extended-precision uniforms (Demchik & Gulov,
arXiv:1401.8230) filled into FP64 device buffers by hand-written HIP
kernels.  See ``prngd`` for the binding and ``include/prngd.h`` for the
C ABI."""
from . import prngd  # noqa: F401
from .prngd import (ENUMERATE, MRG32K3A, PHILOX4X32_10, PHILOX_X1_MRG32K3A_X2,  # noqa: F401
                    Generator, Plan, PrngdError, describe, fill_batch, get_tuning,
                    natural_range, reset_tuning, set_tuning)
