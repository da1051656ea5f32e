"""Matrix-free stochastic reconfiguration on MI355X (gfx950).

The compute path is libsr.so (hand-written HIP kernels behind a C ABI, include/sr.h);
`sr` is its thin ctypes binding.
"""
from . import sr  # noqa: F401
from .sr import (  # noqa: F401
    Matrix, SrError, as_matrix, lm_hv_product, sr_cg_solve, sr_grad, sr_quantize, sr_sv_product,
)

__version__ = "0.1.0"
