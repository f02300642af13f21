"""MI355X-native matrix-free global stability analysis of compressible flows.

The computation lives in libsa.so (HIP kernels for gfx950, C ABI declared in
include/sa.h); this package is its thin Python binding.  Build the library
with ``python -m paper_1502_03701_amd.build``.
"""
from ._native import (SA_F32, SA_F64, SA_MIXED, SA_OK, SA_NOT_CONVERGED, SA_PC_BLOCK_JACOBI, SA_PC_MEAN_FLOW,
                      Context, SAError, arnoldi_eigs, load)

__all__ = ["Context", "SAError", "arnoldi_eigs", "load", "SA_F64", "SA_F32", "SA_MIXED",
           "SA_OK", "SA_NOT_CONVERGED", "SA_PC_BLOCK_JACOBI", "SA_PC_MEAN_FLOW"]
