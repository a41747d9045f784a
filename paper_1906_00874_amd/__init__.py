"""MI355X (gfx950) hierarchical-matrix LU: Python binding of the C-ABI.

The binding only marshals arguments: planning, assembly upload,
factorisation, solves and matvecs all run inside libhlu.so (HIP kernels for
every step on the device).  PyTorch provides the device buffer and the
stream.  If the shared library is missing the import fails loudly; there is
no fallback.
"""
from .binding import (HLU, Batch, HLUError, Params, Info, PlanStats, lib, build_lib_path,
                      getrf_batched, truncate_add, KERNEL_WEIGHTED, KERNEL_POINT,
                      KERNEL_LOG1D, KERNEL_LOG2D, OP_LU, OP_PRODUCT, OP_INVERSE,
                      PREC_FP64, PREC_MIXED)

__all__ = ["HLU", "Batch", "HLUError", "Params", "Info", "PlanStats", "lib", "build_lib_path",
           "getrf_batched", "truncate_add", "KERNEL_WEIGHTED", "KERNEL_POINT",
           "KERNEL_LOG1D", "KERNEL_LOG2D", "OP_LU", "OP_PRODUCT", "OP_INVERSE",
           "PREC_FP64", "PREC_MIXED"]
