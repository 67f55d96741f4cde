"""MI355X-native elastic ADER-DG element kernels (Python binding).

Thin ctypes binding of the C ABI declared in include/dg.h.  Argument
marshalling only: every stage of the scheme runs in the HIP library
(libdg_mi355x.so, built in-tree by paper_1903_11521_amd/build.py).  PyTorch
provides device memory and the current stream.  There is no CPU fallback: if
the library is missing, every call raises.
"""
from . import perfmodel
from ._lib import (DG_BF16X3, DG_FP32, DG_FP64, DG_MIXED, Batch, DGError, Lts, Plan, element_data, flop_model,
                   visco_element_data, visco_shape, visco_step, visco_tune,
                   library_path,
                   lina_coefficients, lina_step, mra_apply, reference_blob, reference_matrices,
                   set_debug_checks)

__all__ = ["Plan", "Batch", "Lts", "DGError", "DG_FP64", "DG_FP32", "DG_MIXED", "DG_BF16X3", "reference_blob", "reference_matrices",
           "element_data", "library_path", "flop_model", "perfmodel", "set_debug_checks", "mra_apply",
           "lina_coefficients", "lina_step", "visco_element_data", "visco_shape", "visco_step", "visco_tune"]
