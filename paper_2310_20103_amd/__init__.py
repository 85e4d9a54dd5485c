"""MI355X (gfx950) implementation of the Lanczos full-frequency GW correlation
self-energy (Gao, Tang, Zhao, Chelikowsky).

The computation lives in the HIP library ``_lib/libgwl.so`` behind the C ABI
of ``include/gwl.h``; this package is its Python binding.
"""
from .binding import (Context, GwlError, lib, qp_solve, save_coefficients, load_coefficients, FP64, MIXED_F16, REORTH, PRECISIONS,  # noqa: F401
                      KEY_PRECISION, KEY_REORTH, KEY_BLOCK, KEY_POLY_LO, KEY_POLY_HI,
                      KEY_POLY_DEGREE, KEY_N_VC, KEY_LAST_MS_TOTAL, KEY_LAST_C_MATVECS,
                      KEY_GEMM_SPLITK, KEY_KERNELS, KEY_PROFILE, KEY_PROF, KEY_GRAPHS, KEY_TUNED_BLOCK,
                      KEY_TUNED_SPLITK, KEY_BF16_TILE, KEY_TDA, KEY_QUADRATURE, KEY_ISDF, KEY_ISDF_NMU,
                      KEY_TUNED_TILE, KEY_ADJOINT_STORE, KEY_ADJOINT_STORED, KEY_HI_RESIDUAL, KEY_SCHEDULER,
                      LIB_PATH)

__all__ = ["Context", "GwlError", "lib", "LIB_PATH"]
