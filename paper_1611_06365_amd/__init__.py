"""MI355X-native blocked LU factorization with partial pivoting (arXiv 1611.06365).

The product is libmlu.so (HIP kernels for gfx950 behind the C ABI in
include/mlu.h); `mlu` is its thin ctypes binding.
"""
from . import mlu  # noqa: F401
from .mlu import getrf, getrf_et, getrs, gesv_ir, gesv_gmres_ir, trsm, gemm_update, laswp, getf2_block, workspace  # noqa: F401
