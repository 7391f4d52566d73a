"""MI355X-native multiscale spectral multigrid PCG for high-contrast Darcy flow.

The numerical work lives in libspecmg.so (HIP kernels for gfx950, C-ABI in
include/specmg.h); `specmg` is its ctypes binding.
"""
from .specmg import SpecMG, SpecMGError, load_library, FP64, FP32_VCYCLE  # noqa: F401
