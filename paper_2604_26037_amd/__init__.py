"""MI355X-native residual-based Chebyshev filter for the FE-PAW eigenproblem.

The compute lives in libpawfe.so (HIP kernels for gfx950 behind the C ABI
of include/pawfe.h); this package holds the build script and the ctypes
binding.
"""

from .pawfe import (  # noqa: F401
    Operator, Batch, PawfeError, load, band_energy_function, EXPORTS, LIB_PATH,
    FP64, FP32, BF16X3, tune_cache_load, tune_cache_save, tune_cache_clear, tune_cache_size,
)
